"""GPU parity of the batch of unequal layouts (grouping plan, padded fill,
per-system ports, complex64 LU with FP64 refinement) through the C ABI.

Small batch: six layouts of 5..37 elements (ragged, padded to multiples of
8 antennas, at most two systems per group so several groups are formed), each
at one or two of three frequencies, on one and on two streams -- every system
against the FP64 oracle (fill per block, X and Y against LAPACK), the padding
exactly the identity / zero.
Batched layouts: 48 station layouts of 64..512 elements, 8 of the 16 sweep
frequencies each (384 systems, n = 528..4056), as timed (one HIP graph over
four streams) -- every system by recomputed residual, reciprocity and exact
padding, and every system's fill, X (per port) and Y against the oracle
(in eight chunks of 48 systems, each its own test).
Graph replays: the captured step replayed several times, with eager work and
synchronisations between, equals the eager step bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fill as ofill, fit as ofit, solve as osolve  # noqa: E402
from workloads import batched_layouts, element, layout_disk  # noqa: E402

from parity import block_eps, oracle_fill_threads, oracle_models, pack  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1702_03781_amd import api as A
    return A


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _port_rel(a, b):
    return float((np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max())


@pytest.fixture(scope="module")
def small(api):
    el = element(4, 32, seed=201)
    freqs = [100e6, 130e6, 170e6]
    models = [ofit.fit(f, el.samples, 7, 6, 1.5, wire_radius=el.wire_radius) for f in freqs]
    layouts = []
    for i, na in enumerate([5, 9, 16, 23, 37, 12]):
        x, y = layout_disk(na, 1.5 + 1.2 * np.sqrt(na), 1.5, seed=500 + i)
        layouts.append((x, y, [i % 3] if i % 2 else [0, 2]))
    mb = api.stack_models([pack(api, m) for m in models])
    return models, layouts, mb


# fill precision -> (fill bar against the oracle, stored type of the self blocks)
FILLS = {"c128": (1e-12, np.complex128), "c64": (1e-5, np.complex64)}


@pytest.mark.parametrize("streams,fill", [(1, "c128"), (2, "c128"), (2, "c64")])
def test_batched_small_matches_oracle(api, small, streams, fill):
    models, layouts, mb = small
    fill_tol, zdt = FILLS[fill]
    S = api.BatchSolver(mb, layouts, tol=1e-10, streams=streams, max_batch=2, fill=fill)
    S.step()
    torch.cuda.synchronize()
    assert len(S.groups) >= 3
    s = 0
    for x, y, fidx in layouts:
        for f in fidx:
            m = models[f]
            na, n = x.size, x.size * m.n_mbf
            X, Y, info, finfo = S.system(s)
            assert int(info) == 0 and int(finfo) == 0, s
            assert S.reports[s]["converged"], S.reports[s]
            Zp, Xp, Yp = (t.cpu().numpy() for t in S.padded(s))
            N = Zp.shape[0]
            Zo = ofill.fill(m, x, y)
            assert Zp.dtype == zdt
            eps, zero_ok, _ = block_eps(Zp[:n, :n], Zo, m.n_mbf)
            assert eps <= fill_tol and zero_ok, (s, eps)
            for a in range(na):
                blk = slice(a * m.n_mbf, (a + 1) * m.n_mbf)
                assert np.array_equal(Zp[blk, blk], m.Z_self.astype(zdt))
            assert (Zp[n:, :n] == 0).all() and (Zp[:n, n:] == 0).all()
            assert np.array_equal(Zp[n:, n:], np.eye(N - n))
            Bo = osolve.port_rhs(m.w, na)
            Xo = osolve.solve(Zo, Bo)
            Yo = osolve.admittance(Xo, m.w, na)
            assert _port_rel(X.cpu().numpy(), Xo) <= 1e-6
            assert _rel(Y.cpu().numpy(), Yo) <= 1e-6
            assert (Xp[n:, :] == 0).all() and (Xp[:, na:] == 0).all()
            assert (Yp[na:, :] == 0).all() and (Yp[:, na:] == 0).all()
            s += 1
    # the complex64 copy written beside the fill is its rounding (c128) or the
    # same values (c64); the solver's own copy holds the LU factors by now
    g = S.groups[-1]
    Zf, Z32, info = api.harp_fill_systems(mb, S.x, S.y, g.sys, g.n_pad, dtype=fill, dual=True)
    torch.cuda.synchronize()
    assert not info.any() and torch.equal(Zf, g.Zres) and torch.equal(Z32, Zf.to(torch.complex64))


def test_bad_descriptor_is_reported(api, small):
    models, layouts, mb = small
    x = torch.from_numpy(layouts[0][0]).cuda()
    y = torch.from_numpy(layouts[0][1]).cuda()
    na = x.numel()
    sys = api.systems_tensor([0, 5, 1, 0], [na, na, na + 1, na], [0, 0, 0, 1], "cuda")
    _, _, info = api.harp_fill_systems(mb, x, y, sys, na + 1, dtype="c128", check_domain=False)
    torch.cuda.synchronize()
    # model 5 out of range; positions [0, na+1) and [1, na+1) beyond the array
    assert info.cpu().tolist() == [0, -2, -2, -2]
    with pytest.raises(api.HarpError) as e:
        api.harp_fill_systems(mb, x, y, sys, na + 1, dtype="c128")
    assert e.value.status == api.HARP_E_ARG


@pytest.fixture(scope="module", params=["c64", "c128"])
def batched(api, request):
    """The benchmark's batch (one HIP graph over four streams) with each fill
    precision."""
    wl, models = oracle_models("station_sweep")
    mb = api.stack_models([pack(api, m) for m in models])
    layouts = batched_layouts()
    S = api.BatchSolver(mb, layouts, tol=1e-10, streams=4, graph=True, fill=request.param)
    S.step()
    torch.cuda.synchronize()
    yield models, layouts, S
    del S
    torch.cuda.empty_cache()


def test_batched_layouts_every_system(api, batched):
    models, layouts, S = batched
    assert S.n_systems == 384
    for s in range(S.n_systems):
        X, Y, info, finfo = S.system(s)
        rep = S.reports[s]
        assert int(info) == 0 and int(finfo) == 0, s
        assert rep["converged"] and rep["iters"] <= 3, (s, rep)
        na = Y.shape[0]
        n = X.shape[0]
        Zp, Xp, Yp = S.padded(s)
        gi, k = S.where[s]
        B = S.groups[gi].B[k, :n, :na]
        Z = Zp[:n, :n].to(torch.complex128)   # the residual's matrix, widened as the refinement reads it
        R = B - Z @ X
        rel = (torch.linalg.norm(R) / (torch.linalg.norm(Z) * torch.linalg.norm(X))).item()
        assert rel <= 1.001e-10, (s, rel)
        assert torch.linalg.norm(Y - Y.T).item() <= 1e-8 * torch.linalg.norm(Y).item()
        assert not Xp[n:].any() and not Xp[:, na:].any()
        assert not Yp[na:].any() and not Yp[:, na:].any()


@pytest.mark.parametrize("chunk", range(8))
def test_batched_layouts_against_oracle(api, batched, chunk):
    """Systems [48 chunk, 48 chunk + 48): the oracle's fill of each (its own
    FP64 Eq. 4 evaluation) against the GPU's block by block, and the GPU's
    refined X (every port) and Y against LAPACK on the oracle's matrix."""
    models, layouts, S = batched
    worst = 0.0
    for s in range(48 * chunk, 48 * chunk + 48):
        li, f = S.layout_of[s]
        x, y, _ = layouts[li]
        m = models[f]
        na, n = x.size, x.size * m.n_mbf
        X, Y, _, _ = S.system(s)
        Zo = oracle_fill_threads(m, x, y)
        Zp = S.padded(s)[0][:n, :n].cpu().numpy()
        fill_tol, zdt = FILLS["c64" if S.fill32 else "c128"]
        eps, zero_ok, _ = block_eps(Zp, Zo, m.n_mbf)
        assert eps <= fill_tol and zero_ok, (s, eps)
        for a in range(0, na, max(1, na // 7)):
            assert np.array_equal(Zp[a * m.n_mbf:(a + 1) * m.n_mbf, a * m.n_mbf:(a + 1) * m.n_mbf],
                                  m.Z_self.astype(zdt))
        del Zp
        Xo = osolve.solve(Zo, osolve.port_rhs(m.w, na))
        Yo = osolve.admittance(Xo, m.w, na)
        ex, ey = _port_rel(X.cpu().numpy(), Xo), _rel(Y.cpu().numpy(), Yo)
        assert ex <= 1e-6 and ey <= 1e-6, (s, ex, ey)
        worst = max(worst, ex, ey)
    print(f"chunk {chunk}: worst relative error {worst:.2e}")


def test_batched_graph_replays_equal_eager(api, small):
    """The captured step replayed three times, with the program's own eager
    work and synchronisations between the replays, gives every system's X,
    Y and report exactly as the eager step (one and two streams)."""
    models, layouts, mb = small
    E = api.BatchSolver(mb, layouts, tol=1e-10, max_batch=2)
    E.step()
    torch.cuda.synchronize()
    ref = [(E.system(s)[0].clone(), E.system(s)[1].clone()) for s in range(E.n_systems)]
    for streams in (1, 2):
        G = api.BatchSolver(mb, layouts, tol=1e-10, max_batch=2, streams=streams, graph=True)
        for rep in range(3):
            for g in G.groups:           # stale values that a replay must overwrite
                g.X.fill_(float("nan"))
                g.Y.fill_(float("nan"))
                g.rep_dev.zero_()
            torch.cuda.synchronize()
            G.step()
            torch.cuda.synchronize()
            for s in range(G.n_systems):
                X, Y, info, finfo = G.system(s)
                assert torch.equal(X, ref[s][0]) and torch.equal(Y, ref[s][1]), (streams, rep, s)
                assert int(info) == 0 and int(finfo) == 0
                assert G.reports[s]["converged"] and G.reports[s]["iters"] == E.reports[s]["iters"]
            # eager work between replays
            _ = (torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")).sum().item()


def test_autotuned_costs(api, small):
    """The autotuner's fitted cost model reproduces its own measurements to a
    factor of two and yields a valid plan; the batch solved under that plan
    gives the same systems as under the default plan."""
    models, layouts, mb = small
    cost, pts = api.autotune_batch_costs(mb, sizes=(8, 24, 40), counts=(1, 4), reps=2)
    assert len(cost) == 3 and all(c >= 0.0 for c in cost) and len(pts) == 6
    for p in pts:
        pred = cost[0] + cost[1] * p["order"] + cost[2] * p["systems"] * p["order"] ** 3
        assert 0.5 * p["seconds"] <= pred <= 2.0 * p["seconds"], (p, pred)
    A = api.BatchSolver(mb, layouts, tol=1e-10)
    B = api.BatchSolver(mb, layouts, tol=1e-10, cost=cost)
    A.step()
    B.step()
    torch.cuda.synchronize()
    for s in range(A.n_systems):
        xa, ya, _, _ = A.system(s)
        xb, yb, _, _ = B.system(s)
        assert torch.linalg.norm(xa - xb) <= 1e-9 * torch.linalg.norm(xa)
        assert torch.linalg.norm(ya - yb) <= 1e-9 * torch.linalg.norm(ya)


def test_kernel_autotuner(api, small):
    """The kernel autotuner picks a feasible panel width and GEMM tile switch
    for every group order of the plan (timed on this GPU); the batch solved
    under that table equals the batch under the built-in choices to 1e-9 (the
    choices change the order of operations, not the method)."""
    models, layouts, mb = small
    A = api.BatchSolver(mb, layouts, tol=1e-10, max_batch=2)
    groups = [(g.n, len(g.members), g.n_ports_pad) for g in A.groups]
    entries, points = api.autotune_kernels(groups, reps=1)
    assert [e["max_order"] for e in entries] == sorted({g[0] for g in groups})
    assert all(e["panel_width_c64"] in (4, 8, 16) and e["small_grid_wgs"] in (256, 1024, 4096) for e in entries)
    assert len(points) >= len(entries) and api.get_tuning() == []
    B = api.BatchSolver(mb, layouts, tol=1e-10, max_batch=2, tuning=entries)
    try:
        A.step()
        B.step()
        torch.cuda.synchronize()
        assert api.get_tuning() == entries
        for s in range(A.n_systems):
            xa, ya, _, _ = A.system(s)
            xb, yb, _, _ = B.system(s)
            assert torch.linalg.norm(xa - xb) <= 1e-9 * torch.linalg.norm(xa)
            assert torch.linalg.norm(ya - yb) <= 1e-9 * torch.linalg.norm(ya)
    finally:
        api.set_tuning(None)
