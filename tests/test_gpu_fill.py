"""GPU parity: model build (harp_fit) and Eq. (4) fill (harp_fill) against the
FP64 CPU oracle, on the same seeded inputs, through the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fill as ofill, fit as ofit, solve as osolve  # noqa: E402
from workloads import element, layout_disk, workload  # noqa: E402

from parity import block_eps, oracle_models, pack  # noqa: E402

pytestmark = pytest.mark.gpu

FILL_TOL = {"c64": 1e-5, "c128": 1e-12}


@pytest.fixture(scope="module")
def api():
    from paper_1702_03781_amd import api as A
    return A


def _gpu_fill(api, models_o, x, y, dtype, ri=0.0, dual=False, check_domain=True):
    mb = api.stack_models([pack(api, m) for m in models_o])
    xt = torch.from_numpy(np.asarray(x, np.float64)).cuda()
    yt = torch.from_numpy(np.asarray(y, np.float64)).cuda()
    Z, Z32, info = api.harp_fill(mb, xt, yt, dtype=dtype, ri=ri, dual=dual, check_domain=check_domain)
    torch.cuda.synchronize()
    return Z.cpu().numpy(), (Z32.cpu().numpy() if Z32 is not None else None), info.cpu().numpy()


@pytest.mark.parametrize("cfg,P_freq", [("small16", None), ("station_sweep", 15)])
def test_fit_matches_oracle(api, cfg, P_freq):
    wl = workload(cfg)
    i = 0 if P_freq is None else P_freq
    f, P = wl.freqs[i], wl.P[i]
    mo = ofit.fit(f, wl.elem.samples, P, wl.Q, wl.r_min, wire_radius=wl.elem.wire_radius)
    s = api.to_device_samples(wl.elem.samples)
    mg = api.harp_fit(s, wl.elem.wire_radius, f, P, wl.Q, wl.r_min)
    torch.cuda.synchronize()
    arr = api.model_arrays(mg)
    scale = np.abs(mo.C).max()
    assert np.abs(arr["C"] - mo.C).max() <= 1e-9 * scale
    assert np.abs(arr["Z_self"] - mo.Z_self).max() <= 1e-12 * np.abs(mo.Z_self).max()
    assert np.array_equal(arr["w"], mo.w)
    assert np.array_equal(arr["C32"], arr["C"].astype(np.complex64))
    h = arr["header"]
    assert (h["n_mbf"], h["P"], h["Q"]) == (wl.elem.n_mbf, P, wl.Q)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fill_small16(api, dtype):
    wl, models = oracle_models("small16")
    Zg, _, info = _gpu_fill(api, models, wl.x, wl.y, dtype)
    Zo = ofill.fill(models[0], wl.x, wl.y)
    eps, zero_ok, _ = block_eps(Zg[0], Zo, wl.elem.n_mbf)
    assert eps <= FILL_TOL[dtype], eps
    nm = wl.elem.n_mbf
    for a in range(wl.n_ant):
        blk = Zg[0][a * nm:(a + 1) * nm, a * nm:(a + 1) * nm]
        assert np.array_equal(blk, models[0].Z_self.astype(Zg.dtype))
    assert info[0] == 0
    # reciprocity of the GPU output
    sym = np.abs(Zg[0] - Zg[0].T).max() / np.abs(Zg[0]).max()
    assert sym <= (1e-13 if dtype == "c128" else 1e-6)


@pytest.mark.parametrize("mode", ["c64", "c128", "dual", "twin64"])
def test_fill_station_sweep_all_frequencies(api, mode):
    """Full station sweep (256 elements, 8 MBFs, 16 frequencies), every block.
    dual: complex128 plus its complex64 rounding; twin64: the complex64 fill
    written twice."""
    wl, models = oracle_models("station_sweep")
    dtype = "c64" if mode in ("c64", "twin64") else "c128"
    Zg, Z32, info = _gpu_fill(api, models, wl.x, wl.y, dtype, dual=mode in ("dual", "twin64"))
    assert (info == 0).all()
    for f, m in enumerate(models):
        Zo = ofill.fill(m, wl.x, wl.y)
        eps, _, glob = block_eps(Zg[f], Zo, wl.elem.n_mbf)
        assert eps <= FILL_TOL[dtype], (f, eps)
        if mode == "dual":
            # the complex64 copy is the rounding of the FP64 result
            assert np.array_equal(Z32[f], Zg[f].astype(np.complex64))
        if mode == "twin64":
            # the second copy holds the same complex64 values
            assert Z32.dtype == np.complex64 and np.array_equal(Z32[f], Zg[f])


def test_fill_ragged_and_radius_of_influence(api):
    """37 antennas (a ragged tile), 3 MBFs, Q = 4, and a radius of influence."""
    el = element(3, 9, seed=77)
    x, y = layout_disk(37, 9.0, 1.2, seed=78)
    P, Q = 5, 4
    mo = ofit.fit(130e6, el.samples, P, Q, 1.2, wire_radius=el.wire_radius)
    for ri in (0.0, 6.0):
        for dtype in ("c128", "c64"):
            Zg, _, info = _gpu_fill(api, [mo], x, y, dtype, ri=ri)
            Zo = ofill.fill(mo, x, y, ri=ri)
            eps, zero_ok, _ = block_eps(Zg[0], Zo, 3)
            assert eps <= FILL_TOL[dtype]
            assert zero_ok
            assert info[0] == 0


@pytest.mark.parametrize("n_mbf,n_ant", [(20, 23), (1, 40), (64, 5)])
def test_fill_lane_layouts(api, n_mbf, n_ant):
    """Element sizes that change the fill's lane layout: 20 MBFs (3 testing
    antennas per workgroup, 60 of 64 lanes), 1 MBF (16 antennas, 16 lanes),
    64 MBFs (one antenna per wave); ragged antenna counts, with and without a
    radius of influence, both precisions."""
    el = element(n_mbf, 6, seed=300 + n_mbf)
    x, y = layout_disk(n_ant, 1.2 * np.sqrt(n_ant) + 1.5, 1.2, seed=301 + n_mbf)
    P, Q = (2, 2) if n_mbf == 64 else (4, 3)
    mo = ofit.fit(120e6, el.samples, P, Q, 1.2, wire_radius=el.wire_radius)
    for ri in (0.0, 4.0):
        Zo = ofill.fill(mo, x, y, ri=ri)
        for dtype in ("c128", "c64"):
            Zg, _, info = _gpu_fill(api, [mo], x, y, dtype, ri=ri)
            eps, zero_ok, _ = block_eps(Zg[0], Zo, n_mbf)
            assert eps <= FILL_TOL[dtype], (dtype, ri, eps)
            assert zero_ok and info[0] == 0


@pytest.mark.parametrize("n_ant", [1, 2])
def test_fill_one_and_two_antennas(api, n_ant):
    """Degenerate layouts: one antenna (the self block only) and a single pair."""
    wl, models = oracle_models("small16")
    x, y = wl.x[:n_ant].copy(), wl.y[:n_ant].copy()
    Zo = ofill.fill(models[0], x, y)
    for dtype in ("c128", "c64"):
        Zg, _, info = _gpu_fill(api, models, x, y, dtype)
        assert info[0] == 0
        nm = models[0].n_mbf
        for a in range(n_ant):
            blk = slice(a * nm, (a + 1) * nm)
            assert np.array_equal(Zg[0][blk, blk], Zo[blk, blk].astype(Zg.dtype))
        if n_ant == 2:
            eps, zero_ok, _ = block_eps(Zg[0], Zo, nm)
            assert eps <= FILL_TOL[dtype] and zero_ok


def test_fill_rejects_oversized_coefficient_slab(api):
    """The coefficients of one source MBF (all testing MBFs, all p, q) must fit
    the 64 KB staging area: a synthetic blob of 64 MBFs with P = 8, Q = 6
    (64 x 17 x 7 complex128 = 122 KB) is refused before anything is enqueued."""
    nm, P, Q = 64, 8, 6
    C = np.zeros((nm, nm, 2 * P + 1, Q + 1), dtype=np.complex128)
    model = api.pack_model(C, np.eye(nm, dtype=np.complex128), np.ones(nm, dtype=np.complex128),
                           np.zeros((nm, 1, 8)), 1e8, 2.0, 1.0, 1.5, 0.02)
    mb = api.stack_models([model])
    xt = torch.zeros(2, dtype=torch.float64, device="cuda")
    xt[1] = 3.0
    from paper_1702_03781_amd._lib import HarpError
    with pytest.raises(HarpError):
        api.harp_fill(mb, xt, torch.zeros_like(xt), dtype="c128")


def test_fill_counts_pairs_below_rmin(api):
    wl, models = oracle_models("small16")
    x = wl.x.copy()
    y = wl.y.copy()
    x[5] = x[4] + 0.7          # one pair closer than r_min = 1.5 m
    y[5] = y[4]
    _, _, info = _gpu_fill(api, models, x, y, "c64", check_domain=False)
    assert info[0] == ofill.count_below_rmin(models[0], x, y) >= 2
    # the binding raises it by default
    with pytest.raises(api.HarpError) as e:
        _gpu_fill(api, models, x, y, "c64")
    assert e.value.status == api.HARP_E_DOMAIN


def test_fill_rejects_mismatched_model(api):
    wl, models = oracle_models("small16")
    mb = api.stack_models([pack(api, models[0])])
    mb.n_mbf = 3               # wrong element size for this blob
    xt = torch.from_numpy(wl.x[:10].copy()).cuda()
    yt = torch.from_numpy(wl.y[:10].copy()).cuda()
    _, _, info = api.harp_fill(mb, xt, yt, dtype="c64", check_domain=False)
    torch.cuda.synchronize()
    assert info.cpu().numpy()[0] == -1
    with pytest.raises(api.HarpError) as e:
        api.harp_fill(mb, xt, yt, dtype="c64")
    assert e.value.status == api.HARP_E_ARG


def test_ports_rhs_and_admittance(api):
    wl, models = oracle_models("small16")
    m = models[0]
    mb = api.stack_models([pack(api, m)])
    B = api.harp_port_rhs(mb, wl.n_ant)
    torch.cuda.synchronize()
    Bo = osolve.port_rhs(m.w, wl.n_ant)
    assert np.array_equal(B.cpu().numpy()[0], Bo)
    Zo = ofill.fill(m, wl.x, wl.y)
    Xo = osolve.solve(Zo, Bo)
    Xt = api.colmajor(1, Xo.shape[0], Xo.shape[1], torch.complex128, "cuda")
    Xt.copy_(torch.from_numpy(Xo)[None])
    Y = api.harp_port_admittance(mb, Xt)
    torch.cuda.synchronize()
    Yo = osolve.admittance(Xo, m.w, wl.n_ant)
    assert np.abs(Y.cpu().numpy()[0] - Yo).max() <= 1e-14 * np.abs(Yo).max()


def test_fill_exact_radius_of_influence_and_rmin(api):
    """Pairs exactly at r = RI and at r = r_min, on axis-aligned offsets whose
    distance both sides compute exactly (3-4-5 triangles and axis pairs, all
    coordinates dyadic): a block at r = RI is kept (the inclusive rule), a
    block one ulp beyond RI is zero, and a pair at exactly r = r_min is inside
    the model (no domain count)."""
    wl, models = oracle_models("small16")
    m = models[0]
    ri = 5.0
    # antenna 0 at the origin; 1 at (3, 4): r = 5 = RI exactly; 2 at
    # (-1.5, 0): r = r_min exactly; 3 at (0, 5 + 2^-48 * 8): just beyond RI
    x = np.array([0.0, 3.0, -1.5, 0.0, 40.0])
    y = np.array([0.0, 4.0, 0.0, np.nextafter(5.0, 6.0), 40.0])
    Z, _, info = _gpu_fill(api, [m], x, y, "c128", ri=ri)
    Z = Z[0]
    assert info[0] == 0
    Zo = ofill.fill(m, x, y, ri)
    nm = m.n_mbf
    blk = lambda M, a, b: M[a * nm:(a + 1) * nm, b * nm:(b + 1) * nm]   # noqa: E731
    for a, b in [(0, 1), (1, 0), (0, 2), (2, 0)]:
        assert np.abs(blk(Zo, a, b)).max() > 0
        assert np.linalg.norm(blk(Z, a, b) - blk(Zo, a, b)) <= 1e-12 * np.linalg.norm(blk(Zo, a, b))
    for a, b in [(0, 3), (3, 0), (0, 4), (4, 0)]:
        assert (blk(Z, a, b) == 0).all() and (blk(Zo, a, b) == 0).all()
    # complex64 evaluation takes the same keep / zero decisions (made in FP64)
    Z32, _, info32 = _gpu_fill(api, [m], x, y, "c64", ri=ri)
    Z32 = Z32[0]
    assert info32[0] == 0
    for a, b in [(0, 1), (1, 0), (0, 2), (2, 0)]:
        assert np.abs(blk(Z32, a, b)).max() > 0
    for a, b in [(0, 3), (3, 0), (0, 4), (4, 0)]:
        assert (blk(Z32, a, b) == 0).all()


def test_fitted_models_are_reciprocal(api):
    """The GPU-built model of every frequency of the station sweep gives a
    complex-symmetric reduced matrix (reciprocity, Z = Z^T) to rounding: the
    fit's even angular grid makes C^{ST}_p = (-1)^p C^{TS}_p, which the
    adjoint's solve with Z instead of Z^T relies on."""
    wl = workload("station_sweep", n_freq=4)
    s = api.to_device_samples(wl.elem.samples)
    mb = api.stack_models([api.harp_fit(s, wl.elem.wire_radius, f, P, wl.Q, wl.r_min)
                           for f, P in zip(wl.freqs, wl.P)])
    xt = torch.from_numpy(wl.x).cuda()
    yt = torch.from_numpy(wl.y).cuda()
    Z, _, _ = api.harp_fill(mb, xt, yt, dtype="c128")
    for f in range(mb.n_freq):
        Zf = Z[f]
        asym = (torch.linalg.norm(Zf - Zf.transpose(0, 1)) / torch.linalg.norm(Zf)).item()
        assert asym <= 1e-13, (f, asym)
    # an odd angular grid is refused by the library
    with pytest.raises(api.HarpError):
        api.harp_fit(s, wl.elem.wire_radius, wl.freqs[0], wl.P[0], wl.Q, wl.r_min, n_alpha=4 * (wl.P[0] + 1) + 1)
