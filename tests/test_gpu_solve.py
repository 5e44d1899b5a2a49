"""GPU parity of the dense reduced solve: the MFMA complex GEMM, the blocked LU
with partial pivoting, the triangular solves and the FP64 refinement, through
the C ABI, against numpy/LAPACK and the FP64 CPU oracle."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fill as ofill, solve as osolve  # noqa: E402

from parity import oracle_models, pack  # noqa: E402

pytestmark = pytest.mark.gpu

REL_SOLVE = 1e-6      # refined complex64 path vs the FP64 oracle
REL_PLAIN = 1e-10     # complex128 path vs the FP64 oracle


@pytest.fixture(scope="module")
def api():
    from paper_1702_03781_amd import api as A
    return A


def _rand(shape, seed, dtype=np.complex128):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


def _to_cm(api, M, dtype):
    """numpy (b, r, c) -> batched column-major CUDA tensor."""
    b, r, c = M.shape
    T = api.colmajor(b, r, c, dtype, "cuda")
    T.copy_(torch.from_numpy(M))
    return T


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("shape", [(64, 128, 16), (70, 33, 21), (130, 200, 64), (1, 1, 1), (40, 17, 0)])
def test_cgemm_hook(api, dt, shape):
    from paper_1702_03781_amd._lib import lib
    M, N, K = shape
    batch = 3
    npdt = np.complex64 if dt == "c64" else np.complex128
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    A = _rand((batch, M, K), 1, npdt)
    B = _rand((batch, K, N), 2, npdt)
    C = _rand((batch, M, N), 3, npdt)
    At, Bt, Ct = _to_cm(api, A, tdt), _to_cm(api, B, tdt), _to_cm(api, C, tdt)
    Dt = api.colmajor(batch, M, N, tdt, "cuda")
    for alpha, beta in [(-1.0, 1.0), (1.0, 0.0)]:
        st = lib().harp_debug_cgemm(0 if dt == "c64" else 1, M, N, K, batch, alpha,
                                    At.data_ptr(), M, M * K, Bt.data_ptr(), max(K, 1), K * N,
                                    beta, Ct.data_ptr(), M, M * N, Dt.data_ptr(), M, M * N,
                                    torch.cuda.current_stream().cuda_stream)
        assert st == 0
        torch.cuda.synchronize()
        ref = beta * C.astype(np.complex128) + alpha * (A.astype(np.complex128) @ B.astype(np.complex128))
        got = Dt.cpu().numpy()
        scale = np.abs(ref).max() + 1e-30
        tol = 1e-5 if dt == "c64" else 1e-13
        assert np.abs(got - ref).max() <= tol * scale * max(1, np.sqrt(K))


@pytest.mark.parametrize("dt,n,batch", [("c128", 70, 2), ("c128", 300, 3), ("c64", 111, 2),
                                        ("c64", 257, 3), ("c128", 64, 1), ("c64", 1, 2),
                                        ("c64", 700, 2), ("c128", 513, 2)])
def test_factor_and_solve_random(api, dt, n, batch):
    """Diagonally weighted random systems (ragged block sizes): solve vs LAPACK;
    the complex64 factors with FP64 refinement reach the FP64 solution."""
    A = _rand((batch, n, n), 10 + n) + 4 * np.sqrt(n) * np.eye(n)[None]
    Bh = _rand((batch, n, 5), 20 + n)
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    LU = _to_cm(api, A.astype(np.complex64 if dt == "c64" else np.complex128), tdt)
    F = api.reduced_factor(LU)
    info = F.info
    B = _to_cm(api, Bh, torch.complex128)
    X, _ = api.reduced_solve(F, B)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    ref = np.linalg.solve(A, Bh)
    err = np.linalg.norm(X.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= (1e-5 if dt == "c64" else 1e-12), err
    if dt == "c64":
        Z64 = _to_cm(api, A, torch.complex128)
        X2, rep = api.reduced_solve(F, B, Z64=Z64, tol=1e-13, max_iter=10)
        torch.cuda.synchronize()
        err2 = np.linalg.norm(X2.cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err2 <= 1e-11, (err2, rep)
        assert all(r["converged"] for r in rep)


@pytest.mark.parametrize("n,batch,nrhs", [(37, 2, 5), (70, 3, 33), (129, 2, 7), (1100, 2, 19)])
def test_refinement_against_a_complex64_matrix(api, n, batch, nrhs):
    """FP64 refinement whose residual reads the complex64 matrix itself
    (widened on load; odd orders and ragged K chunks take the guarded loads):
    the result is the FP64 solution of that complex64 matrix, and its FP64
    residual against it, recomputed on the host, is at the tolerance (plus
    the host product's own rounding)."""
    A = (_rand((batch, n, n), 30 + n) + 4 * np.sqrt(n) * np.eye(n)[None]).astype(np.complex64)
    Bh = _rand((batch, n, nrhs), 40 + n)
    Z32 = _to_cm(api, A, torch.complex64)
    F = api.reduced_factor(_to_cm(api, A, torch.complex64))
    B = _to_cm(api, Bh, torch.complex128)
    X, rep = api.reduced_solve(F, B, Z64=Z32, tol=1e-13, max_iter=10)
    torch.cuda.synchronize()
    assert all(r["converged"] for r in rep), rep
    A64 = A.astype(np.complex128)
    ref = np.linalg.solve(A64, Bh)
    Xh = X.cpu().numpy()
    assert np.linalg.norm(Xh - ref) <= 1e-11 * np.linalg.norm(ref)
    for b in range(batch):
        R = Bh[b] - A64[b] @ Xh[b]
        assert np.linalg.norm(R) <= 5e-13 * np.linalg.norm(A64[b]) * np.linalg.norm(Xh[b])


def _sparse_rhs(perm, nrhs, seed):
    """Right-hand sides placed by their rows' positions in P B (perm: row i of
    P B is row perm[i] of B): columns 0-31 are non-zero only at positions in
    the last, ragged group, columns 32-63 only in the second group (whole
    32-column tiles that start late), column 64 is zero, column 65 has 24
    entries anywhere, the rest one entry each at an early position."""
    n = perm.size
    rng = np.random.default_rng(seed)
    B = np.zeros((n, nrhs), np.complex128)
    groups = [(1024, n)] * 32 + [(256, 512)] * 32 + [None, (0, n)]
    for c in range(nrhs):
        span = groups[c] if c < len(groups) else (c, c + 1)
        if span is None:
            continue
        lo, hi = span
        pos = np.arange(lo, hi) if hi - lo < 8 else rng.choice(np.arange(lo, hi), size=min(hi - lo, 24), replace=False)
        B[perm[pos], c] = rng.standard_normal(pos.size) + 1j * rng.standard_normal(pos.size)
    return B


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sparse_right_hand_sides_with_row_exchanges(api, dtype):
    """The first forward substitution leaves out the products of right-hand
    sides that are still exactly zero in a group's rows (whole 32-column
    tiles).  A general matrix, whose pivots move rows between the 256-row
    groups, at a ragged order, with right-hand-side tiles placed by LAPACK's
    row order to start in the last or the second group: every column agrees
    with LAPACK, and the zero column's solution is exactly zero."""
    import scipy.linalg
    n, batch, nrhs = 1100, 2, 70
    A = _rand((batch, n, n), 61)
    Bh = np.empty((batch, n, nrhs), np.complex128)
    for b in range(batch):
        _, piv = scipy.linalg.lu_factor(A[b])
        perm = np.arange(n)
        for i, p in enumerate(piv):
            perm[i], perm[p] = perm[p], perm[i]
        assert np.abs(perm // 256 - np.arange(n) // 256).max() >= 2   # rows cross groups
        Bh[b] = _sparse_rhs(perm, nrhs, 70 + b)
    B = _to_cm(api, Bh, torch.complex128)
    if dtype == "c128":
        F = api.reduced_factor(_to_cm(api, A, torch.complex128))
        X, _ = api.reduced_solve(F, B)
        A_ref, tol = A, 1e-9
    else:
        A32 = A.astype(np.complex64)
        F = api.reduced_factor(_to_cm(api, A32, torch.complex64))
        X, rep = api.reduced_solve(F, B, Z64=_to_cm(api, A32, torch.complex64), tol=1e-13, max_iter=10)
        assert all(r["converged"] for r in rep), rep
        # forward error up to cond (1.4e3-4.0e3 here) x the 1e-13 residual; a
        # skipped product that was not zero would leave O(1) errors
        A_ref, tol = A32.astype(np.complex128), 1e-8
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    for b in range(batch):
        ref = np.linalg.solve(A_ref[b], Bh[b])
        for c in range(nrhs):
            if c == 64:
                assert not np.any(Xh[b][:, c]), "zero right-hand side"
                continue
            err = np.linalg.norm(Xh[b][:, c] - ref[:, c]) / np.linalg.norm(ref[:, c])
            assert err <= tol, (b, c, err)


@pytest.mark.parametrize("n", [3000, 5000])
def test_tall_complex64_panels_pivot_and_solve(api, n):
    """Complex64 panels taller than 2048 rows keep two register blocks (16
    columns at 4 rows per thread up to 4096 rows, 8 at 8 rows per thread
    above), the first block re-read from memory for the second's update.  A
    row-permuted, strongly diagonally dominant matrix makes partial pivoting
    unambiguous in any precision: the pivots must undo the permutation
    exactly, and the complex64 solve agrees with LAPACK."""
    rng = np.random.default_rng(700 + n)
    D = 0.1 * _rand((n, n), 701 + n) + 10.0 * n * np.exp(1j * rng.uniform(0, 2 * np.pi, n)) * np.eye(n)
    p0 = rng.permutation(n)
    A = D[p0][None].astype(np.complex64)             # row i of A is row p0[i] of D
    F = api.reduced_factor(_to_cm(api, A, torch.complex64))
    Bh = _rand((1, n, 7), 702 + n)
    X, _ = api.reduced_solve(F, _to_cm(api, Bh, torch.complex128))
    torch.cuda.synchronize()
    perm = np.arange(n)
    for i, q in enumerate(F.ipiv.cpu().numpy()[0]):
        perm[i], perm[q] = perm[q], perm[i]
    assert np.array_equal(p0[perm], np.arange(n))   # position j holds D's row j
    ref = np.linalg.solve(A[0].astype(np.complex128), Bh[0])
    assert np.linalg.norm(X.cpu().numpy()[0] - ref) <= 1e-5 * np.linalg.norm(ref)


def test_pivots_follow_partial_pivoting(api):
    """Generic matrix: the pivot sequence is LAPACK's (first max |Re|+|Im|)."""
    import scipy.linalg
    n = 200
    A = _rand((1, n, n), 5)
    LU = _to_cm(api, A, torch.complex128)
    ipiv, info = api.reduced_factor(LU)
    torch.cuda.synchronize()
    _, piv = scipy.linalg.lu_factor(A[0])
    assert np.array_equal(ipiv.cpu().numpy()[0], piv)
    # U (upper triangle) agrees with LAPACK's
    U = np.triu(LU.cpu().numpy()[0])
    lu_ref, _ = scipy.linalg.lu_factor(A[0])
    assert np.abs(U - np.triu(lu_ref)).max() <= 1e-11 * np.abs(lu_ref).max()


def test_complex64_pivot_ties_take_the_smallest_row(api):
    """Single precision, n = 2048 (one panel row per 1024-thread workgroup
    thread and a second one 1024 rows further): exact ties of the largest
    |Re| + |Im| in column 0 within one thread, within one wave, across waves
    and over the whole column go to the smallest row (LAPACK's first maximum);
    a zero or NaN column is a zero pivot on the diagonal row.  The
    factors of the nonsingular ones solve the system (refined to FP64)."""
    n = 2048
    rng = np.random.default_rng(31)
    A = 0.25 * (rng.standard_normal((6, n, n)) + 1j * rng.standard_normal((6, n, n)))
    A[:, :, 0] *= 0.1                                  # column 0 below the ties' magnitude
    A[0, [1724, 700], 0] = [3.0, -3.0j]                # rows 700 and 700 + 1024: same thread
    A[1, [703, 1725, 701], 0] = [1.5 + 1.5j, -3.0, 3.0j]   # one wave, three rows
    A[2, [2000, 1500, 900], 0] = [3.0, 2.0 - 1.0j, -1.0 + 2.0j]   # three waves
    A[3, :, 0] = rng.choice([1, -1], n) + 1j * rng.choice([1, -1], n)   # the whole column ties
    A[4, :, 0] = 0.0
    A[5, :, 0] = np.nan
    A = A.astype(np.complex64)
    LU = _to_cm(api, A, torch.complex64)
    F = api.reduced_factor(LU, check_singular=False)
    torch.cuda.synchronize()
    piv = F.ipiv.cpu().numpy()
    assert list(piv[:, 0]) == [700, 701, 900, 0, 0, 0], piv[:, 0]
    assert list(F.info.cpu().numpy()) == [0, 0, 0, 0, 1, 1]
    assert ((piv >= np.arange(n)[None]) & (piv < n)).all()
    # each pivot has the largest |Re| + |Im| of its column at its step, so
    # every multiplier has modulus at most sqrt(2)
    L = np.tril(LU.cpu().numpy()[:4], -1)
    assert np.abs(L).max() <= np.sqrt(2.0) * (1 + 1e-5)
    Bh = _rand((6, n, 3), 32)
    A64 = A.astype(np.complex128)
    X, rep = api.reduced_solve(F, _to_cm(api, Bh, torch.complex128), Z64=_to_cm(api, A64, torch.complex128),
                               tol=1e-12, max_iter=10, raise_noconv=False)
    torch.cuda.synchronize()
    assert all(r["converged"] for r in rep[:4]), rep
    ref = np.linalg.solve(A64[:4], Bh[:4])
    err = np.linalg.norm(X.cpu().numpy()[:4] - ref) / np.linalg.norm(ref)
    assert err <= 1e-9, err


def test_exact_zero_pivot_sets_info(api):
    n = 100
    A = _rand((2, n, n), 7)
    A[1, :, 37] = 0.0                 # exactly singular: zero column 37
    LU = _to_cm(api, A, torch.complex128)
    ipiv, info = api.reduced_factor(LU, check_singular=False)
    torch.cuda.synchronize()
    assert list(info.cpu().numpy()) == [0, 38]
    # the binding raises it by default
    with pytest.raises(api.HarpError) as e:
        api.reduced_factor(_to_cm(api, A, torch.complex128))
    assert e.value.status == api.HARP_E_SINGULAR


def test_station_solver_raises_domain_and_singular(api):
    """The solver classes read the fill's domain counts and the zero pivots
    after their step: a pair closer than r_min raises HARP_E_DOMAIN; an
    element with an all-zero MBF (zero rows and columns in Z) raises
    HARP_E_SINGULAR."""
    wl, models = oracle_models("small16")
    m = models[0]
    mb = api.stack_models([pack(api, m)])
    x, y = wl.x.copy(), wl.y.copy()
    x[5], y[5] = x[4] + 0.7, y[4]
    S = api.StationSolver(mb, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), "refined")
    with pytest.raises(api.HarpError) as e:
        S.step()
    assert e.value.status == api.HARP_E_DOMAIN
    C, Zs, w = m.C.copy(), m.Z_self.copy(), m.w.copy()
    C[1, :], C[:, 1], Zs[1, :], Zs[:, 1] = 0, 0, 0, 0    # MBF 1 interacts with nothing
    mz = api.pack_model(C, Zs, w, m.samples, m.freq, m.k, 1.0, m.r_min, m.wire_radius)
    for mode in ("refined", "plain"):
        S = api.StationSolver(api.stack_models([mz]), torch.from_numpy(wl.x).cuda(),
                              torch.from_numpy(wl.y).cuda(), mode)
        with pytest.raises(api.HarpError) as e:
            S.step()
        assert e.value.status == api.HARP_E_SINGULAR, mode


def test_refinement_report_and_noconv(api):
    n = 96
    A = _rand((1, n, n), 8) + 3 * np.sqrt(n) * np.eye(n)[None]
    LU = _to_cm(api, A.astype(np.complex64), torch.complex64)
    F = api.reduced_factor(LU)
    B = _to_cm(api, _rand((1, n, 4), 9), torch.complex128)
    Z64 = _to_cm(api, A, torch.complex128)
    from paper_1702_03781_amd._lib import HarpError
    with pytest.raises(HarpError) as e:
        api.reduced_solve(F, B, Z64=Z64, tol=1e-300, max_iter=0)
    assert e.value.status == -4
    X, rep = api.reduced_solve(F, B, Z64=Z64, tol=1e-300, max_iter=0, raise_noconv=False)
    assert rep[0]["iters"] == 0 and not rep[0]["converged"]
    X, rep = api.reduced_solve(F, B, Z64=Z64, tol=1e-12, max_iter=5)
    assert rep[0]["converged"] and 1 <= rep[0]["iters"] <= 5 and rep[0]["resid_rel"] <= 1e-12


@pytest.mark.parametrize("zdt", ["c128", "c64"])
@pytest.mark.parametrize("max_iter", [0, 1, 4])
def test_refinement_device_control_matches_host(api, max_iter, zdt):
    """The refinement without a host report (nothing synchronises; every
    sweep of the budget is enqueued and converged systems skip it) gives the
    same solution and the same per-system report as with one, bit for bit,
    over a batch whose systems need different numbers of corrections (one
    system never converges within the budget); against a complex128 matrix
    and against a complex64 one (whose first check after a correction is the
    complex64 residual update)."""
    n = 130
    A = _rand((3, n, n), 18) + np.array([3.0, 0.5, 3.0])[:, None, None] * np.sqrt(n) * np.eye(n)[None]
    if zdt == "c64":
        A = A.astype(np.complex64).astype(np.complex128)
    Z64 = _to_cm(api, A, torch.complex128) if zdt == "c128" else _to_cm(api, A.astype(np.complex64), torch.complex64)
    F = api.reduced_factor(_to_cm(api, A.astype(np.complex64), torch.complex64))
    B = _to_cm(api, _rand((3, n, 5), 19), torch.complex128)
    tols = 1e-13
    Xh, rh = api.reduced_solve(F, B, Z64=Z64, tol=tols, max_iter=max_iter, raise_noconv=False)
    Xd, rd_dev = api.reduced_solve(F, B, Z64=Z64, tol=tols, max_iter=max_iter, device_report=True)
    torch.cuda.synchronize()
    rd = api.read_reports(rd_dev)
    assert rd == rh, (rd, rh)
    assert torch.equal(Xh, Xd)
    for r in rh:
        assert r["iters"] <= max_iter
    if max_iter >= 4:
        assert all(r["converged"] for r in rh)
        ref = np.linalg.solve(A, B.cpu().numpy())
        assert np.linalg.norm(Xd.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,nrhs", [(300, 9), (1100, 19), (2048, 64)])
def test_updated_residual_within_its_bound(api, n, nrhs):
    """Against a complex64 matrix, the check after the first correction
    updates the residual, R1 = R0 - Z D, with complex64 products summed over
    K slices in FP64, and accepts only when |R1| plus its error bound meets
    the tolerance.  The correction D is X1 - X0 (max_iter 0 and 1 give X0 and
    X1; the kernels are deterministic), so the host can recompute the true
    FP64 residual of X1 and the bound sqrt(2) gamma_{2 Ks + 2} |Z| |D| (Ks the
    slice length, at most 256 here): the reported residual is within the
    bound of the true one, and the true one within the tolerance."""
    # well conditioned (diagonal 8 sqrt(n) against a spectral radius of about
    # sqrt(2 n)), so that one correction is small enough to be certified by
    # the update (a poorly conditioned system would take a second, FP64 check)
    A = (_rand((1, n, n), 90 + n) + 8 * np.sqrt(n) * np.eye(n)[None]).astype(np.complex64)
    Bh = _rand((1, n, nrhs), 91 + n)
    Zc = _to_cm(api, A, torch.complex64)
    F = api.reduced_factor(_to_cm(api, A, torch.complex64))
    B = _to_cm(api, Bh, torch.complex128)
    X0, r0 = api.reduced_solve(F, B, Z64=Zc, tol=0.0, max_iter=0, raise_noconv=False)
    X1, r1 = api.reduced_solve(F, B, Z64=Zc, tol=1e-10, max_iter=1)
    torch.cuda.synchronize()
    assert r1[0]["iters"] == 1 and r1[0]["converged"], r1
    A64 = A[0].astype(np.complex128)
    x0, x1 = X0.cpu().numpy()[0], X1.cpu().numpy()[0]
    d = x1 - x0
    zn, xn = np.linalg.norm(A64), np.linalg.norm(x1)
    true = np.linalg.norm(Bh[0] - A64 @ x1)
    reported = r1[0]["resid_rel"] * zn * xn
    n_sl = min(16, max(1, (n + 255) // 256))
    ks = ((n + n_sl - 1) // n_sl + 15) // 16 * 16
    m = 2 * ks + 2
    bound = 1.01 * np.sqrt(2) * m * 2.0**-24 / (1 - m * 2.0**-24) * zn * np.linalg.norm(d) + 2.0**-53 * zn * xn
    # the host's own FP64 product rounds too: a margin of n u64 |Z| |X|
    slack = n * 2.0**-53 * zn * xn
    assert abs(reported - true) <= bound + slack, (reported, true, bound)
    assert true <= 1e-10 * zn * xn


def _pipeline(api, models_o, x, y, refined=True, keep_z=False):
    """refined: True (FP64 fill, complex64 LU, FP64 refinement against the
    complex128 matrix), "refined32" (complex64 fill written twice, FP64
    refinement against one copy) or False (complex128 throughout)."""
    mb = api.stack_models([pack(api, m) for m in models_o])
    xt = torch.from_numpy(np.asarray(x, np.float64)).cuda()
    yt = torch.from_numpy(np.asarray(y, np.float64)).cuda()
    n_ant = len(x)
    B = api.harp_port_rhs(mb, n_ant)
    Zres = None
    if refined == "refined32":
        Zr, Z32, info = api.harp_fill(mb, xt, yt, dtype="c64", dual=True)
        F = api.reduced_factor(Z32)
        finfo = F.info
        X, rep = api.reduced_solve(F, B, Z64=Zr, tol=1e-10, max_iter=10)
        Zres = Zr
    elif refined:
        Z64, Z32, info = api.harp_fill(mb, xt, yt, dtype="c128", dual=True)
        F = api.reduced_factor(Z32)
        finfo = F.info
        X, rep = api.reduced_solve(F, B, Z64=Z64, tol=1e-10, max_iter=10)
    else:
        Z64, _, info = api.harp_fill(mb, xt, yt, dtype="c128")
        F = api.reduced_factor(Z64)
        finfo = F.info
        X, rep = api.reduced_solve(F, B)
    Y = api.harp_port_admittance(mb, X)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all() and (finfo.cpu().numpy() == 0).all()
    if keep_z:
        return X.cpu().numpy(), Y.cpu().numpy(), rep, Zres.cpu().numpy(), B.cpu().numpy()
    return X.cpu().numpy(), Y.cpu().numpy(), rep


def _check_against_oracle(wl, models, X, Y, tol):
    worst = 0.0
    for f, m in enumerate(models):
        Zo = ofill.fill(m, wl.x, wl.y)
        Bo = osolve.port_rhs(m.w, wl.n_ant)
        Xo = osolve.solve(Zo, Bo)
        Yo = osolve.admittance(Xo, m.w, wl.n_ant)
        ex = np.linalg.norm(X[f] - Xo) / np.linalg.norm(Xo)
        ey = np.linalg.norm(Y[f] - Yo) / np.linalg.norm(Yo)
        col = (np.linalg.norm(X[f] - Xo, axis=0) / np.linalg.norm(Xo, axis=0)).max()
        worst = max(worst, ex, ey, col)
        assert ex <= tol and ey <= tol and col <= tol, (f, ex, ey, col)
    return worst


@pytest.mark.parametrize("refined", [True, False])
def test_hot_path_small16(api, refined):
    wl, models = oracle_models("small16")
    X, Y, rep = _pipeline(api, models, wl.x, wl.y, refined)
    _check_against_oracle(wl, models, X, Y, REL_SOLVE if refined else REL_PLAIN)


@pytest.mark.parametrize("refined", [True, False])
def test_hot_path_station_sweep_all_frequencies(api, refined):
    """The benchmark's configuration: 256 elements x 8 MBFs (n = 2048), 256
    ports, 16 frequencies in one batch; every frequency vs the oracle."""
    wl, models = oracle_models("station_sweep")
    X, Y, rep = _pipeline(api, models, wl.x, wl.y, refined)
    _check_against_oracle(wl, models, X, Y, REL_SOLVE if refined else REL_PLAIN)
    if refined:
        assert all(r["converged"] for r in rep)


def test_hot_path_station_sweep_complex64_fill(api):
    """The same configuration with the complex64 fill (FP32 evaluation) and
    the FP64 residual taken against that complex64 matrix: every frequency
    within the refined bar of the oracle, and each system at its own fixed
    point (FP64 residual against the complex64 matrix, recomputed on the
    host, within the refinement tolerance)."""
    wl, models = oracle_models("station_sweep")
    X, Y, rep, Zr, B = _pipeline(api, models, wl.x, wl.y, "refined32", keep_z=True)
    assert all(r["converged"] for r in rep)
    _check_against_oracle(wl, models, X, Y, REL_SOLVE)
    for f in range(len(models)):
        Z = Zr[f].astype(np.complex128)
        R = B[f] - Z @ X[f]
        rel = np.linalg.norm(R) / (np.linalg.norm(Z) * np.linalg.norm(X[f]))
        assert rel <= 1e-10, (f, rel)


def test_hot_path_strong_coupling(api):
    """Larger self-block regularisation: off-diagonal blocks ~ 1/4 of the
    diagonal, so the solve depends on the coupling (16-element array's element, a_w = 0.3)."""
    wl, models = oracle_models("small16", wire_radius=0.3)
    for refined in (True, False):
        X, Y, _ = _pipeline(api, models, wl.x, wl.y, refined)
        _check_against_oracle(wl, models, X, Y, REL_SOLVE if refined else REL_PLAIN)
