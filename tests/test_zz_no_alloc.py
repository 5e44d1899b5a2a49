"""The allocation-free solve (reduced_solve_noalloc, scratch in a static
device array) against reduced_solve with a caller workspace, through the C
ABI: two calls in a row, the second with a smaller system and fewer
right-hand sides, with and without FP64 refinement; a call whose scratch
would exceed the static array is refused."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1702_03781_amd import api as A
    return A


def _case(api, n, nrhs, batch, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((batch, n, n)) + 1j * rng.standard_normal((batch, n, n))
    A += 2.0 * np.sqrt(n) * np.eye(n)[None]
    B = rng.standard_normal((batch, n, nrhs)) + 1j * rng.standard_normal((batch, n, nrhs))
    Z64 = api.colmajor(batch, n, n, torch.complex128, "cuda")
    Z64.copy_(torch.from_numpy(A))
    Z32 = api.colmajor(batch, n, n, torch.complex64, "cuda")
    Z32.copy_(torch.from_numpy(A.astype(np.complex64)))
    Bt = api.colmajor(batch, n, nrhs, torch.complex128, "cuda")
    Bt.copy_(torch.from_numpy(B))
    F = api.reduced_factor(Z32)
    return A, B, Z64, F, Bt


def _noalloc(api, F, Bt, Z64, tol, max_iter, refine):
    from paper_1702_03781_amd._lib import HarpRefine, HarpRefineReport, lib
    LU = F.LU
    b, n, _ = LU.shape
    nrhs = Bt.shape[-1]
    X = api.colmajor(b, n, nrhs, torch.complex128, "cuda")
    pl, lda, sl = api._cm(LU, "LU")
    pb, ldb, sb = api._cm(Bt, "B")
    px, ldx, sx = api._cm(X, "X")
    ref, rep = None, None
    if refine:
        pz, ldz, sz = api._cm(Z64, "Z64")
        ref = HarpRefine(pz, ldz, sz, tol, max_iter, None)
        rep = (HarpRefineReport * b)()
    st = lib().reduced_solve_noalloc(n, nrhs, b, api.C64, pl, lda, sl, api._ptr(F.ipiv), api._ptr(F.aux),
                                     F.aux.numel(), pb, ldb, sb, px, ldx, sx,
                                     ctypes.byref(ref) if ref is not None else None, rep,
                                     torch.cuda.current_stream().cuda_stream)
    reports = None if rep is None else [{"iters": r.iters, "converged": bool(r.converged),
                                         "resid_rel": r.resid_rel} for r in rep]
    return st, X, reports


@pytest.mark.parametrize("refine", [True, False])
def test_noalloc_matches_workspace_solve(api, refine):
    for n, nrhs, batch, seed in [(700, 33, 3, 1), (300, 7, 2, 2)]:
        A, B, Z64, F, Bt = _case(api, n, nrhs, batch, seed)
        st, Xs, rs = _noalloc(api, F, Bt, Z64, 1e-12, 8, refine)
        assert st == 0
        Xw, rw = api.reduced_solve(F, Bt, Z64=Z64 if refine else None, tol=1e-12, max_iter=8)
        torch.cuda.synchronize()
        # same kernels on the same inputs: identical results and reports
        assert torch.equal(Xs, Xw), (n, refine)
        assert rs == rw
        ref = np.linalg.solve(A, B)
        err = np.linalg.norm(Xs.cpu().numpy() - ref) / np.linalg.norm(ref)
        # forward error <= condition number (a few here) x the residual tolerance
        assert err <= (1e-10 if refine else 1e-4), err


def test_noalloc_refuses_oversized_scratch(api):
    from paper_1702_03781_amd._lib import lib
    L = lib()
    cap = L.reduced_solve_noalloc_max_bytes()
    assert cap == 64 << 20
    need = ctypes.c_size_t()
    n, nrhs, batch = 2048, 1024, 4
    assert L.reduced_solve_ws(n, nrhs, batch, api.C64, 1, ctypes.byref(need)) == 0 and need.value > cap
    # refused before anything is enqueued (no device pointer is read)
    st = L.reduced_solve_noalloc(n, nrhs, batch, api.C64, 1, n, n * n, 1, 1, 1 << 40, 1, n, n * nrhs, 1, n,
                                 n * nrhs, None, None, torch.cuda.current_stream().cuda_stream)
    assert st == -6
