"""GPU parity at the large-array size: 1024 elements in a 38 m disk, 8 MBFs
(n = 8192), 200 MHz, radius of influence 12 m (block-sparse fill), 1024 ports,
complex64 LU with FP64 refinement -- the whole hot path in the benchmark's
launch configuration, checked against the FP64 oracle on every block of the
matrix and on every port's solution, and on properties that hold at any
size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import solve as osolve  # noqa: E402

from parity import block_eps, oracle_fill_threads, oracle_models, pack  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1702_03781_amd import api as A
    return A


@pytest.fixture(scope="module")
def large(api):
    wl, models = oracle_models("large1024")
    m = models[0]
    mb = api.stack_models([pack(api, m)])
    xt = torch.from_numpy(wl.x).cuda()
    yt = torch.from_numpy(wl.y).cuda()
    Z64, Z32, info = api.harp_fill(mb, xt, yt, dtype="c128", ri=wl.ri, dual=True)
    B = api.harp_port_rhs(mb, wl.n_ant)
    F = api.reduced_factor(Z32)
    X, rep = api.reduced_solve(F, B, Z64=Z64, tol=1e-10, max_iter=10)
    Y = api.harp_port_admittance(mb, X)
    torch.cuda.synchronize()
    return wl, m, Z64, info, F, B, X, rep, Y


@pytest.fixture(scope="module")
def oracle_large(large):
    """The oracle's matrix of the large array and its LAPACK solution for all
    1024 ports."""
    wl, m = large[0], large[1]
    Zo = oracle_fill_threads(m, wl.x, wl.y, wl.ri)
    Xo = osolve.solve(Zo, osolve.port_rhs(m.w, wl.n_ant))
    Yo = osolve.admittance(Xo, m.w, wl.n_ant)
    return Zo, Xo, Yo


def test_large_fill_every_block(api, large, oracle_large):
    """Every off-diagonal block within the radius of influence against the
    oracle's evaluation (1e-12), every block beyond it exactly zero, every
    self block exactly Z_self."""
    wl, m, Z64, info, *_ = large
    Zo = oracle_large[0]
    assert int(info.cpu()[0]) == 0
    Zg = Z64[0].cpu().numpy()
    eps, zero_ok, glob = block_eps(Zg, Zo, m.n_mbf)
    assert eps <= 1e-12 and zero_ok and glob <= 1e-12, (eps, zero_ok, glob)
    nm = m.n_mbf
    for a in range(wl.n_ant):
        assert np.array_equal(Zg[a * nm:(a + 1) * nm, a * nm:(a + 1) * nm], m.Z_self), a
    # the radius of influence leaves most blocks at zero
    d = np.hypot(wl.x[:, None] - wl.x[None, :], wl.y[:, None] - wl.y[None, :])
    assert 0.05 < ((d <= wl.ri) & (d > 0)).mean() < 0.2


def test_large_solve_refined(api, large, oracle_large):
    """Refinement converges; the FP64 residual (recomputed here with a plain
    complex128 product) meets the tolerance; the admittance matrix is
    symmetric (reciprocity); every port's solution and the whole admittance
    matrix match the oracle's LAPACK solve of the oracle's matrix to 1e-6."""
    wl, m, Z64, info, F, B, X, rep, Y = large
    Zo, Xo, Yo = oracle_large
    assert int(F.info.cpu()[0]) == 0
    assert rep[0]["converged"] and rep[0]["iters"] <= 3, rep
    R = B[0] - Z64[0] @ X[0]
    rel = (torch.linalg.norm(R) / (torch.linalg.norm(Z64[0]) * torch.linalg.norm(X[0]))).item()
    assert rel <= 1e-10, rel
    Yh = Y[0].cpu().numpy()
    assert np.linalg.norm(Yh - Yh.T) <= 1e-8 * np.linalg.norm(Yh)
    Xg = X[0].cpu().numpy()
    err = np.linalg.norm(Xg - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    assert err.max() <= 1e-6, err.max()
    assert np.linalg.norm(Yh - Yo) <= 1e-6 * np.linalg.norm(Yo)
