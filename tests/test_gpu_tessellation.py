"""GPU parity of the overlapping-subarray tessellation (Section II-D) on the
large array (1024 elements in a 38 m disk, 8 MBFs, 200 MHz): R_in = R_ext =
6 m, 61 cells, subarrays of 21-90 elements solved as one batch (complex64 LU,
FP64 refinement, inner ports only).  Every antenna's subarray, X column,
Y column and embedded pattern against the FP64 oracle's tessellation; and the
tessellated patterns approach the full n = 8192 solution as R_ext grows."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import tessellation as ot  # noqa: E402
from workloads import directions  # noqa: E402

from parity import oracle_models, pack  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1702_03781_amd import api as A
    return A


@pytest.fixture(scope="module")
def large(api):
    wl, models = oracle_models("large1024")
    m = models[0]
    model = pack(api, m)
    mb = api.stack_models([model])
    th, ph = directions(128, seed=9)
    return wl, m, model, mb, th, ph


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_tessellated_matches_oracle(api, large):
    wl, m, model, mb, th, ph = large
    T = api.TessellatedSolver(mb, wl.x, wl.y, [0], 6.0, 6.0, tol=1e-10)
    T.step()
    E = T.patterns([model], 0, torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    assert len(T.cells) == 61
    assert all(r["converged"] for r in T.batch.reports)
    assert all(int(T.batch.system(s)[2]) == 0 and int(T.batch.system(s)[3]) == 0
               for s in range(T.batch.n_systems))
    res, Eo = ot.solve_tessellated(m, wl.x, wl.y, 6.0, 6.0, th, ph)
    worst = 0.0
    for a in range(wl.n_ant):
        mem, xg, yg = T.port(a, 0)
        mo, xo, yo = res[a]
        assert np.array_equal(mem, mo), a
        worst = max(worst, _rel(xg.cpu().numpy(), xo), _rel(yg.cpu().numpy(), yo), _rel(E[a], Eo[a]))
    assert worst <= 1e-6, worst


def test_tessellation_converges_to_the_full_solution(api, large):
    """Mean relative EEP error of the tessellated solution against the full
    refined solve of the whole array decreases as R_ext grows (Section IV-B)."""
    wl, m, model, mb, th, ph = large
    tht, pht = torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda()
    full = api.StationSolver(mb, torch.from_numpy(wl.x).cuda(), torch.from_numpy(wl.y).cuda(), "refined",
                             tol=1e-10)
    X, _ = full.step()
    assert all(r["converged"] for r in full.reports)
    Ef = api.embedded_patterns(model, full.x, full.y, X, tht, pht).cpu().numpy()
    del full, X
    errs = []
    for r_ext in (0.0, 3.0, 6.0, 12.0):
        T = api.TessellatedSolver(mb, wl.x, wl.y, [0], 6.0, r_ext, tol=1e-10)
        T.step()
        E = T.patterns([model], 0, tht, pht).cpu().numpy()
        e = np.linalg.norm((E - Ef).reshape(wl.n_ant, -1), axis=1) / np.linalg.norm(Ef.reshape(wl.n_ant, -1), axis=1)
        errs.append(float(e.mean()))
        del T
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
