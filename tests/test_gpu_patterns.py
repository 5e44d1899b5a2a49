"""GPU parity of embedded_patterns (Eqs. 5-6) against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fill as ofill, patterns as opat, solve as osolve  # noqa: E402
from workloads import directions, workload  # noqa: E402

from parity import oracle_models, pack  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1702_03781_amd import api as A
    return A


def _run(api, m, wl, X, th, ph):
    model = pack(api, m)
    Xt = api.colmajor(1, X.shape[0], X.shape[1], torch.complex128, "cuda")
    Xt.copy_(torch.from_numpy(X)[None])
    E = api.embedded_patterns(model, torch.from_numpy(wl.x).cuda(), torch.from_numpy(wl.y).cuda(),
                              Xt, torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda())
    torch.cuda.synchronize()
    return E.cpu().numpy()


def test_patterns_small_array(api):
    wl, models = oracle_models("small16")
    m = models[0]
    X = osolve.solve(ofill.fill(m, wl.x, wl.y), osolve.port_rhs(m.w, wl.n_ant))
    th, ph = directions(37, seed=5)
    E = _run(api, m, wl, X, th, ph)
    Eo = opat.embedded_patterns(m.freq, m.samples, wl.x, wl.y, X, th, ph)
    assert E.shape == Eo.shape == (wl.n_ant, 37, 2)
    assert np.abs(E - Eo).max() <= 1e-12 * np.abs(Eo).max()


def test_patterns_station_all_ports(api):
    """256 elements x 8 MBFs, 256 ports, 1024 directions (the adjoint
    configuration's pattern set)."""
    wl = workload("station_110mhz")
    from oracle import fit as ofit
    m = ofit.fit(wl.freqs[0], wl.elem.samples, wl.P[0], wl.Q, wl.r_min,
                 wire_radius=wl.elem.wire_radius)
    X = osolve.solve(ofill.fill(m, wl.x, wl.y), osolve.port_rhs(m.w, wl.n_ant))
    th, ph = wl.extra["theta"], wl.extra["phi"]
    E = _run(api, m, wl, X, th, ph)
    Eo = opat.embedded_patterns(m.freq, m.samples, wl.x, wl.y, X, th, ph)
    err = np.linalg.norm(E - Eo) / np.linalg.norm(Eo)
    assert err <= 1e-12, err
