"""Pins of the oracle's position gradient (oracle/adjoint.py) against finite
differences of the oracle's own forward chain, which it shares only through
the model: the model derivative, the objective's cotangents, and the whole
adjoint gradient on a small array."""
import numpy as np
import pytest

from oracle import adjoint as oadj, fill as ofill
from workloads import directions, workload

from parity import oracle_models


@pytest.fixture(scope="module")
def small():
    wl, models = oracle_models("small16")
    th, ph = directions(48, seed=7)
    return wl, models[0], th, ph


def test_model_derivative_matches_central_differences(small):
    _, m, _, _ = small
    rng = np.random.default_rng(3)
    r = rng.uniform(1.6, 9.0, 12)
    a = rng.uniform(-np.pi, np.pi, 12)
    Rx, Ry = r * np.cos(a), r * np.sin(a)
    dx, dy = oadj.eval_model_grad(m, Rx, Ry)
    h = 1e-5
    fx = (ofill.eval_model(m, Rx + h, Ry) - ofill.eval_model(m, Rx - h, Ry)) / (2 * h)
    fy = (ofill.eval_model(m, Rx, Ry + h) - ofill.eval_model(m, Rx, Ry - h)) / (2 * h)
    scale = np.abs(dx).max() + np.abs(dy).max()
    assert np.abs(dx - fx).max() <= 1e-7 * scale
    assert np.abs(dy - fy).max() <= 1e-7 * scale


def test_objective_cotangents_directional(small):
    wl, m, th, ph = small
    Y, E, _, _ = oadj.response(m, wl.x, wl.y, th, ph)
    gY, gE = oadj.objective_cotangents(Y, E, 1.0, 1e9)
    rng = np.random.default_rng(5)
    dY = rng.standard_normal(Y.shape) + 1j * rng.standard_normal(Y.shape)
    dE = rng.standard_normal(E.shape) + 1j * rng.standard_normal(E.shape)
    dY *= 1e-6 * np.abs(Y).max() / np.abs(dY).max()
    dE *= 1e-6 * np.abs(E).max() / np.abs(dE).max()
    lin = np.real(np.sum(np.conj(gY) * dY) + np.sum(np.conj(gE) * dE))
    fd = (oadj.objective(Y + dY, E + dE, 1.0, 1e9) - oadj.objective(Y - dY, E - dE, 1.0, 1e9)) / 2
    assert abs(lin - fd) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("w1,w2,steps,tol,h2", [
    # J1 (port impedances of the synthetic element, ~MOhm) is ~1e9 and moves by
    # a relative 1e-12 per 1e-4 m: central differences are limited by rounding
    # near 1e-3 m, so only the level is checked
    (1.0, 0.0, (2e-3, 1e-3), 2e-5, False),
    # J2 (pattern gain spread) is O(1) and well conditioned: level and h^2 decay
    (0.0, 1.0, (1e-3, 5e-4), 1e-6, True),
])
def test_gradient_matches_finite_differences(small, w1, w2, steps, tol, h2):
    """All 2 N_a coordinates by central differences at two steps: the error at
    the smaller step is below tol and, where rounding allows, shrinks as h^2
    (factor 4 for a halved step, >= 2.5 asked)."""
    wl, m, th, ph = small
    gx, gy = oadj.gradient(m, wl.x, wl.y, th, ph, w1=w1, w2=w2)
    g = np.concatenate([gx, gy])

    def J(x, y):
        Y, E, _, _ = oadj.response(m, x, y, th, ph)
        return oadj.objective(Y, E, w1, w2)

    errs = []
    for h in steps:
        fd = np.zeros_like(g)
        for c in range(2 * wl.x.size):
            x, y = wl.x.copy(), wl.y.copy()
            v = x if c < wl.x.size else y
            i = c % wl.x.size
            v[i] += h
            jp = J(x, y)
            v[i] -= 2 * h
            jm = J(x, y)
            fd[c] = (jp - jm) / (2 * h)
        errs.append(np.linalg.norm(fd - g) / np.linalg.norm(g))
    assert errs[1] <= tol, errs
    if h2:
        assert errs[1] <= errs[0] / 2.5, errs


def test_gradient_translation_invariance(small):
    """Moving the whole array rigidly leaves Y unchanged and E changed by a
    phase, so J is invariant: the gradients sum to zero in x and in y."""
    wl, m, th, ph = small
    gx, gy = oadj.gradient(m, wl.x, wl.y, th, ph)
    assert abs(gx.sum()) <= 1e-9 * np.abs(gx).sum()
    assert abs(gy.sum()) <= 1e-9 * np.abs(gy).sum()
