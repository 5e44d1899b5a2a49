"""Pins of the oracle's Eq. (4) fill: one-hot tables, the harmonic (Laplace)
property of the model in the modified coordinates, the mean-value property,
reciprocity, self blocks and the radius of influence."""
import math

import numpy as np
import pytest

from oracle import em, fill, fit
from workloads import workload


def _onehot_model(P, Q, p, q, k=0.7, r_min=1.5):
    C = np.zeros((1, 1, 2 * P + 1, Q + 1), dtype=complex)
    C[0, 0, p + P, q] = 1.0
    return fit.Model(100e6, k, P, Q, r_min, C, np.eye(1, dtype=complex), np.ones(1))


@pytest.mark.parametrize("p,q", [(0, 0), (3, 1), (-2, 4), (5, 0), (-5, 6)])
def test_onehot_table_gives_basis_function(p, q):
    m = _onehot_model(5, 6, p, q)
    rng = np.random.default_rng(1)
    R = rng.uniform(-20, 20, size=(50, 2))
    R = R[np.hypot(R[:, 0], R[:, 1]) > 1.5]
    Z = fill.eval_model(m, R[:, 0], R[:, 1])[:, 0, 0]
    # basis function written with plain cos/sin, the angle measured from +x
    # toward the testing antenna
    r = np.hypot(R[:, 0], R[:, 1])
    cos_a, sin_a = R[:, 0] / r, R[:, 1] / r
    w = cos_a + 1j * sin_a
    expect = np.exp(-1j * m.k * r) * (m.r_min / r) ** q * w ** p
    assert np.abs(Z - expect).max() < 1e-13


def _phase_free(m):
    return fit.Model(m.freq, 0.0, m.P, m.Q, m.r_min, m.C, m.Z_self, m.w)


def _model_at_XY(m, X, Y):
    """Evaluate the model at modified-plane point (X, Y) = t (cos a, sin a)."""
    t = np.hypot(X, Y)
    r = m.r_min / t
    return fill.eval_model(m, r * X / t, r * Y / t)


def test_harmonic_laplace_property():
    """In the modified plane (X, Y) = t (cos alpha, sin alpha) the model term
    t^q e^{j p alpha} has Laplacian (q^2 - p^2) t^(q-2) e^{j p alpha}; a 5-point
    stencil of the phase-stripped fill reproduces it."""
    wl = workload("small16")
    m = _phase_free(fit.fit(wl.freqs[0], wl.elem.samples, 6, 6, wl.r_min))
    P, Q = m.P, m.Q
    p = np.arange(-P, P + 1)[:, None]
    q = np.arange(Q + 1)[None, :]
    for (X0, Y0) in [(0.4, 0.3), (-0.2, 0.55), (0.1, -0.6)]:
        h = 2e-4
        f0 = _model_at_XY(m, X0, Y0)
        lap = (_model_at_XY(m, X0 + h, Y0) + _model_at_XY(m, X0 - h, Y0)
               + _model_at_XY(m, X0, Y0 + h) + _model_at_XY(m, X0, Y0 - h) - 4 * f0) / h**2
        t0, a0 = math.hypot(X0, Y0), math.atan2(Y0, X0)
        kern = (q**2 - p**2) * t0 ** (q - 2.0) * np.exp(1j * p * a0)
        expect = np.einsum("tspq,pq->ts", m.C, kern)
        assert np.abs(lap[0] - expect).max() < 1e-6 * np.abs(expect).max()


def test_mean_value_property_of_harmonic_terms():
    """Terms with q = |p| are (X +- jY)^|p|: harmonic, so their mean over a
    circle equals the value at its centre (64-point trapezoid is exact)."""
    P, Q = 4, 6
    C = np.zeros((1, 1, 2 * P + 1, Q + 1), dtype=complex)
    rng = np.random.default_rng(2)
    for p in range(-P, P + 1):
        C[0, 0, p + P, abs(p)] = rng.standard_normal() + 1j * rng.standard_normal()
    m = fit.Model(1e8, 0.0, P, Q, 1.5, C, np.eye(1, dtype=complex), np.ones(1))
    cX, cY, rad = 0.35, -0.2, 0.15
    ang = 2 * math.pi * np.arange(64) / 64
    vals = _model_at_XY(m, cX + rad * np.cos(ang), cY + rad * np.sin(ang))
    centre = _model_at_XY(m, cX, cY)
    assert abs(vals.mean() - centre[0, 0, 0]) < 1e-13 * abs(centre[0, 0, 0])


@pytest.fixture(scope="module")
def small16():
    wl = workload("small16")
    return wl, fit.fit(wl.freqs[0], wl.elem.samples, 6, 6, wl.r_min)


def test_fill_reciprocity_and_self_blocks(small16):
    wl, m = small16
    Z = fill.fill(m, wl.x, wl.y)
    assert np.abs(Z - Z.T).max() <= 1e-13 * np.abs(Z).max()
    nm = m.n_mbf
    for a in range(wl.n_ant):
        assert np.array_equal(Z[a * nm:(a + 1) * nm, a * nm:(a + 1) * nm], m.Z_self)
    # block (a, b) is the model at R = r_a - r_b
    a, b = 3, 11
    blk = fill.eval_model(m, [wl.x[a] - wl.x[b]], [wl.y[a] - wl.y[b]])[0]
    # (equal up to the summation order of the library matrix product)
    assert np.abs(Z[a * nm:(a + 1) * nm, b * nm:(b + 1) * nm] - blk).max() <= 1e-14 * np.abs(blk).max()


def test_radius_of_influence_zeroes_far_blocks(small16):
    wl, m = small16
    ri = 5.0
    Z = fill.fill(m, wl.x, wl.y, ri=ri)
    Zf = fill.fill(m, wl.x, wl.y)
    nm = m.n_mbf
    d = np.hypot(wl.x[:, None] - wl.x[None, :], wl.y[:, None] - wl.y[None, :])
    for a in range(wl.n_ant):
        for b in range(wl.n_ant):
            blk = Z[a * nm:(a + 1) * nm, b * nm:(b + 1) * nm]
            if d[a, b] > ri:
                assert not blk.any()
            else:
                assert np.array_equal(blk, Zf[a * nm:(a + 1) * nm, b * nm:(b + 1) * nm])


def test_hybrid_fill_close_to_brute_force(small16):
    """Model accuracy on the 16-element system (synthetic analogue of the
    paper's 16-element testbed check against brute-force MoM): off-diagonal
    blocks within 1e-2 of the exact reactions (reported, not a parity gate)."""
    wl, m = small16
    Z = fill.fill(m, wl.x, wl.y)
    nm = m.n_mbf
    num = den = 0.0
    for a in range(wl.n_ant):
        for b in range(wl.n_ant):
            if a == b:
                continue
            ex = em.reaction_grid(wl.freqs[0], wl.elem.samples,
                                  [wl.x[a] - wl.x[b]], [wl.y[a] - wl.y[b]])[0]
            num += np.linalg.norm(Z[a * nm:(a + 1) * nm, b * nm:(b + 1) * nm] - ex) ** 2
            den += np.linalg.norm(ex) ** 2
    assert math.sqrt(num / den) < 1e-2


def test_count_below_rmin():
    m = _onehot_model(2, 2, 0, 0)
    x = np.array([0.0, 1.0, 5.0])
    y = np.array([0.0, 0.0, 0.0])
    assert fill.count_below_rmin(m, x, y) == 2
