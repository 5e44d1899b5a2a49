"""Pins of the oracle's port excitation, dense solve and admittances, and of the
pattern sum (Eqs. 5-6), plus the paper's own accuracy figure on a 16-element
array (Section III-B)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import em, fill, fit, patterns, solve
from workloads import element, workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_complex(n, m, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))


def test_plain_lu_matches_lapack_pivots_and_solution():
    A = _rand_complex(40, 40, 1)
    LU, piv = solve.lu_partial_pivot(A)
    lu_ref, piv_ref = scipy.linalg.lu_factor(A)
    assert np.array_equal(piv, piv_ref)
    assert np.abs(LU - lu_ref).max() < 1e-12 * np.abs(lu_ref).max()
    B = _rand_complex(40, 5, 2)
    X = solve.lu_solve(LU, piv, B)
    assert np.abs(X - np.linalg.solve(A, B)).max() < 1e-11 * np.abs(X).max()


@pytest.fixture(scope="module")
def small16_system():
    wl = workload("small16")
    m = fit.fit(wl.freqs[0], wl.elem.samples, 6, 6, wl.r_min)
    Z = fill.fill(m, wl.x, wl.y)
    return wl, m, Z


def test_backward_error_and_recovery(small16_system):
    _, _, Z = small16_system
    n = Z.shape[0]
    Xt = _rand_complex(n, 7, 3)
    B = Z @ Xt
    X = solve.solve(Z, B)
    u = np.finfo(np.float64).eps / 2
    assert np.linalg.norm(Z @ X - B) / (np.linalg.norm(Z) * np.linalg.norm(X)) < 10 * n * u
    assert np.linalg.norm(X - Xt) / np.linalg.norm(Xt) < 10 * n * u * np.linalg.cond(Z)


def test_port_rhs_layout():
    w = np.array([1 + 2j, 3 - 1j, 0.5j])
    B = solve.port_rhs(w, 4)
    assert B.shape == (12, 4)
    for j in range(4):
        col = np.zeros(12, complex)
        col[3 * j:3 * j + 3] = w
        assert np.array_equal(B[:, j], col)


def test_admittance_symmetric_and_single_element(small16_system):
    wl, m, Z = small16_system
    B = solve.port_rhs(m.w, wl.n_ant)
    X = solve.solve(Z, B)
    Y = solve.admittance(X, m.w, wl.n_ant)
    assert np.abs(Y - Y.T).max() < 1e-12 * np.abs(Y).max()
    # one element: X = Z_self^{-1} w, Y = w^T Z_self^{-1} w
    X1 = solve.solve(m.Z_self, m.w.reshape(-1, 1))
    Y1 = solve.admittance(X1, m.w, 1)
    assert abs(Y1[0, 0] - m.w @ np.linalg.inv(m.Z_self) @ m.w) < 1e-12 * abs(Y1[0, 0])


def test_pattern_of_lone_mbf_is_its_radiation_vector():
    el = element(3, 5, seed=9)
    th = np.array([0.3, 1.1, 2.0])
    ph = np.array([0.0, 2.5, 4.0])
    X = np.zeros((3, 1), complex)
    X[1, 0] = 1.0
    E = patterns.embedded_patterns(100e6, el.samples, np.zeros(1), np.zeros(1), X, th, ph)
    Fth, Fph = patterns.mbf_patterns(100e6, el.samples, th, ph)
    pref = -1j * em.omega_mu(100e6) / (4 * math.pi)
    assert np.allclose(E[0, :, 0], pref * Fth[:, 1], rtol=1e-14, atol=0)
    assert np.allclose(E[0, :, 1], pref * Fph[:, 1], rtol=1e-14, atol=0)


def test_pattern_is_far_limit_of_the_radiated_field():
    """E(theta, phi) is r e^{jkr} times the exact field -j omega mu0 sum G.J at
    distance r, in the limit r -> infinity (error ~ 1/r)."""
    f = 90e6
    k = em.wavenumber(f)
    el = element(2, 3, seed=4)
    x = np.array([0.0, 2.0])
    y = np.array([0.0, -1.0])
    X = _rand_complex(4, 1, 5)
    th, ph = 0.8, 1.3
    E = patterns.embedded_patterns(f, el.samples, x, y, X, [th], [ph])[0, 0]
    u, eth, eph = patterns.unit_vectors([th], [ph])
    errs = []
    rs = [3e2, 3e3, 3e4]
    for r in rs:
        field = np.zeros(3, complex)
        for i in range(2):
            for j in range(2):
                for s in range(3):
                    smp = el.samples[j, s]
                    src = np.array([x[i], y[i], 0.0]) + smp[0:3]
                    G = em.dyadic(k, r * u[0] - src)
                    field += -1j * em.omega_mu(f) * G @ smp[3:6] * (smp[6] + 1j * smp[7]) * X[2 * i + j, 0]
        lim = r * np.exp(1j * k * r) * np.array([field @ eth[0], field @ eph[0]])
        errs.append(np.abs(lim - E).max())
    slopes = np.diff(np.log(errs)) / np.diff(np.log(rs))
    assert np.all(np.abs(slopes + 1) < 0.1), slopes
    assert errs[-1] < 1e-3 * np.abs(E).max()


def test_paper_accuracy_bound_on_16_element_array(small16_system):
    """Section III-B: on a 16-element array the EEPs of the HARP solution
    differ from those of the brute-force solution by less than -30 dB
    (Eq. 8, normalised to the isolated-pattern maximum)."""
    gold = json.load(open(os.path.join(GOLDEN, "paper_eep_accuracy.json")))
    wl, m, Z = small16_system
    nm = m.n_mbf
    Zb = Z.copy()
    for a in range(wl.n_ant):
        for b in range(wl.n_ant):
            if a != b:
                Zb[a * nm:(a + 1) * nm, b * nm:(b + 1) * nm] = em.reaction_grid(
                    wl.freqs[0], wl.elem.samples, [wl.x[a] - wl.x[b]], [wl.y[a] - wl.y[b]])[0]
    B = solve.port_rhs(m.w, wl.n_ant)
    X = solve.solve(Z, B)
    Xb = solve.solve(Zb, B)
    th = np.linspace(0.01, 0.5 * math.pi, 13)
    TH, PH = np.meshgrid(th, np.linspace(0, 2 * math.pi, 24, endpoint=False), indexing="ij")
    E = patterns.embedded_patterns(wl.freqs[0], wl.elem.samples, wl.x, wl.y, X, TH, PH)
    Eb = patterns.embedded_patterns(wl.freqs[0], wl.elem.samples, wl.x, wl.y, Xb, TH, PH)
    Xi = solve.solve(m.Z_self, m.w.reshape(-1, 1))
    Ei = patterns.embedded_patterns(wl.freqs[0], wl.elem.samples, [0.0], [0.0], Xi, TH, PH)
    norm = np.sqrt((np.abs(Ei) ** 2).sum(-1)).max()
    eps = np.sqrt((np.abs(E - Eb) ** 2).sum(-1)) / norm
    assert 20 * np.log10(eps.max()) < gold["bound_db"]
