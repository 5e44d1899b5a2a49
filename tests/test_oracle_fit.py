"""Pins of the oracle's HARP model construction (Eqs. 2-3, Section II-B)."""
import math

import numpy as np
import pytest

from oracle import em, fit, fill
from workloads import element, workload

F0 = 120e6


@pytest.fixture(scope="module")
def small_model():
    el = element(3, 10, seed=21)
    return el, fit.fit(F0, el.samples, 5, 5, 1.5, wire_radius=0.02)


def test_dft_plus_ls_equals_joint_least_squares(small_model):
    """On a uniform alpha grid with N_alpha >= 2P+1 the DFT over alpha followed
    by per-harmonic least squares over t is the joint least-squares fit of
    Eq. (3) on the full tensor grid (the paper's DFT improvement loses
    nothing)."""
    el, _ = small_model
    P, Q = 5, 5
    alpha, t, B, _ = fit.remainder_samples(F0, el.samples, P, Q, 1.5)
    b = fit.dft_harmonics(B, alpha, P)
    c, _ = fit.ls_poly(t, np.moveaxis(b, 1, 0), Q)                 # (q, p, T, S)
    p = np.arange(-P, P + 1)
    A = (np.exp(1j * np.outer(alpha, p))[:, None, :, None]
         * (t[:, None] ** np.arange(Q + 1))[None, :, None, :]).reshape(alpha.size * t.size, -1)
    data = B.reshape(alpha.size * t.size, -1)
    cj, *_ = np.linalg.lstsq(A, data, rcond=None)                   # ((p,q), TS)
    cj = cj.reshape(2 * P + 1, Q + 1, -1)
    cs = np.moveaxis(c, 0, 1).reshape(2 * P + 1, Q + 1, -1)
    assert np.abs(cj - cs).max() <= 1e-9 * np.abs(cj).max()


def test_in_model_data_is_recovered():
    """Data generated from a random table of the model form is fitted back
    exactly by the DFT + least-squares steps."""
    rng = np.random.default_rng(3)
    P, Q = 4, 5
    alpha, t = fit.grid(P, Q, 1.5)
    c = rng.standard_normal((2 * P + 1, Q + 1)) + 1j * rng.standard_normal((2 * P + 1, Q + 1))
    p = np.arange(-P, P + 1)
    B = np.einsum("pq,ip,lq->il", c, np.exp(1j * np.outer(alpha, p)),
                  t[:, None] ** np.arange(Q + 1))
    b = fit.dft_harmonics(B, alpha, P)                              # (p, l)
    cr, res = fit.ls_poly(t, b.T, Q)                                # (q, p)
    assert np.abs(cr.T - c).max() < 1e-11
    assert res.max() < 1e-11


def test_table_parity_symmetry(small_model):
    """Reciprocity Z_TS(R) = Z_ST(-R) and alpha -> alpha + pi give
    C^{ST}_pq = (-1)^p C^{TS}_pq (N_alpha even)."""
    _, m = small_model
    sign = (-1.0) ** np.arange(-m.P, m.P + 1)
    CT = np.swapaxes(m.C, 0, 1)
    assert np.abs(CT - sign[None, None, :, None] * m.C).max() <= 1e-10 * np.abs(m.C).max()


def test_constant_term_vanishes(small_model):
    """B -> 0 at t = 0 (r = infinity), so the q = 0 column is at the level of
    the least-squares residual, not of the table."""
    _, m = small_model
    assert np.abs(m.C[..., 0]).max() <= 5 * m.fit_resid + 1e-9 * np.abs(m.C).max()
    assert np.abs(m.C[..., 0]).max() < 1e-2 * np.abs(m.C).max()


def test_model_reproduces_grid_and_converges():
    """Model accuracy (reported, not a parity gate): off the grid, out to
    array-scale distances, the model's error against brute-force reactions
    falls as the orders grow."""
    el = element(2, 12, seed=33)
    R = []
    rng = np.random.default_rng(4)
    for i in range(40):
        r = 1.5 + (10 if i < 30 else 80) * rng.uniform()
        a = 2 * math.pi * rng.uniform()
        R.append((r * math.cos(a), r * math.sin(a)))
    R = np.array(R)
    Zex = em.reaction_grid(F0, el.samples, R[:, 0], R[:, 1])
    errs = []
    for P, Q in [(3, 3), (6, 6), (10, 8)]:
        m = fit.fit(F0, el.samples, P, Q, 1.5)
        Zm = fill.eval_model(m, R[:, 0], R[:, 1])
        errs.append(np.linalg.norm(Zm - Zex) / np.linalg.norm(Zex))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def test_far_field_fourier_expansion():
    """The far-field factor folded into the table is the truncated Fourier
    series of G_ff (Eq. 1): at off-grid angles sum_p f_p e^{jp alpha}
    reproduces G_ff once P exceeds the angular bandwidth k D."""
    el = element(3, 10, seed=21)
    P = 14
    alpha, _ = fit.grid(P, 4, 1.5)
    f = fit.dft_harmonics(em.g_far(F0, el.samples, alpha), alpha, P)      # (p, T, S)
    a_off = np.array([0.123, 1.9, 3.3, 5.77])
    series = np.einsum("ap,pts->ats", np.exp(1j * np.outer(a_off, np.arange(-P, P + 1))), f)
    G = em.g_far(F0, el.samples, a_off)
    assert np.abs(series - G).max() < 1e-8 * np.abs(G).max()


def test_small16_fit_is_deterministic():
    wl = workload("small16")
    m1 = fit.fit(wl.freqs[0], wl.elem.samples, 6, 6, wl.r_min)
    m2 = fit.fit(wl.freqs[0], wl.elem.samples, 6, 6, wl.r_min)
    assert np.array_equal(m1.C, m2.C)
    assert m1.C.shape == (4, 4, 13, 7)
