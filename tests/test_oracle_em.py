"""Pins of the oracle's exact reactions and far-field patterns (Section II-A,
Eq. 1) against independent mathematics: finite differences, the radiated-power
identity, reciprocity and the far-field asymptote."""
import math

import numpy as np
import pytest

from oracle import em
from workloads import element

F0 = 150e6
K0 = em.wavenumber(F0)


def _g(k, d):
    r = np.linalg.norm(d)
    return np.exp(-1j * k * r) / (4 * math.pi * r)


def _fd_dyadic(k, d, h):
    """(I + grad grad / k^2) g by central differences of the scalar g."""
    H = np.zeros((3, 3), dtype=complex)
    e = np.eye(3)
    for i in range(3):
        for j in range(3):
            if i == j:
                H[i, i] = (_g(k, d + h * e[i]) - 2 * _g(k, d) + _g(k, d - h * e[i])) / h**2
            else:
                H[i, j] = (_g(k, d + h * e[i] + h * e[j]) - _g(k, d + h * e[i] - h * e[j])
                           - _g(k, d - h * e[i] + h * e[j]) + _g(k, d - h * e[i] - h * e[j])) / (4 * h * h)
    return _g(k, d) * np.eye(3) + H / k**2


@pytest.mark.parametrize("d", [(0.7, -0.3, 1.1), (2.5, 0.4, -0.2), (0.05, 0.3, 0.02)])
def test_dyadic_matches_finite_differences(d):
    d = np.array(d)
    G = em.dyadic(K0, d)
    errs = []
    for h in (1e-3, 5e-4):
        h = h * np.linalg.norm(d)
        errs.append(np.abs(_fd_dyadic(K0, d, h) - G).max() / np.abs(G).max())
    assert errs[1] < 1e-5
    # second-order convergence: halving h divides the error by ~4
    assert 2.5 < errs[0] / errs[1] < 6.0


def _sphere_quadrature(n_th=48, n_ph=96):
    x, wx = np.polynomial.legendre.leggauss(n_th)       # x = cos(theta)
    ph = 2 * math.pi * np.arange(n_ph) / n_ph
    th = np.arccos(x)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(wx, np.full(n_ph, 2 * math.pi / n_ph))
    u = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    return u.reshape(-1, 3), W.ravel()


@pytest.mark.parametrize("seed", [1, 2])
def test_radiated_power_identity(seed):
    """Re(x^H Z^(H) x) = -(omega mu0 k / 16 pi^2) closed-integral |F_perp|^2 dOmega
    for conjugate testing; the s = s' terms use Im G(0) = -(k / 6 pi) I, which
    for one dipole is the Hertzian-dipole radiation resistance."""
    el = element(1, 12, seed=seed)
    smp = el.samples[0].copy()
    J = smp[:, 6] + 1j * smp[:, 7]
    om = em.omega_mu(F0)
    lhs = 0.0
    for s in range(smp.shape[0]):
        Ts = smp[s:s + 1].copy()
        Ts[0, 6], Ts[0, 7] = J[s].real, -J[s].imag        # conjugated testing moment
        for q in range(smp.shape[0]):
            if q == s:
                continue
            lhs += em.reaction(F0, Ts, smp[q:q + 1], (0.0, 0.0, 0.0)).real
    lhs += -om * K0 / (6 * math.pi) * np.sum(np.abs(J) ** 2)
    u, W = _sphere_quadrature()
    F = em.far_patterns(F0, smp[None], u[:, 0], u[:, 1], u[:, 2], +1)[:, 0, :]
    rhs = -(om * K0 / (16 * math.pi**2)) * np.sum(W * np.sum(np.abs(F) ** 2, -1))
    assert abs(lhs - rhs) <= 1e-9 * abs(rhs)


def test_single_dipole_radiation_resistance_closed_form():
    """-eta k^2 |a|^2 / (6 pi) from the power integral of one Hertzian dipole."""
    smp = np.zeros((1, 8))
    smp[0, 5] = 1.0
    smp[0, 6] = 0.8
    smp[0, 7] = -0.6
    u, W = _sphere_quadrature()
    F = em.far_patterns(F0, smp[None], u[:, 0], u[:, 1], u[:, 2], +1)[:, 0, :]
    om = em.omega_mu(F0)
    rhs = -(om * K0 / (16 * math.pi**2)) * np.sum(W * np.sum(np.abs(F) ** 2, -1))
    eta = em.MU0 * em.C0
    assert abs(rhs - (-eta * K0**2 * 1.0 / (6 * math.pi))) < 1e-10 * abs(rhs)


def test_reaction_reciprocity():
    el = element(3, 10, seed=7)
    R = np.array([2.1, -1.3, 0.0])
    for t in range(3):
        for s in range(3):
            a = em.reaction(F0, el.samples[t], el.samples[s], R)
            b = em.reaction(F0, el.samples[s], el.samples[t], -R)
            assert abs(a - b) <= 1e-13 * abs(a)


def test_far_field_asymptote_is_eq1():
    """|r e^{jkr} Z_exact(r, alpha) - G_ff(alpha)| decays as 1/r (Eq. 1 is the
    exact large-distance limit)."""
    el = element(2, 8, seed=11)
    alpha = 0.7
    G = em.g_far(F0, el.samples, [alpha])[0]
    errs = []
    rs = [1e2, 1e3, 1e4]
    for r in rs:
        Z = em.reaction_grid(F0, el.samples, [r * math.cos(alpha)], [r * math.sin(alpha)])[0]
        errs.append(np.abs(r * np.exp(1j * K0 * r) * Z - G).max())
    slopes = np.diff(np.log(errs)) / np.diff(np.log(rs))
    assert np.all(np.abs(slopes + 1.0) < 0.05), slopes
    assert errs[-1] < 1e-3 * np.abs(G).max()


def test_self_block_symmetric_and_reduced_kernel_limit():
    """The zero-distance block is complex-symmetric, and the reduced kernel
    tends to the exact one when the wire radius is negligible against the
    sample spacing."""
    el = element(3, 6, seed=5)
    Zs = em.self_block(F0, el.samples, 0.02)
    assert np.abs(Zs - Zs.T).max() <= 1e-13 * np.abs(Zs).max()
    # one sample per MBF, far apart: reduced kernel -> exact reaction
    smp = el.samples[:, :1].copy()
    smp[:, 0, 0:3] = [[0, 0, 0], [3.0, 0, 0.5], [0, 4.0, 1.0]]
    Zr = em.self_block(F0, smp, 1e-7)
    Zx = em.reaction(F0, smp[0], smp[1], (0, 0, 0))
    assert abs(Zr[0, 1] - Zx) < 1e-9 * abs(Zx)
