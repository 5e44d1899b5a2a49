"""Oracle: embedded element patterns (test infrastructure only).

Eqs. (5)-(6), Section II-C: with one MBF set shared by all identical elements,
the pattern radiated for a coefficient vector c (one column of X, i.e. the
excitation of one port) is

  F(theta, phi) = sum_j F_j(theta, phi) sum_i c_ij e^{jk (u_x x_i + u_y y_i)}

(F_j the pattern of MBF j, (x_i, y_i) the antenna positions, u the unit vector
toward (theta, phi)).  Here it is evaluated by the direct double sum.

Normalisation (a reading): E = -(j omega mu0 / 4 pi) F, so that the far
electric field is E e^{-jkr} / r; components on theta-hat and phi-hat.
"""
from __future__ import annotations

import math

import numpy as np

from . import em


def unit_vectors(theta, phi):
    th, ph = np.ravel(theta), np.ravel(phi)
    u = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    eth = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], -1)
    eph = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], -1)
    return u, eth, eph


def mbf_patterns(freq, samples, theta, phi):
    """(F_theta, F_phi) of every MBF: arrays (n_dir, n_mbf)."""
    u, eth, eph = unit_vectors(theta, phi)
    F = em.far_patterns(freq, samples, u[:, 0], u[:, 1], u[:, 2], +1)   # (D, M, 3)
    return np.einsum("dmc,dc->dm", F, eth), np.einsum("dmc,dc->dm", F, eph)


def embedded_patterns(freq, samples, x, y, X, theta, phi) -> np.ndarray:
    """E[port, dir, 0/1] = (E_theta, E_phi) for every column of X."""
    k = em.wavenumber(freq)
    u, _, _ = unit_vectors(theta, phi)
    n_mbf = samples.shape[0]
    na = np.size(x)
    Fth, Fph = mbf_patterns(freq, samples, theta, phi)                  # (D, M)
    AF_phase = np.exp(1j * k * (np.outer(u[:, 0], x) + np.outer(u[:, 1], y)))  # (D, Na)
    Xr = np.asarray(X).reshape(na, n_mbf, -1)                           # (i, j, port)
    AF = np.einsum("di,ijk->djk", AF_phase, Xr, optimize=True)          # (D, M, port)
    pref = -1j * em.omega_mu(freq) / (4.0 * math.pi)
    Eth = pref * np.einsum("dj,djk->kd", Fth, AF)
    Eph = pref * np.einsum("dj,djk->kd", Fph, AF)
    return np.stack([Eth, Eph], axis=-1)
