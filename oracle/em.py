"""Oracle: exact MBF reactions and far-field patterns (test infrastructure only).

Conventions (the paper gives none; these are readings):
  c0 = 299 792 458 m/s, mu0 = 4 pi 1e-7 H/m, omega = 2 pi f, k = omega / c0,
  time factor e^{+j omega t} (implied by the outgoing e^{-jkr} of Eqs. 1-4).
"""
from __future__ import annotations

import math

import numpy as np

from . import _clib

C0 = 299_792_458.0
MU0 = 4.0e-7 * math.pi


def wavenumber(freq_hz: float) -> float:
    return 2.0 * math.pi * freq_hz / C0


def omega_mu(freq_hz: float) -> float:
    return 2.0 * math.pi * freq_hz * MU0


def dyadic(k: float, d) -> np.ndarray:
    """Free-space dyadic Green's function (I + grad grad / k^2) e^{-jkr}/(4 pi r)
    at displacement d, evaluated in closed form by the C oracle."""
    out = np.zeros(18)
    _clib.lib().oracle_dyadic(k, float(d[0]), float(d[1]), float(d[2]), _clib.ptr(out))
    return (out[0::2] + 1j * out[1::2]).reshape(3, 3)


def reaction(freq_hz: float, T: np.ndarray, S: np.ndarray, R, reg: float = 0.0) -> complex:
    """Galerkin reaction of testing cloud T (reference point at R) with source
    cloud S (reference point at the origin), Section II-A exact interaction.
    T, S: (n, 8) sample records."""
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1, 8)
    S = np.ascontiguousarray(S, dtype=np.float64).reshape(-1, 8)
    out = np.zeros(2)
    _clib.lib().oracle_reaction(wavenumber(freq_hz), omega_mu(freq_hz), T.shape[0],
                                _clib.ptr(T), S.shape[0], _clib.ptr(S),
                                float(R[0]), float(R[1]), float(R[2]), float(reg),
                                _clib.ptr(out))
    return complex(out[0], out[1])


def reaction_grid(freq_hz: float, samples: np.ndarray, Rx, Ry, reg: float = 0.0) -> np.ndarray:
    """Exact reactions Z_TS(R) for every ordered MBF pair and every in-plane
    displacement R = (Rx[p], Ry[p], 0).  Returns (n_pts, n_mbf, n_mbf)."""
    samples = np.ascontiguousarray(samples, dtype=np.float64)
    n_mbf, n_samp = samples.shape[0], samples.shape[1]
    Rx = np.ascontiguousarray(Rx, dtype=np.float64).ravel()
    Ry = np.ascontiguousarray(Ry, dtype=np.float64).ravel()
    out = np.zeros((Rx.size, n_mbf, n_mbf, 2))
    _clib.lib().oracle_reaction_grid(wavenumber(freq_hz), omega_mu(freq_hz), n_mbf, n_samp,
                                     _clib.ptr(samples), Rx.size, _clib.ptr(Rx),
                                     _clib.ptr(Ry), float(reg), _clib.ptr(out))
    return out[..., 0] + 1j * out[..., 1]


def self_block(freq_hz: float, samples: np.ndarray, wire_radius: float) -> np.ndarray:
    """Zero-distance interaction (Section III-A: the self impedance sits at
    zero distance).  Reading: the thin-wire reduced kernel with radius a_w."""
    return reaction_grid(freq_hz, samples, [0.0], [0.0], reg=wire_radius)[0]


def far_patterns(freq_hz: float, samples: np.ndarray, ux, uy, uz, sign: int) -> np.ndarray:
    """Transverse radiation vector of every MBF toward unit directions u:
    F(u) = sum_s a_s (s_hat - (u . s_hat) u) exp(sign * j k u . rho_s).
    sign = +1 is the source pattern of Eq. (1); sign = -1 the testing pattern
    (the reading of the conjugate mark of Eq. (1) that keeps the model the
    exact asymptote for complex currents).  Returns (n_dir, n_mbf, 3)."""
    k = wavenumber(freq_hz)
    u = np.stack([np.ravel(ux), np.ravel(uy), np.ravel(uz)], axis=-1)        # (D, 3)
    pos = samples[..., 0:3]                                                  # (M, N, 3)
    sh = samples[..., 3:6]
    a = samples[..., 6] + 1j * samples[..., 7]                              # (M, N)
    phase = np.exp(sign * 1j * k * np.einsum("dc,mnc->dmn", u, pos))         # (D, M, N)
    us = np.einsum("dc,mnc->dmn", u, sh)                                     # (D, M, N)
    perp = sh[None, :, :, :] - us[..., None] * u[:, None, None, :]           # (D, M, N, 3)
    return np.einsum("mn,dmn,dmnc->dmc", a, phase, perp)


def g_far(freq_hz: float, samples: np.ndarray, alpha) -> np.ndarray:
    """Angular factor of Eq. (1): Z_app(r, alpha) = G_ff(alpha) e^{-jkr} / r with
    G_ff = -(j omega mu0 / 4 pi) F^-_T(alpha) . F^+_S(alpha), alpha-hat in the
    array plane.  Returns (n_alpha, n_mbf (T), n_mbf (S))."""
    alpha = np.ravel(alpha)
    ux, uy, uz = np.cos(alpha), np.sin(alpha), np.zeros_like(alpha)
    Fm = far_patterns(freq_hz, samples, ux, uy, uz, -1)
    Fp = far_patterns(freq_hz, samples, ux, uy, uz, +1)
    return -(1j * omega_mu(freq_hz) / (4.0 * math.pi)) * np.einsum("dtc,dsc->dts", Fm, Fp)
