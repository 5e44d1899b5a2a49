"""Oracle: HARP model construction (test infrastructure only).

Section II-A, Eqs. (1)-(3), with the improvements of Section II-B:
  * the remainder B = (Z_exact - Z_app) / e^{-jkr}  (Eq. 2) is sampled on a
    polar grid, regular in the angle alpha and regular in 1/r (Section II-B);
  * it is modelled as sum_{|p|<=P} e^{j p alpha} sum_{q=0..Q} c_pq d^q  (Eq. 3)
    with the modified variable d = 1/r of Section II-B, here normalised as
    t = r_min / r in [0, 1] (t = 0 is r = infinity);
  * the harmonic coefficients come from a DFT over alpha (Section II-B) and the
    polynomial coefficients from a least-squares fit over t (Householder QR).

Readings (the paper gives no numbers): N_alpha = 4 (P + 1), N_t = 2 (Q + 1)
radial samples t_l = l / N_t (l = 0..N_t), B = 0 at t = 0 (the exact limit,
because Z_app is the exact asymptote of Z_exact).

Tabulated form.  The far-field term of Eq. (4) is expanded on the same Fourier
basis, f_p = DFT of G_ff, and folded into the q = 1 column (1/r = t / r_min):

  C_pq = c_pq + delta_{q1} f_p / r_min,
  Z(r, alpha) = e^{-jkr} sum_p e^{j p alpha} sum_q C_pq t^q          (Eq. 4).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import em


@dataclass
class Model:
    freq: float
    k: float
    P: int
    Q: int
    r_min: float
    C: np.ndarray        # (n_mbf T, n_mbf S, 2P+1 (index p+P), Q+1) complex128
    Z_self: np.ndarray   # (n_mbf, n_mbf) complex128, rows T, columns S
    w: np.ndarray        # (n_mbf,) port weights
    fit_resid: float = 0.0   # max over (T,S,p) of the LS residual norm
    samples: np.ndarray | None = None
    wire_radius: float = 0.02

    @property
    def n_mbf(self) -> int:
        return int(self.C.shape[0])


def grid(P: int, Q: int, r_min: float, n_alpha: int | None = None, n_t: int | None = None):
    """Polar sampling grid: alpha_i = 2 pi i / N_alpha, t_l = l / N_t."""
    n_alpha = 4 * (P + 1) if n_alpha is None else n_alpha
    n_t = 2 * (Q + 1) if n_t is None else n_t
    alpha = 2.0 * np.pi * np.arange(n_alpha) / n_alpha
    t = np.arange(n_t + 1) / n_t
    return alpha, t


def remainder_samples(freq, samples, P, Q, r_min, n_alpha=None, n_t=None):
    """Eq. (2) on the grid: B[i, l, T, S] (l = 0 row is zero) and G_ff[i, T, S]."""
    alpha, t = grid(P, Q, r_min, n_alpha, n_t)
    k = em.wavenumber(freq)
    na, nt1 = alpha.size, t.size
    n_mbf = samples.shape[0]
    r = r_min / t[1:]                                            # (N_t,)
    Rx = (r[None, :] * np.cos(alpha)[:, None]).ravel()           # (i, l) order
    Ry = (r[None, :] * np.sin(alpha)[:, None]).ravel()
    Zex = em.reaction_grid(freq, samples, Rx, Ry).reshape(na, nt1 - 1, n_mbf, n_mbf)
    Gff = em.g_far(freq, samples, alpha)                          # (i, T, S)
    Zapp = Gff[:, None, :, :] * (np.exp(-1j * k * r) / r)[None, :, None, None]
    B = np.zeros((na, nt1, n_mbf, n_mbf), dtype=np.complex128)
    B[:, 1:] = (Zex - Zapp) * np.exp(1j * k * r)[None, :, None, None]
    return alpha, t, B, Gff


def dft_harmonics(values: np.ndarray, alpha: np.ndarray, P: int) -> np.ndarray:
    """h_p = N_alpha^-1 sum_i values[i, ...] e^{-j p alpha_i}, p = -P..P
    (first axis of the result is p + P)."""
    p = np.arange(-P, P + 1)
    E = np.exp(-1j * np.outer(p, alpha)) / alpha.size             # (2P+1, N_alpha)
    return np.tensordot(E, values, axes=(1, 0))


def ls_poly(t: np.ndarray, b: np.ndarray, Q: int):
    """Least squares of sum_q c_q t_l^q against b[l, ...] by Householder QR.
    Returns (c[q, ...], residual norm per trailing index)."""
    V = t[:, None] ** np.arange(Q + 1)[None, :]                   # (L, Q+1)
    Qm, Rm = np.linalg.qr(V)                                       # reduced QR
    bb = b.reshape(b.shape[0], -1)
    c = np.linalg.solve(Rm, Qm.conj().T @ bb)
    res = np.linalg.norm(V @ c - bb, axis=0)
    return c.reshape((Q + 1,) + b.shape[1:]), res.reshape(b.shape[1:])


def fit(freq: float, samples: np.ndarray, P: int, Q: int, r_min: float,
        wire_radius: float = 0.02, n_alpha=None, n_t=None) -> Model:
    """Build the HARP model of one element at one frequency (Eqs. 1-3)."""
    samples = np.ascontiguousarray(samples, dtype=np.float64)
    alpha, t, B, Gff = remainder_samples(freq, samples, P, Q, r_min, n_alpha, n_t)
    b = dft_harmonics(B, alpha, P)                                 # (p, l, T, S)
    c, res = ls_poly(t, np.moveaxis(b, 1, 0), Q)                   # c: (q, p, T, S)
    f = dft_harmonics(Gff, alpha, P)                               # (p, T, S)
    C = np.moveaxis(c, (0, 1), (3, 2)).copy()                      # (T, S, p, q)
    C[:, :, :, 1] += np.moveaxis(f, 0, 2) / r_min
    Zs = em.self_block(freq, samples, wire_radius)
    w = (samples[:, 0, 6] + 1j * samples[:, 0, 7]).astype(np.complex128)
    return Model(freq, em.wavenumber(freq), P, Q, r_min, C, Zs, w, float(res.max()),
                 samples, wire_radius)
