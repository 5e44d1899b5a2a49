"""Oracle: reduced-matrix fill from a HARP model (test infrastructure only).

Eq. (4): for a testing antenna m and a source antenna n at relative position
R = (x_m - x_n, y_m - y_n) with distance r and angle alpha (alpha-hat points
from the source reference point to the testing one, Section II-A),

  Z_TS(r, alpha) = e^{-jkr} sum_{p=-P..P} e^{j p alpha} sum_{q=0..Q} C_pq t^q,
  t = r_min / r.

Evaluated naively in FP64: atan2, exp(j p alpha), t**q, one library matrix
product over the (p, q) index.  Diagonal blocks take the zero-distance self
block (Section III-A).  With a radius of influence RI > 0, blocks of pairs
farther apart than RI are zero (Section II-D; r <= RI kept, a reading).

Layout: Z[m * N_m + T, n * N_m + S].
"""
from __future__ import annotations

import numpy as np

from .fit import Model


def eval_model(model: Model, Rx, Ry) -> np.ndarray:
    """Z_TS at displacements (Rx, Ry): returns (n_pts, n_mbf, n_mbf)."""
    Rx = np.ravel(np.asarray(Rx, dtype=np.float64))
    Ry = np.ravel(np.asarray(Ry, dtype=np.float64))
    r = np.hypot(Rx, Ry)
    alpha = np.arctan2(Ry, Rx)
    t = model.r_min / r
    p = np.arange(-model.P, model.P + 1)
    q = np.arange(model.Q + 1)
    Ep = np.exp(1j * np.outer(alpha, p))                            # (n, 2P+1)
    Tq = t[:, None] ** q[None, :]                                   # (n, Q+1)
    V = (Ep[:, :, None] * Tq[:, None, :]).reshape(r.size, -1)       # (n, (2P+1)(Q+1))
    nm = model.n_mbf
    Cm = model.C.reshape(nm * nm, -1)                                # (TS, pq)
    Z = (V @ Cm.T).reshape(r.size, nm, nm)
    return Z * np.exp(-1j * model.k * r)[:, None, None]


def fill(model: Model, x, y, ri: float = 0.0) -> np.ndarray:
    """Dense reduced matrix (n x n, n = N_a N_m), complex128."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    na, nm = x.size, model.n_mbf
    Z = np.zeros((na, nm, na, nm), dtype=np.complex128)
    mm, nn = np.meshgrid(np.arange(na), np.arange(na), indexing="ij")
    off = mm != nn
    if ri > 0.0:
        # blocks of pairs beyond the radius of influence stay zero (not evaluated)
        off &= np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :]) <= ri
    Rx = (x[:, None] - x[None, :])[off]
    Ry = (y[:, None] - y[None, :])[off]
    blocks = np.concatenate([eval_model(model, Rx[i:i + 32768], Ry[i:i + 32768])
                             for i in range(0, Rx.size, 32768)] or
                            [np.zeros((0, nm, nm), dtype=np.complex128)])
    Z[mm[off], :, nn[off], :] = blocks
    for m in range(na):
        Z[m, :, m, :] = model.Z_self
    return Z.reshape(na * nm, na * nm)


def count_below_rmin(model: Model, x, y) -> int:
    """Number of ordered pairs m != n with r < r_min (outside the model)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    np.fill_diagonal(d, np.inf)
    return int((d < model.r_min * (1.0 - 1e-12)).sum())
