"""Oracle: gradient of an array-synthesis objective with respect to the antenna
positions (test infrastructure only).

The forward model is the paper's chain for one element type at one frequency:
the Eq. (4) fill, one solve with a right-hand side per port (Section I), the
port admittances Y = W^T X, and the embedded element patterns of Eqs. (5)-(6).

Objective (a reading: the paper states no synthesis objective):
  J  = J1 + J2
  J1 = sum_i |Zin_i - 50|^2 / (N_a 50^2),   Zin = diag(Y^-1)   (port input impedances)
  J2 = var_d(g) / mean_d(g)^2,  g_d = (1/N_p) sum_{p,c} |E_{p,d,c}|^2  (mean embedded gain)

Gradient by the adjoint method written out plainly in FP64 numpy, independent
of the GPU path: the cotangents of Y and E from J in closed form, the
cotangent of X (ports and patterns), one adjoint solve with Z^H (a full LAPACK
solve, no symmetry assumed), the cotangent of Z, and the analytic derivative of
the Eq. (4) model with respect to the pair displacement R:
  Z_TS = e^{-jkr} sum_pq C_pq e^{jp alpha} t^q,  t = r_min / r
  dZ/dr     = -jk Z - (1/r) e^{-jkr} sum_pq q C_pq e^{jp alpha} t^q
  dZ/dalpha = e^{-jkr} sum_pq jp C_pq e^{jp alpha} t^q
  d/dR_x = cos(alpha) d/dr - sin(alpha)/r d/dalpha,  d/dR_y = sin(alpha) d/dr + cos(alpha)/r d/dalpha.
Complex cotangents follow dJ = Re sum conj(G) dZ.
"""
from __future__ import annotations

import math

import numpy as np

from . import em, fill as ofill, patterns as opat, solve as osolve
from .fit import Model

Z_REF = 50.0


def eval_model_grad(model: Model, Rx, Ry):
    """(dZ/dR_x, dZ/dR_y) of the Eq. (4) model at displacements (Rx, Ry):
    arrays (n_pts, n_mbf, n_mbf)."""
    Rx = np.ravel(np.asarray(Rx, dtype=np.float64))
    Ry = np.ravel(np.asarray(Ry, dtype=np.float64))
    r = np.hypot(Rx, Ry)
    alpha = np.arctan2(Ry, Rx)
    t = model.r_min / r
    p = np.arange(-model.P, model.P + 1)
    q = np.arange(model.Q + 1)
    Ep = np.exp(1j * np.outer(alpha, p))
    Tq = t[:, None] ** q[None, :]
    V = Ep[:, :, None] * Tq[:, None, :]                               # (n, 2P+1, Q+1)
    nm = model.n_mbf
    Cm = model.C.reshape(nm * nm, -1)
    ph = np.exp(-1j * model.k * r)
    flat = lambda A: A.reshape(r.size, -1)                            # noqa: E731
    Z = (flat(V) @ Cm.T) * ph[:, None]
    Zr = -1j * model.k * Z - (flat(V * q[None, None, :]) @ Cm.T) * (ph / r)[:, None]
    Za = (flat(V * (1j * p)[None, :, None]) @ Cm.T) * ph[:, None]
    ca, sa = np.cos(alpha)[:, None], np.sin(alpha)[:, None]
    dx = ca * Zr - (sa / r[:, None]) * Za
    dy = sa * Zr + (ca / r[:, None]) * Za
    return dx.reshape(r.size, nm, nm), dy.reshape(r.size, nm, nm)


def response(model: Model, x, y, theta, phi, ri: float = 0.0):
    """Y (N_a x N_a), E [port][dir][theta/phi], and the intermediates."""
    na = np.size(x)
    Z = ofill.fill(model, x, y, ri)
    B = osolve.port_rhs(model.w, na)
    X = osolve.solve(Z, B)
    Y = osolve.admittance(X, model.w, na)
    E = opat.embedded_patterns(model.freq, model.samples, x, y, X, theta, phi)
    return Y, E, Z, X


def objective(Y: np.ndarray, E: np.ndarray, w1: float = 1.0, w2: float = 1.0) -> float:
    """w1 J1 + w2 J2 (the weights let each term be checked on its own)."""
    na = Y.shape[0]
    zin = np.diag(np.linalg.inv(Y))
    j1 = float(np.sum(np.abs(zin - Z_REF) ** 2)) / (na * Z_REF ** 2)
    g = np.mean(np.sum(np.abs(E) ** 2, axis=2), axis=0)               # (n_dir,)
    j2 = float(np.var(g) / np.mean(g) ** 2)
    return w1 * j1 + w2 * j2


def objective_cotangents(Y: np.ndarray, E: np.ndarray, w1: float = 1.0, w2: float = 1.0):
    """(gY, gE) with dJ = Re sum conj(gY) dY + Re sum conj(gE) dE."""
    na = Y.shape[0]
    Yi = np.linalg.inv(Y)
    e = np.diag(Yi) - Z_REF
    c = w1 * 2.0 / (na * Z_REF ** 2)
    # dJ1 = c Re sum_i conj(e_i) dZin_i, dZin_i = -(Yi dY Yi)_ii
    gY = -c * np.conj((Yi @ np.diag(np.conj(e)) @ Yi).T)
    n_ports, n_dir = E.shape[0], E.shape[1]
    g = np.mean(np.sum(np.abs(E) ** 2, axis=2), axis=0)
    gm, g2 = np.mean(g), np.mean(g * g)
    dJ_dg = (2.0 * g / n_dir) / gm ** 2 - 2.0 * g2 / gm ** 3 / n_dir
    gE = (w2 * 2.0 / n_ports) * dJ_dg[None, :, None] * E
    return gY, gE


def fill_vjp(model: Model, x, y, W: np.ndarray, ri: float = 0.0):
    """gx_i = Re sum_ab W_ab dZ_ab/dx_i (and y) for the Eq. (4) fill."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    na, nm = x.size, model.n_mbf
    Wr = np.asarray(W).reshape(na, nm, na, nm)
    mm, nn = np.meshgrid(np.arange(na), np.arange(na), indexing="ij")
    d = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    sel = mm != nn
    if ri > 0.0:
        sel &= d <= ri
    Rx = (x[:, None] - x[None, :])[sel]
    Ry = (y[:, None] - y[None, :])[sel]
    dZx, dZy = eval_model_grad(model, Rx, Ry)                               # (pairs, T, S)
    Wp = Wr[mm[sel], :, nn[sel], :]                                          # (pairs, T, S)
    cx = np.real(np.sum(Wp * dZx, axis=(1, 2)))
    cy = np.real(np.sum(Wp * dZy, axis=(1, 2)))
    # R = p_m - p_n: + for the testing antenna, - for the source antenna
    gx = np.zeros(na)
    gy = np.zeros(na)
    np.add.at(gx, mm[sel], cx)
    np.add.at(gx, nn[sel], -cx)
    np.add.at(gy, mm[sel], cy)
    np.add.at(gy, nn[sel], -cy)
    return gx, gy


def patterns_vjp(model: Model, x, y, X: np.ndarray, theta, phi, gE: np.ndarray):
    """For E[p, d, c] = pref sum_{i,T} F_{T,c}(d) e^{jk u_d . r_i} X[(i,T), p]:
    the cotangent of X (A^H gE) and the explicit position gradient."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    na, nm = x.size, model.n_mbf
    k = em.wavenumber(model.freq)
    u, _, _ = opat.unit_vectors(theta, phi)
    Fth, Fph = opat.mbf_patterns(model.freq, model.samples, theta, phi)     # (D, M)
    Fc = np.stack([Fth, Fph], axis=-1)                                       # (D, M, 2)
    pref = -1j * em.omega_mu(model.freq) / (4.0 * math.pi)
    ph = np.exp(1j * k * (np.outer(u[:, 0], x) + np.outer(u[:, 1], y)))      # (D, Na)
    A = pref * ph[:, :, None, None] * Fc[:, None, :, :]                       # (D, Na, M, 2)
    gX = np.einsum("dimc,pdc->imp", np.conj(A), gE, optimize=True).reshape(na * nm, -1)
    Xr = np.asarray(X).reshape(na, nm, -1)                                   # (i, T, p)
    S = np.einsum("dimc,imp,pdc->di", A, Xr, np.conj(gE), optimize=True)     # (D, Na)
    gx = np.real(np.einsum("di,d->i", 1j * k * S, u[:, 0]))
    gy = np.real(np.einsum("di,d->i", 1j * k * S, u[:, 1]))
    return gX, gx, gy


def gradient(model: Model, x, y, theta, phi, ri: float = 0.0, w1: float = 1.0, w2: float = 1.0):
    """dJ/dx, dJ/dy (float64 [N_a]) by the adjoint method."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    na = x.size
    Y, E, Z, X = response(model, x, y, theta, phi, ri)
    gY, gE = objective_cotangents(Y, E, w1, w2)
    # ports: Y = W^T X  ->  gX = conj(W) gY
    Wp = osolve.port_rhs(model.w, na)
    gX = np.conj(Wp) @ gY
    # patterns
    gXe, gx, gy = patterns_vjp(model, x, y, X, theta, phi, gE)
    gX = gX + gXe
    # adjoint solve and the cotangent of Z: dJ = -Re sum_ab M_ab dZ_ab
    Lam = np.linalg.solve(Z.conj().T, gX)
    M = np.conj(Lam) @ X.T
    fx, fy = fill_vjp(model, x, y, -M, ri)
    return gx + fx, gy + fy
