"""Helpers shared by the GPU parity tests: error measures and conversion of
oracle models into library model blobs (inputs only; no expected value ever
comes from the GPU path)."""
from __future__ import annotations

import functools
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import em, fill as ofill, fit as ofit
from workloads import workload


def block_eps(Zg: np.ndarray, Zo: np.ndarray, n_mbf: int, offdiag_only: bool = True):
    """Max over blocks of ||dZ_block||_F / ||Zo_block||_F (zero blocks must be
    exactly zero), plus the global relative Frobenius error."""
    n = Zo.shape[0]
    na = n // n_mbf
    D = (Zg - Zo).reshape(na, n_mbf, na, n_mbf)
    O = Zo.reshape(na, n_mbf, na, n_mbf)
    dn = np.sqrt((np.abs(D) ** 2).sum(axis=(1, 3)))
    on = np.sqrt((np.abs(O) ** 2).sum(axis=(1, 3)))
    mask = np.ones((na, na), bool)
    if offdiag_only:
        np.fill_diagonal(mask, False)
    nz = mask & (on > 0)
    zero = mask & (on == 0)
    eps = float((dn[nz] / on[nz]).max()) if nz.any() else 0.0
    zero_ok = bool((dn[zero] == 0).all()) if zero.any() else True
    glob = float(np.linalg.norm(Zg - Zo) / np.linalg.norm(Zo))
    return eps, zero_ok, glob


def oracle_model(freq, elem, P, Q, r_min):
    return ofit.fit(freq, elem.samples, P, Q, r_min, wire_radius=elem.wire_radius)


@functools.lru_cache(maxsize=None)
def oracle_models(cfg: str, wire_radius: float | None = None):
    """Oracle models of a configuration (cached per process)."""
    wl = workload(cfg)
    if wire_radius is not None:
        wl.elem.wire_radius = wire_radius
    return wl, [oracle_model(f, wl.elem, P, wl.Q, wl.r_min) for f, P in zip(wl.freqs, wl.P)]


def pack(api, m, device="cuda"):
    """Oracle model -> library model blob (same numbers, as data)."""
    return api.pack_model(m.C, m.Z_self, m.w, m.samples, m.freq, m.k, em.omega_mu(m.freq),
                          m.r_min, m.wire_radius, device=device)


def colmajor_to_numpy(M) -> np.ndarray:
    """Batched column-major torch view (b, rows, cols) -> numpy (b, rows, cols)."""
    return M.detach().cpu().numpy()


def oracle_fill_chunked(model, x, y, ri: float = 0.0, chunk: int = 32768) -> np.ndarray:
    """The oracle fill (same numbers as oracle.fill.fill) with the model
    evaluated in chunks of pairs, and blocks beyond a radius of influence left
    at zero without evaluating them (bounded memory at n ~ 8192)."""
    na, nm = x.size, model.n_mbf
    Z = np.zeros((na, nm, na, nm), dtype=np.complex128)
    mm, nn = np.meshgrid(np.arange(na), np.arange(na), indexing="ij")
    sel = mm != nn
    if ri > 0.0:
        d = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
        sel &= d <= ri
    Rx, Ry = (x[:, None] - x[None, :])[sel], (y[:, None] - y[None, :])[sel]
    blocks = np.concatenate([ofill.eval_model(model, Rx[i:i + chunk], Ry[i:i + chunk])
                             for i in range(0, Rx.size, chunk)])
    Z[mm[sel], :, nn[sel], :] = blocks
    for m in range(na):
        Z[m, :, m, :] = model.Z_self
    return Z.reshape(na * nm, na * nm)


def oracle_fill_threads(model, x, y, ri: float = 0.0, chunk: int = 8192, workers: int = 8) -> np.ndarray:
    """oracle.fill.fill (the same numbers, entry for entry) with the model
    evaluated on chunks of pairs by a thread pool (numpy releases the GIL in
    its array kernels); a thread pool, not processes, because the test
    process holds a GPU context."""
    from oracle import fill as ofill
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    na, nm = x.size, model.n_mbf
    mm, nn = np.meshgrid(np.arange(na), np.arange(na), indexing="ij")
    sel = mm != nn
    if ri > 0.0:
        sel &= np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :]) <= ri
    Rx, Ry = (x[:, None] - x[None, :])[sel], (y[:, None] - y[None, :])[sel]
    Z = np.zeros((na, nm, na, nm), dtype=np.complex128)
    if Rx.size:
        with ThreadPoolExecutor(workers) as ex:
            parts = list(ex.map(lambda i: ofill.eval_model(model, Rx[i:i + chunk], Ry[i:i + chunk]),
                                range(0, Rx.size, chunk)))
        Z[mm[sel], :, nn[sel], :] = np.concatenate(parts)
    for m in range(na):
        Z[m, :, m, :] = model.Z_self
    return Z.reshape(na * nm, na * nm)
