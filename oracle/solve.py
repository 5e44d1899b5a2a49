"""Oracle: port excitations, reduced solve and port admittances (test
infrastructure only).

Section I: the reduced MoM system is solved by Gaussian elimination (a direct,
non-iterative solve), with one right-hand side per antenna port; Section II-C:
the induced MBF coefficients c_ij for excitation at each port.

Readings: one port per element, port weights w_T = a_{T,1} (the first sample of
each MBF is the feed), unit port voltages, so B = I_{N_a} (x) w; the port
admittance matrix is Y = W^T X with W = I_{N_a} (x) w (Y_ij = current at port i
for a unit voltage at port j).

The solve itself is LAPACK zgesv (numpy) used as one library step.  A plain
LU with partial pivoting (pivot = first row maximising |Re| + |Im|, the LAPACK
rule) is provided for small systems and pinned against scipy.
"""
from __future__ import annotations

import numpy as np


def port_rhs(w: np.ndarray, n_ant: int) -> np.ndarray:
    """B = I_{N_a} (x) w: column j is w placed on the rows of antenna j."""
    return np.kron(np.eye(n_ant), np.asarray(w).reshape(-1, 1))


def solve(Z: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X = Z^{-1} B by LU with partial pivoting (LAPACK zgesv)."""
    return np.linalg.solve(Z, B)


def admittance(X: np.ndarray, w: np.ndarray, n_ant: int) -> np.ndarray:
    """Y = W^T X."""
    W = port_rhs(w, n_ant)
    return W.T @ X


def lu_partial_pivot(A: np.ndarray):
    """Unblocked Gaussian elimination with partial pivoting, in place on a copy.

    Returns (LU, piv) with LAPACK getrf semantics: row i was swapped with row
    piv[i] (0-based) at step i; L is unit lower (strictly below the diagonal of
    LU), U upper."""
    A = np.array(A, dtype=np.complex128, copy=True)
    n = A.shape[0]
    piv = np.zeros(n, dtype=np.int64)
    for j in range(n):
        col = np.abs(A[j:, j].real) + np.abs(A[j:, j].imag)
        p = j + int(np.argmax(col))          # first maximiser
        piv[j] = p
        if p != j:
            A[[j, p], :] = A[[p, j], :]
        if A[j, j] == 0:
            raise ZeroDivisionError(f"exact zero pivot at column {j}")
        A[j + 1:, j] /= A[j, j]
        A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j, j + 1:])
    return A, piv


def lu_solve(LU: np.ndarray, piv: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve with the factors of lu_partial_pivot: swaps, L, then U."""
    X = np.array(B, dtype=np.complex128, copy=True)
    n = LU.shape[0]
    for i in range(n):
        if piv[i] != i:
            X[[i, piv[i]]] = X[[piv[i], i]]
    for i in range(n):                       # forward, unit diagonal
        X[i + 1:] -= np.outer(LU[i + 1:, i], X[i])
    for i in range(n - 1, -1, -1):           # backward
        X[i] /= LU[i, i]
        X[:i] -= np.outer(LU[:i, i], X[i])
    return X
