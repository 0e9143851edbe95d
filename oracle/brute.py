"""Brute-force references that pin the oracle (TEST INFRASTRUCTURE ONLY).

The minimum of the OMM functional is a plain definition (Sec. 2.1 with Sec. 2.2): when the shift
eta lies above the M-th eigenvalue of the pencil (H, S), the minimum of Eq. 8 for the shifted
Hamiltonian is ``2 sum_{i<=M} (eps_i - eta)`` (two electrons per Wannier function, Eq. 7). When
eta lies below some of the lowest M eigenvalues, the stationary-point analysis of Sec. 2.2 gives
Wannier functions that are either eigenvectors with negative shifted eigenvalue or zero, so the
minimum becomes ``2 sum_{i<=M} min(eps_i - eta, 0)``.

This module computes those closed forms from eigenvalues obtained two independent ways: a
self-written Cholesky factorization plus cyclic Jacobi rotations (small N only), and LAPACK's
generalized symmetric eigensolver through SciPy (any N).
"""

from __future__ import annotations

import math
from typing import Tuple

import numpy as np

__all__ = [
    "cholesky_lower",
    "solve_lower",
    "reduce_to_standard",
    "jacobi_eigenvalues",
    "jacobi_eigh",
    "generalized_eigh_bruteforce",
    "generalized_eigh_lapack",
    "closed_form_energy",
    "eigen_gradients",
]


def cholesky_lower(A: np.ndarray) -> np.ndarray:
    """L with A = L L^T, column by column (Cholesky-Banachiewicz)."""
    n = A.shape[0]
    L = np.zeros_like(A, dtype=np.float64)
    for j in range(n):
        d = A[j, j] - float(L[j, :j] @ L[j, :j])
        if d <= 0.0:
            raise np.linalg.LinAlgError("matrix is not positive definite")
        L[j, j] = math.sqrt(d)
        for i in range(j + 1, n):
            L[i, j] = (A[i, j] - float(L[i, :j] @ L[j, :j])) / L[j, j]
    return L


def solve_lower(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X with L X = B by forward substitution, row by row."""
    n = L.shape[0]
    X = np.zeros_like(B, dtype=np.float64)
    for i in range(n):
        X[i] = (B[i] - L[i, :i] @ X[:i]) / L[i, i]
    return X


def reduce_to_standard(A: np.ndarray, S: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """(L^-1 A L^-T, L) for S = L L^T: the standard-form operator with the same eigenvalues."""
    L = cholesky_lower(S)
    Y = solve_lower(L, A)  # L^-1 A
    Z = solve_lower(L, Y.T)  # L^-1 (L^-1 A)^T = L^-1 A L^-T (A symmetric)
    return 0.5 * (Z + Z.T), L


def jacobi_eigh(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Eigenvalues (ascending) and eigenvectors of a symmetric matrix by cyclic Jacobi rotations."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    scale = float(np.linalg.norm(A))
    for _ in range(max_sweeps):
        off = math.sqrt(max(0.0, float(np.sum(A * A) - np.sum(np.diag(A) ** 2))))
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if apq == 0.0:
                    continue
                theta = (A[q, q] - A[p, p]) / (2.0 * apq)
                t = math.copysign(1.0, theta) / (abs(theta) + math.sqrt(theta * theta + 1.0))
                c = 1.0 / math.sqrt(t * t + 1.0)
                s = t * c
                # rotate rows/columns p and q: A <- J^T A J, V <- V J
                ap = A[:, p].copy()
                aq = A[:, q].copy()
                A[:, p] = c * ap - s * aq
                A[:, q] = s * ap + c * aq
                ap = A[p, :].copy()
                aq = A[q, :].copy()
                A[p, :] = c * ap - s * aq
                A[q, :] = s * ap + c * aq
                vp = V[:, p].copy()
                vq = V[:, q].copy()
                V[:, p] = c * vp - s * vq
                V[:, q] = s * vp + c * vq
    w = np.diag(A).copy()
    order = np.argsort(w)
    return w[order], V[:, order]


def jacobi_eigenvalues(A: np.ndarray) -> np.ndarray:
    return jacobi_eigh(A)[0]


def generalized_eigh_bruteforce(H: np.ndarray, S: np.ndarray):
    """Eigenpairs of H c = eps S c (Sec. 2.1, Eq. 1) by Cholesky + Jacobi; c S-normalized."""
    A, L = reduce_to_standard(H, S)
    w, V = jacobi_eigh(A)
    # c = L^-T v: back substitution on the upper-triangular L^T
    n = L.shape[0]
    Cmat = np.zeros_like(V)
    for i in range(n - 1, -1, -1):
        Cmat[i] = (V[i] - L[i + 1:, i] @ Cmat[i + 1:]) / L[i, i]
    return w, Cmat


def generalized_eigh_lapack(H: np.ndarray, S: np.ndarray, count: int = None):
    """Lowest ``count`` eigenpairs of (H, S) from LAPACK's symmetric-definite solver."""
    import scipy.linalg as sl

    if count is None:
        return sl.eigh(H, S)
    return sl.eigh(H, S, subset_by_index=[0, count - 1])


def closed_form_energy(eps: np.ndarray, M: int, eta: float) -> float:
    """Minimum of the shifted Eq. 8: 2 sum_{i<=M} min(eps_i - eta, 0) (Secs. 2.1-2.2)."""
    e = np.sort(np.asarray(eps, dtype=np.float64))[:M] - eta
    return float(2.0 * np.sum(np.minimum(e, 0.0)))


def eigen_gradients(H: np.ndarray, S: np.ndarray, M: int, eigh=generalized_eigh_lapack):
    """Derivatives of E(H, S) = 2 sum_{i<=M} eps_i from first-order perturbation theory:
    dE/dH = 2 sum c_i c_i^T and dE/dS = -2 sum eps_i c_i c_i^T (S-normalized c_i)."""
    w, V = eigh(H, S)
    c = V[:, :M]
    e = w[:M]
    return 2.0 * c @ c.T, -2.0 * (c * e) @ c.T
