"""Plain complex FP64 CPU oracle of the OMM minimization for Hermitian H, S (k-points).

TEST INFRASTRUCTURE ONLY, like ``oracle.omm``: only ``tests/`` and the benchmark's CPU baseline
may import it, and it shares no code with the library.

The paper writes every equation of Secs. 2.1-2.4 with Hermitian conjugates (complex
coefficients, as at a general k-point); this module takes those forms literally. Row form: the
M x N array ``C`` holds the conjugate transpose of the paper's m x n coefficient matrix (row i is
the conjugated coefficient vector of Wannier function i), so that

* ``HC = C H``, ``SC = C S``, ``HW = HC C^H``, ``SW = SC C^H`` (Eqs. 5-6, Hermitian M x M);
* the functional is 4 Re Tr HW - 2 Re Tr(SW HW) (Eq. 8; both traces are real);
* ``G = 8 HC - 4 HW SC - 4 SW HC`` (Eq. 12) satisfies dE = Re <G, dC> with <A, B> = Tr(A^H B),
  so -G is the steepest-descent direction;
* H' = D HC^H, H'' = D HD^H (Eqs. 14-15) and HW(x) = HW + x (H' + H'^H) + x^2 H'';
* the quartic coefficients of Eq. 13 take real parts of the traces that are not real by
  themselves.

The line minimum, the stopping rule and the Polak-Ribiere reading are those of ``oracle.omm``,
written again here for complex arguments (real parts of the inner products).
"""

from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .omm import Result, converged, line_minimum  # real scalar helpers: same rule, no matrix code

__all__ = [
    "subspace_operators",
    "functional",
    "gradient",
    "projections",
    "quartic_coefficients",
    "polak_ribiere_beta",
    "update_state",
    "minimize",
    "density",
    "inner",
]


def inner(A: np.ndarray, B: np.ndarray) -> float:
    """Re <A, B> = Re Tr(A^H B) = Re sum_ij conj(A_ij) B_ij."""
    return float(np.real(np.vdot(A, B)))


def _re_tr(A: np.ndarray, B: np.ndarray) -> float:
    """Re Tr(A B)."""
    return float(np.real(np.einsum("ij,ji->", A, B)))


def subspace_operators(C, Hs, S):
    """HC = C Hs, SC = C S, HW = HC C^H, SW = SC C^H (Eqs. 5-6, row form)."""
    HC = C @ Hs
    SC = C @ S
    Ch = C.conj().T
    return HC, SC, HC @ Ch, SC @ Ch


def functional(HW, SW) -> float:
    """4 Re Tr HW - 2 Re Tr(SW HW) (Eq. 8)."""
    return 4.0 * float(np.real(np.trace(HW))) - 2.0 * _re_tr(SW, HW)


def gradient(HC, SC, HW, SW):
    """G = 8 HC - 4 HW SC - 4 SW HC (Eq. 12): dE = Re <G, dC>."""
    return 8.0 * HC - 4.0 * HW @ SC - 4.0 * SW @ HC


def projections(D, HC, SC, HD, SD):
    """H' = D HC^H, S' = D SC^H, H'' = D HD^H, S'' = D SD^H (Eqs. 14-15)."""
    return (D @ HC.conj().T, D @ SC.conj().T, D @ HD.conj().T, D @ SD.conj().T)


def quartic_coefficients(HW, SW, H1, S1, H2, S2) -> np.ndarray:
    """alpha_0 .. alpha_4 of E(C + x D) (Eq. 13 with Hermitian conjugates), expanding
    E = 4 Re Tr HW(x) - 2 Re Tr(SW(x) HW(x)) with HW(x) = HW + x (H' + H'^H) + x^2 H''."""
    a0 = 4.0 * float(np.real(np.trace(HW))) - 2.0 * _re_tr(SW, HW)
    a1 = 8.0 * float(np.real(np.trace(H1))) - 4.0 * _re_tr(S1, HW) - 4.0 * _re_tr(SW, H1)
    a2 = (4.0 * float(np.real(np.trace(H2))) - 2.0 * _re_tr(S2, HW) - 2.0 * _re_tr(SW, H2)
          - 4.0 * _re_tr(S1, H1) - 4.0 * _re_tr(S1, H1.conj().T))
    a3 = -4.0 * _re_tr(S2, H1) - 4.0 * _re_tr(S1, H2)
    a4 = -2.0 * _re_tr(S2, H2)
    return np.array([a0, a1, a2, a3, a4], dtype=np.float64)


def polak_ribiere_beta(G, PG, G_prev, PG_prev) -> float:
    """beta = Re <PG_k, G_k - G_{k-1}> / Re <PG_{k-1}, G_{k-1}> (Secs. 2.3-2.4)."""
    num = inner(PG, G - G_prev)
    den = inner(PG_prev, G_prev)
    beta = num / den if den != 0.0 else float("nan")
    return beta if math.isfinite(beta) else 0.0


def update_state(x, C, D, HC, HD, SC, SD, HW, SW, H1, S1, H2, S2):
    """C, HC, SC += x (D, HD, SD); HW += x (H' + H'^H) + x^2 H'' and SW likewise (Eq. 16)."""
    return (C + x * D, HC + x * HD, SC + x * SD,
            HW + x * (H1 + H1.conj().T) + x * x * H2,
            SW + x * (S1 + S1.conj().T) + x * x * S2)


def minimize(H, S, T, C0, eta: float, tau: float, tol: float, max_iter: int) -> Result:
    """CG minimization of Eq. 8 for Hermitian H, S (Secs. 2.1-2.5) with P = (S + T/tau)^-1
    (tau = inf: S^-1; tau <= 0: none)."""
    Hs = H - eta * S
    if not (tau > 0):
        P = None
    elif math.isinf(tau):
        P = np.linalg.inv(S)
    else:
        P = np.linalg.inv(S + T / tau)
    C = np.array(C0, dtype=np.complex128, copy=True)
    HC, SC, HW, SW = subspace_operators(C, Hs, S)
    E = functional(HW, SW)
    energies: List[float] = [E]
    xs: List[float] = []
    betas: List[float] = []
    G_prev = PG_prev = D = None
    status = "max_iter"
    for _ in range(max_iter):
        G = gradient(HC, SC, HW, SW)
        PG = G if P is None else G @ P
        if D is None:
            beta = 0.0
            D = -PG
        else:
            beta = polak_ribiere_beta(G, PG, G_prev, PG_prev)
            D = -PG + beta * D
        HD, SD = D @ Hs, D @ S
        H1, S1, H2, S2 = projections(D, HC, SC, HD, SD)
        x = line_minimum(quartic_coefficients(HW, SW, H1, S1, H2, S2))
        if x is None:
            status = "no_line_min"
            break
        C, HC, SC, HW, SW = update_state(x, C, D, HC, HD, SC, SD, HW, SW, H1, S1, H2, S2)
        E_new = functional(HW, SW)
        energies.append(E_new)
        xs.append(x)
        betas.append(beta)
        done = converged(E_new, E, tol)
        E = E_new
        G_prev, PG_prev = G, PG
        if done:
            status = "converged"
            break
    return Result(E=E, C=C, HW=HW, SW=SW, energies=energies, iterations=len(xs), status=status,
                  xs=xs, betas=betas)


def density(C, SW):
    """rho = 2 C^H (2I - SW) C (N x N Hermitian); at the minimum 2 sum_i c_i c_i^H."""
    M = SW.shape[0]
    return 2.0 * C.conj().T @ (2.0 * np.eye(M) - SW) @ C
