"""Plain FP64 CPU oracle of the dense OMM conjugate-gradient minimization.

TEST INFRASTRUCTURE ONLY. This module is the slow, obviously correct reference that the HIP path
is checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the library and its Python binding never do, and it shares no code
with them.

Notation is the row form of the paper's equations: the paper's m x n coefficient matrix (one
column per Wannier function) is stored here as an M x N array ``C`` (one row per Wannier
function), which holds the same numbers. With real symmetric H and S:

* ``HC = C H`` and ``SC = C S`` are the rows of the paper's H C and S C (Sec. 2.3 footnote);
* ``HW = C H C^T``, ``SW = C S C^T`` (Sec. 2.1, Eqs. 5-6);
* the gradient of Eq. 12 in row form is ``G = 8 HC - 4 HW SC - 4 SW HC``.

Every function states the passage it follows. Matrix products are NumPy (host BLAS) calls; nothing
is blocked, fused or reordered beyond what the equations write.

Readings of passages that are silent or ambiguous (each also listed in the design notes):

* stopping rule (Sec. 2.5.2, Eq. 18) taken with absolute values: stop when
  ``|2 (E_new - E)| <= tol |E_new + E|``;
* Polak-Ribiere with the preconditioned gradient (Sec. 2.3 cites it, Sec. 2.4 premultiplies G by
  P): ``beta_k = <PG_k, G_k - G_{k-1}> / <PG_{k-1}, G_{k-1}>``, ``D_k = -PG_k + beta_k D_{k-1}``,
  ``D_0 = -PG_0``, no restarts, ``beta = 0`` if the ratio is not finite;
* the line minimum of the quartic (Sec. 2.3, "solved for"): the first local minimum met going
  downhill from x = 0 (rule in ``line_minimum``);
* the returned energy is the shifted functional (Sec. 2.2); the unshifted band energy is
  ``E + 2 M eta`` (two electrons per Wannier function).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "shifted_hamiltonian",
    "preconditioner",
    "subspace_operators",
    "trace_of_product",
    "functional",
    "exact_functional",
    "gradient",
    "projections",
    "quartic_coefficients",
    "quartic",
    "line_minimum",
    "cubic_real_roots",
    "polak_ribiere_beta",
    "update_state",
    "converged",
    "minimize",
    "density",
    "energy_density",
    "energy_gradients",
    "Result",
]

# A quartic coefficient is dropped when |alpha_k| <= NEGLIGIBLE * sum_{j=1..4} |alpha_j|.
NEGLIGIBLE = 1e-14


def shifted_hamiltonian(H: np.ndarray, S: np.ndarray, eta: float) -> np.ndarray:
    """Eigenspectrum shift H -> H - eta S (Sec. 2.2, Eq. 9)."""
    return H - eta * S


def preconditioner(S: np.ndarray, T: Optional[np.ndarray], tau: float) -> Optional[np.ndarray]:
    """Kinetic-energy preconditioner P = (S + T/tau)^-1 (Sec. 2.4, Eq. 17).

    ``tau = +inf`` gives the pure tensorial correction P = S^-1 (Sec. 2.4); ``tau <= 0`` selects
    the unpreconditioned flavour (Sec. 3, "no precon."), returned as ``None`` (P = I).
    """
    if not (tau > 0):
        return None
    if math.isinf(tau):
        return np.linalg.inv(S)
    if T is None:
        raise ValueError("a finite tau needs the kinetic matrix T")
    return np.linalg.inv(S + T / tau)


def subspace_operators(C: np.ndarray, Hs: np.ndarray, S: np.ndarray):
    """HC, SC and the subspace operators HW = C H C^T, SW = C S C^T (Sec. 2.1, Eqs. 5-6)."""
    HC = C @ Hs
    SC = C @ S
    HW = HC @ C.T
    SW = SC @ C.T
    return HC, SC, HW, SW


def trace_of_product(A: np.ndarray, B: np.ndarray) -> float:
    """Tr{A B} = sum_ij A_ij B_ji."""
    return float(np.einsum("ij,ji->", A, B))


def functional(HW: np.ndarray, SW: np.ndarray) -> float:
    """OMM functional 4 Tr{HW} - 2 Tr{SW HW} (Sec. 2.1, Eq. 8)."""
    return 4.0 * float(np.trace(HW)) - 2.0 * trace_of_product(SW, HW)


def exact_functional(HW: np.ndarray, SW: np.ndarray) -> float:
    """Subspace energy 2 Tr{SW^-1 HW} (Sec. 2.1, Eq. 7); equals Eq. 8 where SW = I."""
    return 2.0 * float(np.trace(np.linalg.solve(SW, HW)))


def gradient(HC, SC, HW, SW) -> np.ndarray:
    """Gradient of Eq. 8 with respect to C (Sec. 2.3, Eq. 12), row form."""
    return 8.0 * HC - 4.0 * HW @ SC - 4.0 * SW @ HC


def projections(D, HC, SC, HD, SD):
    """H', S', H'', S'' of Sec. 2.3 (Eqs. 14-15), row form: H' = D (HC)^T, H'' = D (HD)^T."""
    return D @ HC.T, D @ SC.T, D @ HD.T, D @ SD.T


def quartic_coefficients(HW, SW, H1, S1, H2, S2) -> np.ndarray:
    """alpha_0 .. alpha_4 of E(C + x D) (Sec. 2.3, Eq. 13); H1 = H', H2 = H'' and likewise S."""
    tr = trace_of_product
    a0 = 4.0 * float(np.trace(HW)) - 2.0 * tr(SW, HW)
    a1 = 8.0 * float(np.trace(H1)) - 4.0 * tr(S1, HW) - 4.0 * tr(SW, H1)
    a2 = (4.0 * float(np.trace(H2)) - 2.0 * tr(S2, HW) - 2.0 * tr(SW, H2)
          - 4.0 * tr(S1, H1) - 4.0 * tr(S1.T, H1))
    a3 = -4.0 * tr(S2, H1) - 4.0 * tr(S1, H2)
    a4 = -2.0 * tr(S2, H2)
    return np.array([a0, a1, a2, a3, a4], dtype=np.float64)


def quartic(alpha, x: float) -> float:
    """sum_k alpha_k x^k."""
    return float(sum(float(alpha[k]) * x ** k for k in range(5)))


def _dq(alpha, x):
    return alpha[1] + 2.0 * alpha[2] * x + 3.0 * alpha[3] * x * x + 4.0 * alpha[4] * x ** 3


def _d2q(alpha, x):
    return 2.0 * alpha[2] + 6.0 * alpha[3] * x + 12.0 * alpha[4] * x * x


def cubic_real_roots(a: float, b: float, c: float, d: float) -> List[float]:
    """Real roots of a x^3 + b x^2 + c x + d (a != 0): depressed cubic t^3 + p t + q, then
    Cardano's formula for one real root or the trigonometric (Viete) form for three."""
    A, B, Cc = b / a, c / a, d / a
    p = B - A * A / 3.0
    q = 2.0 * A ** 3 / 27.0 - A * B / 3.0 + Cc
    shift = -A / 3.0
    disc = (q / 2.0) ** 2 + (p / 3.0) ** 3
    if disc > 0.0:
        u = np.cbrt(-q / 2.0 - math.copysign(math.sqrt(disc), q))
        t = u - p / (3.0 * u)
        return [float(t + shift)]
    if p == 0.0:
        return [float(shift)]
    m = 2.0 * math.sqrt(-p / 3.0)
    arg = min(1.0, max(-1.0, 3.0 * q / (p * m)))
    phi = math.acos(arg) / 3.0
    return [float(m * math.cos(phi - 2.0 * math.pi * k / 3.0) + shift) for k in range(3)]


def _quadratic_real_roots(a: float, b: float, c: float) -> List[float]:
    disc = b * b - 4.0 * a * c
    if disc < 0.0:
        return []
    s = -0.5 * (b + math.copysign(math.sqrt(disc), b))
    roots = []
    if s != 0.0:
        roots.append(c / s)
    roots.append(s / a)
    return roots


def line_minimum(alpha) -> Optional[float]:
    """Position x of the line minimum of the quartic q(x) = sum_k alpha_k x^k (Sec. 2.3).

    The paper only says the line minimum is "solved for". Because the functional has no lower
    bound once part of the shifted spectrum is positive (Sec. 2.2, footnote), "the" line minimum
    is read as the first local minimum met when going downhill from x = 0:

    * the descent side is x > 0 if a1 < 0 and x < 0 if a1 > 0; a1 = 0 gives x = 0;
    * candidates are the real roots of q'(x) = 4 a4 x^3 + 3 a3 x^2 + 2 a2 x + a1 on the descent
      side with q''(x) > 0, each refined by two Newton steps; a4 (then a3) is dropped when its
      magnitude is at most NEGLIGIBLE times |a1| + |a2| + |a3| + |a4|, and with both dropped the
      only candidate is -a1/(2 a2) when a2 > 0;
    * the candidate of smallest |x| wins; none gives ``None`` (q decreases without bound along
      the descent side).
    """
    a = [float(v) for v in alpha]
    if a[1] == 0.0:
        return 0.0
    side = 1.0 if a[1] < 0.0 else -1.0
    scale = abs(a[1]) + abs(a[2]) + abs(a[3]) + abs(a[4])
    tiny = NEGLIGIBLE * scale
    if abs(a[4]) > tiny:
        roots = cubic_real_roots(4.0 * a[4], 3.0 * a[3], 2.0 * a[2], a[1])
    elif abs(a[3]) > tiny:
        roots = _quadratic_real_roots(3.0 * a[3], 2.0 * a[2], a[1])
    else:
        return -a[1] / (2.0 * a[2]) if a[2] > 0.0 else None
    best = None
    for r in roots:
        for _ in range(2):
            h = _d2q(a, r)
            if h == 0.0:
                break
            step = _dq(a, r) / h
            if not math.isfinite(step):
                break
            r = r - step
        if not math.isfinite(r) or side * r <= 0.0 or not _d2q(a, r) > 0.0:
            continue
        if best is None or abs(r) < abs(best):
            best = r
    return None if best is None else float(best)


def polak_ribiere_beta(G, PG, G_prev, PG_prev) -> float:
    """beta = <PG_k, G_k - G_{k-1}> / <PG_{k-1}, G_{k-1}> (Sec. 2.3 with Sec. 2.4's P)."""
    num = float(np.sum(PG * (G - G_prev)))
    den = float(np.sum(PG_prev * G_prev))
    beta = num / den if den != 0.0 else float("nan")
    return beta if math.isfinite(beta) else 0.0


def update_state(x, C, D, HC, HD, SC, SD, HW, SW, H1, S1, H2, S2):
    """Update after the line search (Sec. 2.3, Eq. 16 and footnote): C, HC, SC += x (D, HD, SD);
    HW += x H' + x H'^T + x^2 H'' and SW likewise."""
    return (C + x * D, HC + x * HD, SC + x * SD,
            HW + x * H1 + x * H1.T + x * x * H2,
            SW + x * S1 + x * S1.T + x * x * S2)


def converged(E_new: float, E_old: float, tol: float) -> bool:
    """Stopping rule of Sec. 2.5.2 (Eq. 18), with absolute values."""
    return abs(2.0 * (E_new - E_old)) <= tol * abs(E_new + E_old)


@dataclass
class Result:
    E: float
    C: np.ndarray
    HW: np.ndarray
    SW: np.ndarray
    energies: List[float]
    iterations: int
    status: str  # "converged" | "max_iter" | "no_line_min"
    xs: List[float] = field(default_factory=list)
    betas: List[float] = field(default_factory=list)


def minimize(H, S, T, C0, eta: float, tau: float, tol: float, max_iter: int,
             P: Optional[np.ndarray] = None, use_given_P: bool = False,
             callback=None) -> Result:
    """CG minimization of Eq. 8 with exact quartic line searches (Secs. 2.1-2.5).

    ``P``/``use_given_P`` let a caller supply the preconditioner (``None`` = identity) instead of
    building it from (S, T, tau). ``callback(k, E)`` (optional) is called after the setup
    (k = 0) and after every line search; it does not change the arithmetic.
    """
    Hs = shifted_hamiltonian(H, S, eta)
    if not use_given_P:
        P = preconditioner(S, T, tau)
    C = np.array(C0, dtype=np.float64, copy=True)
    HC, SC, HW, SW = subspace_operators(C, Hs, S)
    E = functional(HW, SW)
    energies = [E]
    if callback is not None:
        callback(0, E)
    xs: List[float] = []
    betas: List[float] = []
    G_prev = PG_prev = D = None
    status = "max_iter"
    it = 0
    for it in range(1, max_iter + 1):
        G = gradient(HC, SC, HW, SW)
        PG = G if P is None else G @ P
        if D is None:
            beta = 0.0
            D = -PG
        else:
            beta = polak_ribiere_beta(G, PG, G_prev, PG_prev)
            D = -PG + beta * D
        HD = D @ Hs
        SD = D @ S
        H1, S1, H2, S2 = projections(D, HC, SC, HD, SD)
        alpha = quartic_coefficients(HW, SW, H1, S1, H2, S2)
        x = line_minimum(alpha)
        if x is None:
            status = "no_line_min"
            it -= 1
            break
        C, HC, SC, HW, SW = update_state(x, C, D, HC, HD, SC, SD, HW, SW, H1, S1, H2, S2)
        E_new = functional(HW, SW)
        energies.append(E_new)
        xs.append(x)
        betas.append(beta)
        done = converged(E_new, E, tol)
        E = E_new
        if callback is not None:
            callback(len(xs), E)
        G_prev, PG_prev = G, PG
        if done:
            status = "converged"
            break
    return Result(E=E, C=C, HW=HW, SW=SW, energies=energies, iterations=len(xs),
                  status=status, xs=xs, betas=betas)


def density(C: np.ndarray, SW: np.ndarray) -> np.ndarray:
    """rho = 2 C^T (2I - SW) C: the derivative of Eq. 8 with respect to the (shifted) H; at the
    minimum (SW = I) it is the density matrix 2 sum_i c_i c_i^T of Sec. 2.1."""
    M = SW.shape[0]
    return 2.0 * C.T @ (2.0 * np.eye(M) - SW) @ C


def energy_density(C: np.ndarray, HW: np.ndarray) -> np.ndarray:
    """EDM = 2 C^T HW C: minus the derivative of Eq. 8 with respect to S through SW."""
    return 2.0 * C.T @ HW @ C


def energy_gradients(C, HW, SW, eta: float) -> Tuple[np.ndarray, np.ndarray]:
    """(dE/dH, dE/dS) of the shifted functional at fixed C, chained through H - eta S:
    dE/dH = rho, dE/dS = -EDM - eta rho. At the minimum these are the derivatives of the
    minimum energy itself (the minimum is stationary in C)."""
    rho = density(C, SW)
    return rho, -energy_density(C, HW) - eta * rho
