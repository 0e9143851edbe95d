"""Finite-range model basis: S, T, H and C0 from a seeded lattice of atoms.

The recipe (all draws from one ``numpy.random.default_rng(seed)`` PCG64 stream, in this order):

1. positions: lattice sites (spacing ``a``) plus i.i.d. U(-0.2, 0.2) jitter per coordinate,
   open boundaries (no periodic images);
2. ``|g|``: an N x N array of U(0.5, 1) draws, then ``sign(g)``: an N x N array of U(0, 1)
   draws mapped to -1 (< 0.5) or +1; only the strict upper triangle is used and mirrored;
3. ``V``: N draws of U(-1, 0), the diagonal local potential.

For orbitals on different atoms at distance r <= r_c (inclusive)
``S_ij = exp(-r/1.5) g_ij``; orbitals on the same atom do not overlap; ``S_ii = 1``.
The diagonal is then shifted by ``s = max(0, 0.1 - lambda_min(S))`` (rounded up to a multiple of
2^-20 so that the result is bit-reproducible), ``T_ij = 0.5 S_ij (3 - r_ij^2/2)`` is built from the
shifted S (so ``T_ii = 1.5 S_ii``), and ``H = T + diag(V)``.

C0 is drawn from its own stream: i.i.d. N(0, sigma^2) with sigma = 0.01, then scaled by
``min(1, 0.5 / (||Z||_2 sqrt(lambda_max(S))))`` (rounded down to a multiple of 2^-12) so that
``lambda_max(C0 S C0^T) <= 0.25``: a start inside the basin of the minimum, because the functional
has no lower bound once a Wannier-function norm passes 1 along a positive-energy direction.

Nothing here computes any part of the minimization: only the model matrices and norms of inputs.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "CONFIGS",
    "System",
    "lattice_positions",
    "make_system",
    "config_system",
    "start_coefficients",
    "perturb_hamiltonian",
    "batched_systems",
    "bloch_system",
    "complex_start_coefficients",
]


@dataclasses.dataclass
class System:
    """One generated problem: FP64 row-major arrays plus the recipe that made them."""

    name: str
    H: np.ndarray  # N x N symmetric
    S: np.ndarray  # N x N symmetric positive definite
    T: np.ndarray  # N x N symmetric (kinetic)
    M: int  # number of Wannier functions
    eta: float
    tau: float
    shift: float  # diagonal shift applied to S
    positions: np.ndarray
    orbitals_per_atom: int
    seed: int

    @property
    def N(self) -> int:
        return self.H.shape[0]


# Workloads (shapes, spacing a, cutoff r_c, orbitals per atom, M, default eta/tau).
CONFIGS: Dict[str, dict] = {
    # 32 atoms on a 4x4x2 lattice, 4 orbitals/atom -> N = 128, M = 24
    "c1": dict(dims=(4, 4, 2), a=2.5, rc=6.0, orbs=4, M=24, eta=0.5, tau=10.0),
    # 512 atoms on 8x8x8 -> N = 2048, M = 384
    "c2": dict(dims=(8, 8, 8), a=2.5, rc=6.0, orbs=4, M=384, eta=0.5, tau=10.0),
    # 1000 atoms on 10x10x10 (a = 3.0, r_c = 8), 13 orbitals/atom -> N = 13000, M = 2000
    "c3": dict(dims=(10, 10, 10), a=3.0, rc=8.0, orbs=13, M=2000, eta=0.0, tau=10.0),
    # 1024 atoms on 16x8x8 -> N = 4096, M = 768
    "c5": dict(dims=(16, 8, 8), a=2.5, rc=6.0, orbs=4, M=768, eta=0.5, tau=10.0),
}

_SHIFT_QUANTUM = 2.0 ** -20
_SCALE_QUANTUM = 2.0 ** -12


def lattice_positions(dims: Sequence[int], a: float, n_atoms: Optional[int] = None) -> np.ndarray:
    """Simple-cubic lattice sites, x index fastest; the first ``n_atoms`` sites if given."""
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz)
    pos = np.stack([idx % nx, (idx // nx) % ny, idx // (nx * ny)], axis=1).astype(np.float64) * a
    if n_atoms is not None:
        pos = pos[:n_atoms]
    return pos


def near_cubic_dims(n_atoms: int) -> Tuple[int, int, int]:
    """Smallest near-cubic box (k, k, k) shrunk one axis at a time while it still holds n_atoms."""
    k = 1
    while k ** 3 < n_atoms:
        k += 1
    dims = [k, k, k]
    for ax in (2, 1, 0):
        if (dims[0] * dims[1] * dims[2]) // dims[ax] * (dims[ax] - 1) >= n_atoms:
            dims[ax] -= 1
    return tuple(dims)  # type: ignore[return-value]


def _lambda_extreme(S: np.ndarray, which: str) -> float:
    """Smallest ('SA') or largest ('LA') eigenvalue of a symmetric matrix, in FP64."""
    n = S.shape[0]
    if n <= 4096:
        w = np.linalg.eigvalsh(S)
        return float(w[0] if which == "SA" else w[-1])
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    A = sp.csr_matrix(S)
    v0 = np.ones(n) / math.sqrt(n)
    w = sla.eigsh(A, k=1, which=which, v0=v0, tol=0.0, ncv=64, maxiter=20000, return_eigenvectors=False)
    return float(w[0])


def make_system(
    positions: np.ndarray,
    orbs: int,
    rc: float,
    M: int,
    rng: np.random.Generator,
    *,
    name: str = "custom",
    eta: float = 0.0,
    tau: float = 10.0,
    seed: int = -1,
) -> System:
    """Build S, T, H for the given atom positions (jitter already applied), drawing g and V."""
    n_atoms = positions.shape[0]
    N = n_atoms * orbs
    if not (0 < M <= N):
        raise ValueError(f"need 0 < M <= N, got M={M}, N={N}")

    g_abs = rng.uniform(0.5, 1.0, size=(N, N))
    g_sign = np.where(rng.random(size=(N, N)) < 0.5, -1.0, 1.0)
    V = rng.uniform(-1.0, 0.0, size=N)

    diff = positions[:, None, :] - positions[None, :, :]
    r_atom = np.sqrt(np.einsum("ijk,ijk->ij", diff, diff))
    atom_of = np.repeat(np.arange(n_atoms), orbs)
    r = r_atom[atom_of][:, atom_of]
    other_atom = atom_of[:, None] != atom_of[None, :]
    within = other_atom & (r <= rc)

    g = g_abs * g_sign
    del g_abs, g_sign
    S = np.where(within, np.exp(-r / 1.5) * g, 0.0)
    del g
    S = np.triu(S, 1)
    S = S + S.T
    np.fill_diagonal(S, 1.0)

    lam_min = _lambda_extreme(S, "SA")
    shift = 0.0
    if lam_min < 0.1:
        shift = math.ceil((0.1 - lam_min) / _SHIFT_QUANTUM) * _SHIFT_QUANTUM
    S[np.diag_indices(N)] += shift

    T = 0.5 * S * (3.0 - 0.5 * r * r)
    T = np.where(within, T, 0.0)
    T = np.triu(T, 1)
    T = T + T.T
    T[np.diag_indices(N)] = 1.5 * np.diag(S)
    del r, within, other_atom

    H = T.copy()
    H[np.diag_indices(N)] += V
    return System(name=name, H=H, S=S, T=T, M=M, eta=eta, tau=tau, shift=shift,
                  positions=positions, orbitals_per_atom=orbs, seed=seed)


def config_system(name: str, seed: int = 0) -> System:
    """One of the named workloads (``c1``, ``c2``, ``c3``, ``c5``) from generator seed ``seed``."""
    cfg = CONFIGS[name]
    rng = np.random.default_rng(seed)
    pos = lattice_positions(cfg["dims"], cfg["a"])
    pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    return make_system(pos, cfg["orbs"], cfg["rc"], cfg["M"], rng, name=name,
                       eta=cfg["eta"], tau=cfg["tau"], seed=seed)


def start_coefficients(S: np.ndarray, M: int, seed: int, sigma: float = 0.01,
                       target: float = 0.25) -> np.ndarray:
    """Random M x N start C0 = sigma Z, scaled so that ||Z sigma||_2^2 lambda_max(S) <= target."""
    N = S.shape[0]
    Z = np.random.default_rng(seed).standard_normal(size=(M, N))
    z2 = float(np.linalg.eigvalsh(Z @ Z.T)[-1]) if M <= N else float(np.linalg.eigvalsh(Z.T @ Z)[-1])
    lam_max = _lambda_extreme(S, "LA")
    bound = sigma * sigma * z2 * lam_max
    scale = 1.0
    if bound > target:
        scale = math.floor(math.sqrt(target / bound) / _SCALE_QUANTUM) * _SCALE_QUANTUM
    return (sigma * scale) * Z


def bloch_system(name: str, k: float, seed: int = 0, M: Optional[int] = None) -> System:
    """Complex Hermitian H(k), S(k), T(k) of a named workload made periodic along x.

    The lattice of ``name`` (with its jitter) is repeated along x with period L = n_x a; every
    orbital pair within r_c, including pairs with images shifted by n L (|n| <= 2), adds its
    real amplitude (the same rule as ``make_system``) times the Bloch phase exp(i k n L). The
    orbital-pair amplitudes are symmetric, so H(k), S(k), T(k) are Hermitian; k = 0 gives real
    matrices with the periodic couplings. The diagonal shift that keeps S(k) positive definite
    is chosen as in ``make_system`` from the smallest eigenvalue of S(k).
    """
    cfg = CONFIGS[name]
    rng = np.random.default_rng(seed)
    pos = lattice_positions(cfg["dims"], cfg["a"])
    pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    orbs, rc = cfg["orbs"], cfg["rc"]
    n_atoms = pos.shape[0]
    N = n_atoms * orbs
    M = cfg["M"] if M is None else M
    L = cfg["dims"][0] * cfg["a"]
    g_abs = rng.uniform(0.5, 1.0, size=(N, N))
    g_sign = np.where(rng.random(size=(N, N)) < 0.5, -1.0, 1.0)
    V = rng.uniform(-1.0, 0.0, size=N)
    g = np.triu(g_abs * g_sign, 1)
    g = g + g.T
    atom_of = np.repeat(np.arange(n_atoms), orbs)
    same_orbital = np.eye(N, dtype=bool)
    S = np.zeros((N, N), dtype=np.complex128)
    T = np.zeros((N, N), dtype=np.complex128)
    for n in range(-2, 3):
        shift_vec = np.array([n * L, 0.0, 0.0])
        diff = pos[:, None, :] - (pos[None, :, :] + shift_vec)
        r_atom = np.sqrt(np.einsum("ijk,ijk->ij", diff, diff))
        r = r_atom[atom_of][:, atom_of]
        if n == 0:
            couple = (atom_of[:, None] != atom_of[None, :]) & (r <= rc)
        else:
            couple = (r <= rc) & ~same_orbital
        phase = np.exp(1j * k * n * L)
        S += np.where(couple, np.exp(-r / 1.5) * g, 0.0) * phase
        T += np.where(couple, 0.5 * np.exp(-r / 1.5) * g * (3.0 - 0.5 * r * r), 0.0) * phase
    S = 0.5 * (S + S.conj().T)
    T = 0.5 * (T + T.conj().T)
    S[np.diag_indices(N)] = 1.0
    lam_min = float(np.linalg.eigvalsh(S)[0])
    shift = 0.0
    if lam_min < 0.1:
        shift = math.ceil((0.1 - lam_min) / _SHIFT_QUANTUM) * _SHIFT_QUANTUM
    S[np.diag_indices(N)] += shift
    T[np.diag_indices(N)] = 1.5 * np.real(np.diag(S))
    H = T.copy()
    H[np.diag_indices(N)] += V
    return System(name=f"{name}-k{k:g}", H=H, S=S, T=T, M=M, eta=cfg["eta"], tau=cfg["tau"],
                  shift=shift, positions=pos, orbitals_per_atom=orbs, seed=seed)


def complex_start_coefficients(S: np.ndarray, M: int, seed: int, sigma: float = 0.01,
                               target: float = 0.25) -> np.ndarray:
    """Complex M x N start sigma (Z1 + i Z2) / sqrt(2), scaled so that
    ||C0||_2^2 lambda_max(S) <= target (S Hermitian)."""
    N = S.shape[0]
    rng = np.random.default_rng(seed)
    Z = (rng.standard_normal(size=(M, N)) + 1j * rng.standard_normal(size=(M, N))) / math.sqrt(2.0)
    z2 = float(np.linalg.eigvalsh(Z @ Z.conj().T)[-1])
    lam_max = float(np.linalg.eigvalsh(S)[-1])
    bound = sigma * sigma * z2 * lam_max
    scale = 1.0
    if bound > target:
        scale = math.floor(math.sqrt(target / bound) / _SCALE_QUANTUM) * _SCALE_QUANTUM
    return (sigma * scale) * Z


def perturb_hamiltonian(H: np.ndarray, seed: int, amplitude: float = 1e-3) -> np.ndarray:
    """H + amplitude * sym(Z): upper triangle (with diagonal) i.i.d. N(0,1), mirrored."""
    N = H.shape[0]
    Z = np.random.default_rng(seed).standard_normal(size=(N, N))
    U = np.triu(Z)
    return H + amplitude * (U + np.triu(U, 1).T)


def batched_systems(count: int = 64, first_seed: int = 100, min_atoms: int = 64,
                    max_atoms: int = 512, a: float = 2.5, rc: float = 6.0, orbs: int = 4,
                    eta: float = 0.5, tau: float = 10.0) -> List[System]:
    """Independent systems of uneven size: atoms ~ U{min..max}, near-cubic boxes, M = round(3N/16)."""
    out = []
    for k in range(count):
        seed = first_seed + k
        rng = np.random.default_rng(seed)
        n_atoms = int(rng.integers(min_atoms, max_atoms + 1))
        dims = near_cubic_dims(n_atoms)
        pos = lattice_positions(dims, a, n_atoms)
        pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
        N = n_atoms * orbs
        M = int(round(3 * N / 16))
        out.append(make_system(pos, orbs, rc, M, rng, name=f"batch{k}", eta=eta, tau=tau, seed=seed))
    return out
