"""Synthetic-input recipe: determinism and the structural properties the workloads state."""

import numpy as np
import pytest

from synth import batched_systems, config_system, perturb_hamiltonian, start_coefficients
from synth.generator import near_cubic_dims


def test_deterministic():
    a, b = config_system("c1", 0), config_system("c1", 0)
    assert np.array_equal(a.H, b.H) and np.array_equal(a.S, b.S) and np.array_equal(a.T, b.T)
    assert np.array_equal(start_coefficients(a.S, a.M, 1), start_coefficients(b.S, b.M, 1))
    assert not np.array_equal(config_system("c1", 1).S, a.S)


@pytest.mark.parametrize("name,N,M", [("c1", 128, 24), ("c2", 2048, 384)])
def test_structure(name, N, M):
    s = config_system(name, 0)
    assert s.N == N and s.M == M
    for X in (s.H, s.S, s.T):
        assert np.array_equal(X, X.T)
    assert np.linalg.eigvalsh(s.S)[0] >= 0.1 - 1e-12
    assert np.allclose(np.diag(s.S), 1.0 + s.shift)
    assert np.allclose(np.diag(s.T), 1.5 * np.diag(s.S))
    v = np.diag(s.H - s.T)
    assert np.all(v <= 0.0) and np.all(v >= -1.0)
    assert np.array_equal(s.H - np.diag(np.diag(s.H)), s.T - np.diag(np.diag(s.T)))
    orb = s.orbitals_per_atom
    atom = np.arange(N) // orb
    same = (atom[:, None] == atom[None, :]) & ~np.eye(N, dtype=bool)
    assert np.all(s.S[same] == 0.0)
    pos = s.positions
    r = np.linalg.norm(pos[atom][:, None, :] - pos[atom][None, :, :], axis=-1)
    rc = 6.0
    assert np.all(s.S[(r > rc)] == 0.0)
    off = ~np.eye(N, dtype=bool) & ~same & (r <= rc)
    mag = np.abs(s.S[off]) / np.exp(-r[off] / 1.5)
    assert mag.min() >= 0.5 - 1e-12 and mag.max() <= 1.0 + 1e-12
    # T_ij = 0.5 S_ij (3 - r^2/2) off the diagonal
    assert np.allclose(s.T[off], 0.5 * s.S[off] * (3.0 - 0.5 * r[off] ** 2))


def test_start_is_inside_the_basin():
    s = config_system("c2", 0)
    C0 = start_coefficients(s.S, s.M, 1)
    SW = C0 @ s.S @ C0.T
    assert np.linalg.eigvalsh(SW)[-1] <= 0.25


def test_batched_and_perturbation():
    systems = batched_systems(count=3)
    for k, s in enumerate(systems):
        assert 256 <= s.N <= 2048 and s.N % 4 == 0
        assert s.M == int(round(3 * s.N / 16))
    H2 = perturb_hamiltonian(systems[0].H, 200)
    d = H2 - systems[0].H
    assert np.array_equal(d, d.T) and 1e-4 < np.std(d) < 1e-2
    for n in (64, 100, 512, 343):
        dims = near_cubic_dims(n)
        assert dims[0] * dims[1] * dims[2] >= n
