"""Pins of the complex (Hermitian, k-point) oracle against what the mathematics fixes."""

import math

import numpy as np
import pytest
import scipy.linalg

from oracle import omm as real_oracle
from oracle import omm_complex as oc
from synth import bloch_system, complex_start_coefficients, config_system, start_coefficients


@pytest.fixture(scope="module")
def ck():
    s = bloch_system("c1", 0.7, 0)
    return s, complex_start_coefficients(s.S, s.M, 1)


def _closed_form(s, eta):
    w = scipy.linalg.eigh(s.H, s.S, eigvals_only=True)
    return 2.0 * float(np.sum(np.minimum(w[: s.M] - eta, 0.0))), w


def test_bloch_matrices_are_hermitian_and_complex(ck):
    s, _ = ck
    assert np.abs(s.S.imag).max() > 1e-3  # the phases make the problem genuinely complex
    for X in (s.H, s.S, s.T):
        assert np.array_equal(X, X.conj().T)
    assert np.linalg.eigvalsh(s.S)[0] > 0.0


def test_minimum_matches_generalized_hermitian_eigenvalues(ck):
    s, C0 = ck
    for tau in (10.0, math.inf, 0.0):
        r = oc.minimize(s.H, s.S, s.T, C0, 0.5, tau, 1e-14, 5000)
        E_ref, w = _closed_form(s, 0.5)
        assert r.status == "converged"
        assert abs(r.E - E_ref) <= 1e-10 * abs(E_ref), tau
        # the minimizing subspace is S-orthonormal: SW = I
        assert np.abs(r.SW - np.eye(s.M)).max() < 1e-5


def test_density_at_the_minimum_is_the_eigenvector_density(ck):
    s, C0 = ck
    r = oc.minimize(s.H, s.S, s.T, C0, 0.5, 10.0, 1e-15, 5000)
    w, V = scipy.linalg.eigh(s.H, s.S)
    Vo = V[:, : s.M]  # S-orthonormal eigenvectors (columns)
    rho_ref = 2.0 * Vo @ Vo.conj().T
    rho = oc.density(r.C, r.SW)
    assert np.abs(rho - rho.conj().T).max() < 1e-12
    assert np.linalg.norm(rho - rho_ref) < 1e-5 * np.linalg.norm(rho_ref)


def test_real_inputs_reproduce_the_real_oracle():
    s = config_system("c1", 0)
    C0 = start_coefficients(s.S, s.M, 1)
    r_real = real_oracle.minimize(s.H, s.S, s.T, C0, 0.5, 10.0, 0.0, 25)
    r_cplx = oc.minimize(s.H.astype(complex), s.S.astype(complex), s.T.astype(complex),
                         C0.astype(complex), 0.5, 10.0, 0.0, 25)
    np.testing.assert_allclose(r_cplx.energies, r_real.energies, rtol=1e-12, atol=0)


def test_gradient_is_the_real_directional_derivative(ck):
    """dE = Re <G, dC> along random complex directions (central differences)."""
    s, C0 = ck
    Hs = s.H - 0.5 * s.S
    rng = np.random.default_rng(5)
    HC, SC, HW, SW = oc.subspace_operators(C0, Hs, s.S)
    G = oc.gradient(HC, SC, HW, SW)
    E = lambda C: oc.functional(*oc.subspace_operators(C, Hs, s.S)[2:])
    for _ in range(3):
        Z = rng.standard_normal(C0.shape) + 1j * rng.standard_normal(C0.shape)
        Z /= np.linalg.norm(Z)
        h = 1e-6
        fd = (E(C0 + h * Z) - E(C0 - h * Z)) / (2 * h)
        assert abs(fd - oc.inner(G, Z)) <= 1e-7 * max(1.0, abs(fd))


def test_quartic_is_exact_along_the_line(ck):
    """E(C + x D) equals the quartic of Eq. 13 (Hermitian forms) at several x; alpha_1 = Re<G, D>."""
    s, C0 = ck
    Hs = s.H - 0.5 * s.S
    rng = np.random.default_rng(6)
    D = 0.01 * (rng.standard_normal(C0.shape) + 1j * rng.standard_normal(C0.shape))
    HC, SC, HW, SW = oc.subspace_operators(C0, Hs, s.S)
    H1, S1, H2, S2 = oc.projections(D, HC, SC, D @ Hs, D @ s.S)
    alpha = oc.quartic_coefficients(HW, SW, H1, S1, H2, S2)
    assert abs(alpha[1] - oc.inner(oc.gradient(HC, SC, HW, SW), D)) <= 1e-10 * abs(alpha[1])
    for x in (-1.3, 0.2, 0.7, 2.5):
        direct = oc.functional(*oc.subspace_operators(C0 + x * D, Hs, s.S)[2:])
        assert abs(real_oracle.quartic(alpha, x) - direct) <= 1e-11 * max(1.0, abs(direct))


def test_planted_mistake_transpose_instead_of_conjugate_fails(ck):
    """A projection built with a plain transpose (H' = D HC^T) breaks quartic exactness."""
    s, C0 = ck
    Hs = s.H - 0.5 * s.S
    rng = np.random.default_rng(7)
    D = 0.01 * (rng.standard_normal(C0.shape) + 1j * rng.standard_normal(C0.shape))
    HC, SC, HW, SW = oc.subspace_operators(C0, Hs, s.S)
    HD, SD = D @ Hs, D @ s.S
    wrong = (D @ HC.T, D @ SC.T, D @ HD.T, D @ SD.T)
    alpha = oc.quartic_coefficients(HW, SW, *wrong)
    x = 0.7
    direct = oc.functional(*oc.subspace_operators(C0 + x * D, Hs, s.S)[2:])
    assert abs(real_oracle.quartic(alpha, x) - direct) > 1e-6 * abs(direct)
