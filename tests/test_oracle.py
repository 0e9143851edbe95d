"""Pins of the CPU oracle against facts the paper and the mathematics fix (CPU only).

Each test names what it pins. The oracle is never checked against itself: the references are
closed forms from a self-written eigensolver and LAPACK, finite differences, direct evaluation
of the functional, exact algebraic identities, and brute-force searches on small inputs.
"""

import math

import numpy as np
import pytest

from oracle import brute, omm
from synth import config_system, start_coefficients


@pytest.fixture(scope="module")
def c1():
    s = config_system("c1", 0)
    C0 = start_coefficients(s.S, s.M, 1)
    w = brute.generalized_eigh_lapack(s.H, s.S)[0]
    return s, C0, w


def _rand_sym(rng, n, scale=1.0):
    A = rng.standard_normal((n, n)) * scale
    return 0.5 * (A + A.T)


# ---- the brute-force references themselves ---------------------------------------------------

def test_bruteforce_eigensolver_matches_lapack():
    """Cholesky + cyclic Jacobi (self-written) vs LAPACK on a random definite pencil."""
    rng = np.random.default_rng(5)
    n = 40
    A = rng.standard_normal((n, n))
    S = A @ A.T / n + 0.5 * np.eye(n)
    H = _rand_sym(rng, n)
    w, V = brute.generalized_eigh_bruteforce(H, S)
    w_ref = brute.generalized_eigh_lapack(H, S)[0]
    assert np.max(np.abs(w - w_ref)) < 1e-11 * np.max(np.abs(w_ref))
    # eigenvectors satisfy H c = eps S c and are S-orthonormal
    assert np.max(np.abs(H @ V - S @ V * w)) < 1e-10
    assert np.max(np.abs(V.T @ S @ V - np.eye(n))) < 1e-10


# ---- the minimum (Secs. 2.1-2.2) --------------------------------------------------------------

@pytest.mark.parametrize("tau", [10.0, math.inf, 0.0])
def test_minimum_is_closed_form(c1, tau):
    """eta above eps_M: E_min = 2 sum_{i<=M} (eps_i - eta), with the self-written eigensolver;
    SW -> I at the minimum (Sec. 2.1) and the minimizer spans eigenvectors (Sec. 2.2)."""
    s, C0, _ = c1
    eta = 0.5
    w_bf = brute.generalized_eigh_bruteforce(s.H, s.S)[0]
    assert w_bf[s.M - 1] < eta  # the shift condition of Sec. 2.2 holds
    r = omm.minimize(s.H, s.S, s.T, C0, eta, tau, 1e-14, 5000)
    assert r.status == "converged"
    E_ref = 2.0 * float(np.sum(w_bf[: s.M] - eta))
    assert abs(r.E - E_ref) <= 1e-10 * abs(E_ref)
    assert np.max(np.abs(r.SW - np.eye(s.M))) < 1e-4
    # stationarity in row form: C Hs = HW C S (the rows span generalized eigenvectors)
    Hs = s.H - eta * s.S
    res = r.C @ Hs - r.HW @ r.C @ s.S
    assert np.linalg.norm(res) < 1e-5 * np.linalg.norm(r.C @ Hs)
    # Eq. 7 and Eq. 8 agree at the minimum
    assert abs(omm.exact_functional(r.HW, r.SW) - r.E) < 1e-8 * abs(r.E)
    # the unshifted band energy is E + 2 M eta = 2 sum eps_i
    assert abs(r.E + 2 * s.M * eta - 2 * np.sum(w_bf[: s.M])) < 1e-9 * abs(r.E)


def test_eta_below_occupied_level_gives_zero_wannier_functions(c1):
    """eta below eps_M (Sec. 2.2): the minimum keeps eigenvectors with eps_i < eta and zero WFs,
    E = 2 sum_{i<=M} min(eps_i - eta, 0); SW is a projector of rank #{eps_i < eta}."""
    s, C0, w = c1
    eta = 0.0
    k = int(np.sum(w[: s.M] < eta))
    assert 0 < k < s.M
    r = omm.minimize(s.H, s.S, s.T, C0, eta, 10.0, 1e-14, 5000)
    E_ref = brute.closed_form_energy(w, s.M, eta)
    assert abs(r.E - E_ref) <= 1e-9 * abs(E_ref)
    ev = np.linalg.eigvalsh(r.SW)
    assert np.sum(ev > 0.5) == k
    assert np.max(np.minimum(np.abs(ev), np.abs(ev - 1.0))) < 1e-3


def test_degenerate_fermi_level_still_converges():
    """A planted degeneracy eps_M = eps_{M+1} (Sec. 2.7): the energy is still recovered."""
    rng = np.random.default_rng(11)
    n, M = 60, 12
    A = rng.standard_normal((n, n))
    S = A @ A.T / n + 0.3 * np.eye(n)
    L = np.linalg.cholesky(S)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    X = np.linalg.solve(L.T, Q)  # X^T S X = I
    eps = np.sort(rng.uniform(-2.0, 3.0, n))
    eps[M] = eps[M - 1]  # degenerate at the Fermi level
    H = S @ X @ np.diag(eps) @ X.T @ S
    H = 0.5 * (H + H.T)
    eta = eps[M - 1] + 0.5 * (eps[M + 1] - eps[M - 1])
    C0 = 0.01 * rng.standard_normal((M, n))
    r = omm.minimize(H, S, None, C0, eta, math.inf, 1e-14, 5000)
    E_ref = 2.0 * float(np.sum(eps[:M] - eta))
    assert r.status == "converged"
    assert abs(r.E - E_ref) <= 1e-9 * abs(E_ref)


# ---- the gradient (Eq. 12) --------------------------------------------------------------------

def _fd_gradient_error(s, grad_fn=omm.gradient, eta=0.5, seed=3):
    rng = np.random.default_rng(seed)
    Hs = s.H - eta * s.S
    C = 0.2 * rng.standard_normal((s.M, s.N))
    HC, SC, HW, SW = omm.subspace_operators(C, Hs, s.S)
    G = grad_fn(HC, SC, HW, SW)
    h = 1e-5
    worst = 0.0
    for _ in range(25):
        i, j = int(rng.integers(s.M)), int(rng.integers(s.N))
        Cp, Cm = C.copy(), C.copy()
        Cp[i, j] += h
        Cm[i, j] -= h
        Ep = omm.functional(*omm.subspace_operators(Cp, Hs, s.S)[2:])
        Em = omm.functional(*omm.subspace_operators(Cm, Hs, s.S)[2:])
        fd = (Ep - Em) / (2 * h)
        worst = max(worst, abs(fd - G[i, j]) / (abs(G[i, j]) + 1e-3 * np.max(np.abs(G))))
    return worst


def test_gradient_matches_finite_differences(c1):
    assert _fd_gradient_error(c1[0]) < 1e-6


# ---- the quartic line search (Eqs. 13-16) -----------------------------------------------------

def _quartic_setup(s, seed=4, eta=0.5):
    rng = np.random.default_rng(seed)
    Hs = s.H - eta * s.S
    C = 0.2 * rng.standard_normal((s.M, s.N))
    D = 0.1 * rng.standard_normal((s.M, s.N))
    HC, SC, HW, SW = omm.subspace_operators(C, Hs, s.S)
    HD, SD = D @ Hs, D @ s.S
    H1, S1, H2, S2 = omm.projections(D, HC, SC, HD, SD)
    return Hs, C, D, HC, SC, HW, SW, HD, SD, H1, S1, H2, S2


def _quartic_error(s, coef_fn=omm.quartic_coefficients):
    Hs, C, D, HC, SC, HW, SW, HD, SD, H1, S1, H2, S2 = _quartic_setup(s)
    alpha = coef_fn(HW, SW, H1, S1, H2, S2)
    worst = 0.0
    for x in (-3.0, -1.0, -0.25, 0.0, 0.3, 1.0, 2.5):
        direct = omm.functional(*omm.subspace_operators(C + x * D, Hs, s.S)[2:])
        scale = sum(abs(alpha[k]) * abs(x) ** k for k in range(5))
        worst = max(worst, abs(direct - omm.quartic(alpha, x)) / scale)
    return worst


def test_quartic_coefficients_are_exact(c1):
    """E(C + x D) evaluated from scratch equals sum_k alpha_k x^k (Eq. 13) to rounding."""
    assert _quartic_error(c1[0]) < 1e-12


def test_alpha1_is_the_directional_derivative(c1):
    s = c1[0]
    Hs, C, D, HC, SC, HW, SW, HD, SD, H1, S1, H2, S2 = _quartic_setup(s)
    alpha = omm.quartic_coefficients(HW, SW, H1, S1, H2, S2)
    G = omm.gradient(HC, SC, HW, SW)
    assert abs(alpha[1] - np.sum(G * D)) < 1e-11 * abs(alpha[1])
    assert abs(alpha[0] - omm.functional(HW, SW)) < 1e-13 * abs(alpha[0])


def test_incremental_update_equals_recomputation(c1):
    """Eq. 16 and the Sec. 2.3 footnote: updated HC, SC, HW, SW equal those of C + x D."""
    s = c1[0]
    Hs, C, D, HC, SC, HW, SW, HD, SD, H1, S1, H2, S2 = _quartic_setup(s)
    x = 0.37
    Cn, HCn, SCn, HWn, SWn = omm.update_state(x, C, D, HC, HD, SC, SD, HW, SW, H1, S1, H2, S2)
    ref = omm.subspace_operators(C + x * D, Hs, s.S)
    for got, want in zip((HCn, SCn, HWn, SWn), ref):
        assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def _first_downhill_min_bruteforce(a, span=50.0, steps=200000):
    """Walk downhill from 0 on a fine grid; return the first grid local minimum (refined)."""
    side = 1.0 if a[1] < 0 else -1.0
    xs = side * np.linspace(0.0, span, steps)
    q = a[0] + xs * (a[1] + xs * (a[2] + xs * (a[3] + xs * a[4])))
    up = np.nonzero(np.diff(q) > 0)[0]
    if len(up) == 0:
        return None
    i = int(up[0])
    lo, hi = xs[max(i - 1, 0)], xs[min(i + 1, steps - 1)]
    lo, hi = min(lo, hi), max(lo, hi)
    f = lambda x: a[0] + x * (a[1] + x * (a[2] + x * (a[3] + x * a[4])))
    g = (math.sqrt(5) - 1) / 2
    for _ in range(200):
        c, d = hi - g * (hi - lo), lo + g * (hi - lo)
        if f(c) < f(d):
            hi = d
        else:
            lo = c
    return 0.5 * (lo + hi)


def test_line_minimum_matches_bruteforce_search():
    """The line-minimum rule against a grid walk downhill from x = 0 (random quartics)."""
    rng = np.random.default_rng(7)
    checked = none_cases = 0
    for _ in range(300):
        a = rng.standard_normal(5) * np.array([1.0, 1.0, 1.0, 0.5, 0.2])
        x = omm.line_minimum(a)
        ref = _first_downhill_min_bruteforce(a)
        if ref is None or abs(ref) > 45.0:
            # no minimum within the walk: only acceptable if the quartic is unbounded there
            if x is None:
                none_cases += 1
                assert a[4] < 0 or abs(a[4]) < 1e-12
            continue
        assert x is not None
        assert abs(x - ref) < 1e-6 * max(1.0, abs(ref))
        checked += 1
    assert checked > 150 and none_cases > 5


def test_cubic_roots_against_companion_matrix():
    rng = np.random.default_rng(8)
    for _ in range(200):
        c = rng.standard_normal(4)
        got = sorted(omm.cubic_real_roots(*c))
        ref = np.roots(c)
        ref = sorted(r.real for r in ref if abs(r.imag) < 1e-7 * max(1.0, abs(r)))
        if len(ref) != len(got):  # near-double roots: compare the residual instead
            for r in got:
                assert abs(np.polyval(c, r)) < 1e-6 * np.sum(np.abs(c)) * max(1, abs(r)) ** 3
            continue
        assert np.allclose(got, ref, rtol=1e-6, atol=1e-8)


# ---- preconditioned Polak-Ribiere (Secs. 2.3-2.4) ---------------------------------------------

def _cholesky_equivalence_error(s, C0, iters=40, eta=0.5):
    """S^-1-preconditioned CG vs unpreconditioned CG on the Cholesky-reduced problem (Sec. 2.4:
    the reduced minimization follows the S^-1-preconditioned one exactly)."""
    L = brute.cholesky_lower(s.S)
    Hs = s.H - eta * s.S
    Li = np.linalg.inv(L)
    Ht = Li @ Hs @ Li.T
    Ht = 0.5 * (Ht + Ht.T)
    r1 = omm.minimize(s.H, s.S, None, C0, eta, math.inf, 0.0, iters)
    r2 = omm.minimize(Ht, np.eye(s.N), None, C0 @ L, 0.0, 0.0, 0.0, iters)
    e1, e2 = np.array(r1.energies), np.array(r2.energies)
    n = min(len(e1), len(e2))
    return float(np.max(np.abs(e1[:n] - e2[:n]) / np.abs(e1[:n]))), n


def test_cholesky_reduction_follows_s_inverse_preconditioning(c1):
    s, C0, _ = c1
    err, n = _cholesky_equivalence_error(s, C0)
    assert n > 30
    assert err < 1e-9


# ---- the kinetic-energy preconditioner (Sec. 2.4, Eq. 17) ------------------------------------

def _precon_pin_error(precon_fn=None):
    """Worst relative error of P(S, T, tau) against two facts fixed independently of Eq. 17's
    matrix inverse: (a) Sec. 2.4's limit tau -> infinity, where P becomes S^-1 (LAPACK inverse
    of S alone); (b) the spectral closed form for commuting S = Q diag(s) Q^T and
    T = Q diag(t) Q^T, where P = Q diag(1 / (s_i + t_i / tau)) Q^T, i.e. each kinetic-energy
    eigendirection is damped by tau / (tau s_i + t_i)."""
    fn = precon_fn or omm.preconditioner
    rng = np.random.default_rng(21)
    n = 24
    A = rng.standard_normal((n, n))
    S = A @ A.T / n + 0.5 * np.eye(n)
    T = _rand_sym(rng, n)
    worst = 0.0
    P = fn(S, T, 1e10)
    Si = np.linalg.inv(S)
    worst = max(worst, np.linalg.norm(P - Si) / np.linalg.norm(Si))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = rng.uniform(0.2, 2.0, n)
    t = rng.uniform(0.1, 30.0, n)  # kinetic eigenvalues: positive, spread over two decades
    Sc = (Q * s) @ Q.T
    Tc = (Q * t) @ Q.T
    for tau in (0.5, 3.0, 10.0):
        ref = (Q * (1.0 / (s + t / tau))) @ Q.T
        worst = max(worst, np.linalg.norm(fn(Sc, Tc, tau) - ref) / np.linalg.norm(ref))
    return float(worst)


def test_preconditioner_limit_and_spectral_closed_form():
    """Eq. 17 pinned without re-typing it: the tau = infinity limit of Sec. 2.4 and the
    commuting-pencil closed form; tau = inf and tau <= 0 select S^-1 and no preconditioning."""
    assert _precon_pin_error() < 1e-8
    rng = np.random.default_rng(22)
    A = rng.standard_normal((10, 10))
    S = A @ A.T / 10 + np.eye(10)
    assert np.allclose(omm.preconditioner(S, None, math.inf) @ S, np.eye(10), atol=1e-12)
    assert omm.preconditioner(S, None, 0.0) is None
    assert omm.preconditioner(S, None, -1.0) is None


# ---- stopping rule (Eq. 18) -------------------------------------------------------------------

def test_stopping_rule_uses_magnitudes():
    assert omm.converged(-10.0, -10.0 + 1e-10, 1e-9)
    assert not omm.converged(-10.0, -10.1, 1e-9)
    # positive energies (start of a run) must not stop spuriously
    assert not omm.converged(5.0, 6.0, 1e-9)


# ---- derivatives of the minimum (density and energy-density matrices) -------------------------

def test_energy_derivatives_match_finite_differences_and_eigenvectors(c1):
    s, C0, _ = c1
    eta, tau = 0.5, 10.0
    r = omm.minimize(s.H, s.S, s.T, C0, eta, tau, 1e-15, 5000)
    dH, dS = omm.energy_gradients(r.C, r.HW, r.SW, eta)
    # eigendecomposition: dE/dH = 2 sum c c^T, dE/dS = -2 sum eps c c^T
    gH, gS = brute.eigen_gradients(s.H, s.S, s.M)
    assert np.linalg.norm(dH - gH) < 1e-6 * np.linalg.norm(gH)
    assert np.linalg.norm(dS - gS) < 1e-6 * np.linalg.norm(gS)
    # central differences along random symmetric directions, re-minimizing from the minimum
    rng = np.random.default_rng(12)
    h = 1e-4
    for _ in range(3):
        Z = _rand_sym(rng, s.N)
        Z /= np.linalg.norm(Z)
        for which, g in (("H", dH), ("S", dS)):
            def E_at(sign):
                H = s.H + sign * h * Z if which == "H" else s.H
                S = s.S + sign * h * Z if which == "S" else s.S
                return omm.minimize(H, S, s.T, r.C, eta, tau, 1e-15, 5000).E
            fd = (E_at(1) - E_at(-1)) / (2 * h)
            assert abs(fd - np.sum(g * Z)) < 1e-6 * max(1.0, abs(fd))


# ---- planted mistakes: each pin above must catch a plausible error in the oracle --------------

def test_pins_catch_planted_mistakes(c1):
    s, C0, _ = c1

    def grad_wrong_sign(HC, SC, HW, SW):
        return 8.0 * HC - 4.0 * HW @ SC + 4.0 * SW @ HC

    def grad_half_scale(HC, SC, HW, SW):
        return 4.0 * HC - 2.0 * HW @ SC - 2.0 * SW @ HC

    assert _fd_gradient_error(s, grad_wrong_sign) > 1e-3
    assert _fd_gradient_error(s, grad_half_scale) > 1e-3

    def coef_dropped_term(HW, SW, H1, S1, H2, S2):
        a = omm.quartic_coefficients(HW, SW, H1, S1, H2, S2)
        a[2] += 4.0 * omm.trace_of_product(S1.T, H1)  # drop -4 Tr{S'^T H'}
        return a

    def coef_dropped_cubic_term(HW, SW, H1, S1, H2, S2):
        a = omm.quartic_coefficients(HW, SW, H1, S1, H2, S2)
        a[3] += 4.0 * omm.trace_of_product(S2, H1)  # drop -4 Tr{S'' H'}
        return a

    assert _quartic_error(s, coef_dropped_term) > 1e-6
    assert _quartic_error(s, coef_dropped_cubic_term) > 1e-6

    orig = omm.polak_ribiere_beta
    try:
        # Fletcher-Reeves-like / unpreconditioned numerator: breaks the Sec. 2.4 equivalence
        omm.polak_ribiere_beta = lambda G, PG, Gp, PGp: float(
            np.sum(G * (G - Gp)) / np.sum(Gp * Gp))
        err, _ = _cholesky_equivalence_error(s, C0)
    finally:
        omm.polak_ribiere_beta = orig
    assert err > 1e-6

    # the kinetic matrix scaled by tau instead of 1/tau, or subtracted: Eq. 17 misread
    def precon_tau_times_T(S, T, tau):
        return np.linalg.inv(S + tau * T)

    def precon_minus_T(S, T, tau):
        return np.linalg.inv(S - T / tau)

    assert _precon_pin_error(precon_tau_times_T) > 1e-2
    assert _precon_pin_error(precon_minus_T) > 1e-2
