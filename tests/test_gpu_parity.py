"""Parity of the HIP path (through the C-ABI) with the CPU oracle and with closed forms.

Every case prints its name, shape and seed before touching the GPU.
"""

import math
import sys

import numpy as np
import pytest

from oracle import brute, omm as oracle
from synth import (config_system, lattice_positions, make_system, perturb_hamiltonian,
                   start_coefficients)

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib_ok():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1312_1549_amd import OMM

    return OMM


@pytest.fixture(scope="module")
def c1():
    s = config_system("c1", 0)
    return s, start_coefficients(s.S, s.M, 1), brute.generalized_eigh_lapack(s.H, s.S)[0]


@pytest.fixture(scope="module")
def ragged():
    # 50 atoms (5x5x2 lattice) x 4 orbitals -> N = 200, M = 37: ragged against 64/128 tiles
    rng = np.random.default_rng(21)
    pos = lattice_positions((5, 5, 2), 2.5)
    pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    s = make_system(pos, 4, 6.0, 37, rng, name="ragged", eta=0.5, tau=10.0, seed=21)
    return s, start_coefficients(s.S, s.M, 22), brute.generalized_eigh_lapack(s.H, s.S)[0]


@pytest.fixture(scope="module")
def c2():
    s = config_system("c2", 0)
    return s, start_coefficients(s.S, s.M, 1), brute.generalized_eigh_lapack(s.H, s.S, s.M + 1)[0]


def _run(OMM, s, C0, eta, tau, tol, max_iter, precision="fp64", refine=True):
    solver = OMM(s.N, s.M, precision=precision, refine=refine)
    solver.set_HS(s.H, s.S, s.T)
    status = solver.minimize(C0, eta=eta, tau=tau, tol=tol, max_iter=max_iter)
    return solver, status


@pytest.mark.parametrize("tau", [10.0, math.inf, 0.0])
def test_fp64_c1_matches_oracle_and_closed_form(lib_ok, c1, tau):
    s, C0, w = c1
    eta = 0.5
    _say(f"fp64 c1 N={s.N} M={s.M} eta={eta} tau={tau} seed=0/1")
    solver, status = _run(lib_ok, s, C0, eta, tau, 1e-14, 5000)
    assert status == 0
    E = solver.energy()
    E_ref = brute.closed_form_energy(w, s.M, eta)
    assert abs(E - E_ref) <= 1e-10 * abs(E_ref)
    ref = oracle.minimize(s.H, s.S, s.T, C0, eta, tau, 1e-14, 5000)
    tr = solver.energy_trace()
    n = min(30, len(tr), len(ref.energies))
    np.testing.assert_allclose(tr[:n], ref.energies[:n], rtol=1e-10, atol=0)
    it, _ = solver.stats()
    assert abs(it - ref.iterations) <= max(5, 0.1 * ref.iterations)
    HW, SW = solver.subspace()
    assert np.max(np.abs(SW - np.eye(s.M))) < 1e-4
    # the incremental update of HW, SW (Eq. 16) writes each upper element to its mirror
    assert np.array_equal(HW, HW.T) and np.array_equal(SW, SW.T)
    # outputs: density and energy-density matrices of the GPU's own C, element by element
    C = solver.get_C()
    SW_c = C @ s.S @ C.T
    HW_c = C @ (s.H - eta * s.S) @ C.T
    np.testing.assert_allclose(SW, SW_c, rtol=0, atol=1e-11 * np.max(np.abs(SW_c)))
    np.testing.assert_allclose(HW, HW_c, rtol=0, atol=1e-11 * np.max(np.abs(HW_c)))
    rho = solver.density()
    edm = solver.edm()
    np.testing.assert_allclose(rho, oracle.density(C, SW_c), rtol=0, atol=1e-12 * np.abs(rho).max())
    np.testing.assert_allclose(edm, oracle.energy_density(C, HW_c), rtol=0,
                               atol=1e-12 * np.abs(edm).max())
    # density of the minimum is unique (gap > 0): compare with the eigenvector projector
    gH, _ = brute.eigen_gradients(s.H, s.S, s.M)
    assert np.linalg.norm(rho - gH) < 1e-5 * np.linalg.norm(gH)


def test_fp64_eta_below_occupied_level(lib_ok, c1):
    s, C0, w = c1
    _say(f"fp64 c1 eta=0 regime N={s.N} M={s.M}")
    solver, status = _run(lib_ok, s, C0, 0.0, 10.0, 1e-14, 5000)
    E_ref = brute.closed_form_energy(w, s.M, 0.0)
    assert abs(solver.energy() - E_ref) <= 1e-9 * abs(E_ref)
    _, SW = solver.subspace()
    ev = np.linalg.eigvalsh(SW)
    assert np.sum(ev > 0.5) == int(np.sum(w[: s.M] < 0.0))


def test_fp64_ragged_shapes(lib_ok, ragged):
    s, C0, w = ragged
    _say(f"fp64 ragged N={s.N} M={s.M} seed=21/22")
    solver, status = _run(lib_ok, s, C0, 0.5, 10.0, 1e-14, 5000)
    E_ref = brute.closed_form_energy(w, s.M, 0.5)
    assert abs(solver.energy() - E_ref) <= 1e-10 * abs(E_ref)
    ref = oracle.minimize(s.H, s.S, s.T, C0, 0.5, 10.0, 1e-14, 40)
    tr = solver.energy_trace()
    np.testing.assert_allclose(tr[:30], ref.energies[:30], rtol=1e-10, atol=0)


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-11), ("fp32", 1e-5)])
def test_tiny_tile_matches_staged_tile(lib_ok, ragged, c1, precision, rtol, monkeypatch):
    """The one-wave 16 x 16 tile that small FP64 / FP32 products take (N = 128 and N = 200 here:
    every product of the line search, the initial products and the outputs) against the staged
    128 x 128 tile pinned with OMM_TILE=0: the same energies along the trajectory to rounding,
    and for FP64 the same minimum as the closed form."""
    for name, (s, C0, w) in (("c1", c1), ("ragged", ragged)):
        _say(f"tiny vs staged tile {name} N={s.N} M={s.M} {precision}")
        traces = []
        for tile in (None, "0"):
            if tile is None:
                monkeypatch.delenv("OMM_TILE", raising=False)
            else:
                monkeypatch.setenv("OMM_TILE", tile)
            solver, status = _run(lib_ok, s, C0, 0.5, 10.0, 1e-14 if precision == "fp64" else 1e-7,
                                  5000, precision=precision, refine=False)
            traces.append(solver.energy_trace())
            if precision == "fp64":
                E_ref = brute.closed_form_energy(w, s.M, 0.5)
                assert abs(solver.energy() - E_ref) <= 1e-10 * abs(E_ref)
            solver.close()
        n = min(20, len(traces[0]), len(traces[1]))
        np.testing.assert_allclose(traces[0][:n], traces[1][:n], rtol=rtol, atol=0)


@pytest.mark.parametrize("tau", [10.0, math.inf])
def test_preconditioner_matches_inverse(lib_ok, ragged, c1, tau):
    for s, C0, _ in (c1, ragged):
        _say(f"precon N={s.N} tau={tau}")
        solver, _ = _run(lib_ok, s, C0, 0.5, tau, 1e-8, 2)
        P = solver.preconditioner()
        ref = oracle.preconditioner(s.S, s.T, tau)
        np.testing.assert_allclose(P, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_fp64_c2_trajectory_and_minimum(lib_ok, c2):
    s, C0, w = c2
    eta, tau = 0.5, 10.0
    _say(f"fp64 c2 N={s.N} M={s.M} eta={eta} tau={tau}")
    solver, status = _run(lib_ok, s, C0, eta, tau, 1e-14, 3000)
    E_ref = brute.closed_form_energy(w, s.M, eta)
    assert abs(solver.energy() - E_ref) <= 1e-10 * abs(E_ref)
    ref = oracle.minimize(s.H, s.S, s.T, C0, eta, tau, 0.0, 25)
    tr = solver.energy_trace()
    np.testing.assert_allclose(tr[:26], ref.energies[:26], rtol=1e-10, atol=0)
    P = solver.preconditioner()
    k = np.random.default_rng(0).integers(0, s.N, size=(64, 2))
    Pref = np.linalg.inv(s.S + s.T / tau)
    np.testing.assert_allclose(P[k[:, 0], k[:, 1]], Pref[k[:, 0], k[:, 1]], rtol=0,
                               atol=1e-11 * np.abs(Pref).max())


def test_indefinite_preconditioner_is_inverted(lib_ok, c2):
    """Sec. 3.1: P need not be positive definite. At tau = 0.1 the kinetic term dominates and
    S + T/tau of the 2048-orbital lattice has negative eigenvalues (T is indefinite there): the
    blocked Gauss-Jordan sweep with pivoting inside each pivot block still inverts it (LAPACK's
    pivoted LU inverse of the oracle to 1e-10), and the first line searches follow the oracle's."""
    s, C0, w = c2
    tau = 0.1
    ev = np.linalg.eigvalsh(s.S + s.T / tau)
    assert ev[0] < 0 < ev[-1] and np.min(np.abs(ev)) > 1e-3
    _say(f"indefinite preconditioner c2 N={s.N} tau={tau} ({int(np.sum(ev < 0))} negative eigenvalues)")
    solver, _ = _run(lib_ok, s, C0, 0.5, tau, 0.0, 3)
    P = solver.preconditioner()
    ref = oracle.preconditioner(s.S, s.T, tau)
    err = np.max(np.abs(P - ref)) / np.max(np.abs(ref))
    print(f"  max |P - P_ref| / max |P_ref| = {err:.2e}")
    assert err <= 1e-10
    tr = solver.energy_trace()
    ref_run = oracle.minimize(s.H, s.S, s.T, C0, 0.5, tau, 0.0, 3)
    np.testing.assert_allclose(tr, ref_run.energies, rtol=1e-10, atol=0)


def test_singular_preconditioner_is_refused(lib_ok, c2):
    """tau = -mu for the most negative eigenvalue mu of the pencil (T, S) makes S + T/tau
    singular (T v = mu S v): the inverse cannot be formed accurately, and the call fails with
    OMM_E_PRECON instead of running with it."""
    from paper_1312_1549_amd import OMMError

    s, C0, w = c2
    mu = brute.generalized_eigh_lapack(s.T, s.S, 1)[0][0]
    assert mu < 0
    tau = -float(mu)
    _say(f"singular preconditioner c2 N={s.N} tau={tau:.6f}")
    solver = lib_ok(s.N, s.M, precision="fp64")
    solver.set_HS(s.H, s.S, s.T)
    with pytest.raises(OMMError) as e:
        solver.minimize(C0, eta=0.5, tau=tau, tol=0.0, max_iter=2)
    assert e.value.code == -6


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mixed_precision_c2(lib_ok, c2, precision):
    s, C0, w = c2
    eta, tau = 0.5, 10.0
    E_ref = brute.closed_form_energy(w, s.M, eta)
    _say(f"{precision} c2 no refinement")
    solver, status = _run(lib_ok, s, C0, eta, tau, 1e-9, 3000, precision=precision, refine=False)
    err_mixed = abs(solver.energy() - E_ref) / abs(E_ref)
    print(f"{precision}: mixed-only rel err {err_mixed:.3e} iters {solver.stats()[0]}")
    assert err_mixed < 1e-5
    _say(f"{precision} c2 with FP64 refinement")
    solver, status = _run(lib_ok, s, C0, eta, tau, 1e-13, 3000, precision=precision, refine=True)
    err = abs(solver.energy() - E_ref) / abs(E_ref)
    print(f"{precision}+refine: rel err {err:.3e} iters {solver.stats()[0]}")
    assert status == 0 and err < 1e-8
    if precision == "bf16x3":
        # the FP64-exact checkpoints of the scheme decrease to the closed form
        its, Es = solver.checkpoints()
        assert its[0] == 0 and np.all(np.diff(its) > 0)
        assert abs(Es[-1] - E_ref) <= 1e-8 * abs(E_ref)
        assert np.all(Es[1:] >= E_ref - 1e-9 * abs(E_ref))  # variational


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_runs_are_bitwise_reproducible(lib_ok, c2, precision):
    """Fixed-order reductions: two identical runs give identical energies, bit for bit (a read of
    uninitialized or stale device memory would show up here)."""
    s, C0, w = c2
    _say(f"reproducibility {precision} c2")
    traces = []
    for _ in range(2):
        solver, _ = _run(lib_ok, s, C0, 0.5, 10.0, 0.0, 60, precision=precision, refine=True)
        traces.append(solver.energy_trace())
        solver.close()
    assert np.array_equal(traces[0], traces[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_odd_sizes_take_the_unvectorized_paths(lib_ok, precision):
    """N = 33 (11 atoms x 3 orbitals), M = 7: rows of odd length defeat every vector load, so
    the predicated scalar staging paths of all GEMM layouts are exercised."""
    rng = np.random.default_rng(33)
    pos = lattice_positions((3, 2, 2), 2.5, 11)
    pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    s = make_system(pos, 3, 6.0, 7, rng, name="odd", eta=0.5, tau=10.0, seed=33)
    C0 = start_coefficients(s.S, s.M, 34)
    w = brute.generalized_eigh_lapack(s.H, s.S)[0]
    eta = w[s.M] - 0.25 * (w[s.M] - w[s.M - 1])
    _say(f"odd sizes N={s.N} M={s.M} {precision}")
    solver, status = _run(lib_ok, s, C0, eta, 10.0, 1e-13, 5000, precision=precision,
                          refine=precision != "fp32")
    E_ref = brute.closed_form_energy(w, s.M, eta)
    tolr = 1e-5 if precision == "fp32" else 1e-10
    assert abs(solver.energy() - E_ref) <= tolr * abs(E_ref)
    if precision == "fp64":
        ref = oracle.minimize(s.H, s.S, s.T, C0, eta, 10.0, 0.0, 20)
        np.testing.assert_allclose(solver.energy_trace()[:21], ref.energies[:21], rtol=1e-10)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("inputs", ["host", "device"])
def test_new_H_keeps_the_preconditioner_new_S_or_T_rebuilds_it(lib_ok, c1, inputs):
    """SCF reuse (Sec. 3: the next SCF step starts from the previous coefficients): omm_set_HS
    (omm_set_HS_device for device inputs) with a new H but the same S and T keeps
    P = (S + T/tau)^-1 (Sec. 2.4, Eq. 17), which stays readable before the next minimization;
    a new S or T drops it, and the next minimization builds the inverse of the new S + T/tau.
    Every minimum matches its closed form."""
    import torch
    from paper_1312_1549_amd import OMMError

    s, C0, w = c1
    eta, tau = 0.5, 10.0
    _say(f"set_HS reuse of P, c1 fp64, {inputs} inputs")
    solver = lib_ok(s.N, s.M, precision="fp64")
    if inputs == "device":
        set_HS = solver.set_HS
        solver.set_HS = lambda *m: set_HS(*(torch.from_numpy(x).cuda() for x in m))

    def run(H, S, T):
        solver.minimize(C0, eta=eta, tau=tau, tol=1e-14, max_iter=5000)
        wv = brute.generalized_eigh_lapack(H, S)[0]
        E_ref = brute.closed_form_energy(wv, s.M, eta)
        assert abs(solver.energy() - E_ref) <= 1e-10 * abs(E_ref)
        P = solver.preconditioner()
        assert _rel(P, np.linalg.inv(S + T / tau)) < 1e-11
        return P

    solver.set_HS(s.H, s.S, s.T)
    P1 = run(s.H, s.S, s.T)
    H2 = perturb_hamiltonian(s.H, 7)
    solver.set_HS(H2, s.S, s.T)  # same S, T: P kept
    assert np.array_equal(solver.preconditioner(), P1)
    run(H2, s.S, s.T)
    S2 = s.S + 0.05 * np.eye(s.N)
    solver.set_HS(H2, S2, s.T)  # new S: P dropped until the next minimization
    with pytest.raises(OMMError) as e:
        solver.preconditioner()
    assert e.value.code == -2
    run(H2, S2, s.T)
    T2 = 1.1 * s.T
    solver.set_HS(H2, S2, T2)  # new T
    with pytest.raises(OMMError):
        solver.preconditioner()
    run(H2, S2, T2)
    solver.close()


@pytest.mark.parametrize("flavour,sparse", [("cholesky", False), ("dense", True)])
def test_new_H_with_kept_S_data(lib_ok, c2, flavour, sparse):
    """What else derives from S alone survives a new H and must still pair with it: the
    Cholesky factor (H~ = L^-1 Hs L^-T is rebuilt from the new H) and the K-block lists of the
    block-sparse products (the list of Hs is rebuilt: the perturbed H is dense). The minima
    match the closed forms of each (H, S) to 1e-8; then a new S is picked up as well."""
    s, C0, w = c2
    eta, tau = 0.5, 10.0
    _say(f"set_HS reuse flavour={flavour} sparse={sparse} c2")
    solver = lib_ok(s.N, s.M, precision="bf16x3", refine=True, flavour=flavour, sparse=sparse)
    H2 = perturb_hamiltonian(s.H, 8)
    S2 = s.S + 0.05 * np.eye(s.N)
    for H, S in ((s.H, s.S), (H2, s.S), (H2, S2)):
        solver.set_HS(H, S, s.T)
        solver.minimize(C0, eta=eta, tau=tau, tol=1e-13, max_iter=6000)
        wv = brute.generalized_eigh_lapack(H, S, s.M + 1)[0]
        E_ref = brute.closed_form_energy(wv, s.M, eta)
        assert abs(solver.energy() - E_ref) <= 1e-8 * abs(E_ref)
    solver.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("n", [1, 4])
def test_single_wannier_function(lib_ok, precision, n):
    """The smallest problems: one Wannier function (M = 1). Over a single orbital (N = 1, h =
    -0.7, s = 1) the functional is 4c^2 h - 2c^4 h with its minimum 2h at c^2 = 1/s (Secs. 2.1,
    2.2); over 2 atoms x 2 orbitals (N = 4) the minimum is 2 (eps_1 - eta) with eta between the
    two lowest levels. Every product is a single partial tile and K is shorter than one K step."""
    if n == 1:
        H, S, T = np.array([[-0.7]]), np.array([[1.0]]), np.array([[1.5]])
        C0 = np.array([[0.3]])
        eta, E_ref = 0.0, -1.4
    else:
        rng = np.random.default_rng(41)
        pos = lattice_positions((2, 1, 1), 2.5)
        pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
        sy = make_system(pos, 2, 6.0, 1, rng, name="tiny", eta=0.0, tau=10.0, seed=41)
        H, S, T = sy.H, sy.S, sy.T
        C0 = start_coefficients(S, 1, 42)
        w = brute.generalized_eigh_lapack(H, S)[0]
        eta = float(w[1] - 0.25 * (w[1] - w[0]))
        E_ref = brute.closed_form_energy(w, 1, eta)
    _say(f"single WF N={n} M=1 {precision}")
    solver = lib_ok(n, 1, precision=precision, refine=precision != "fp32")
    solver.set_HS(H, S, T)
    status = solver.minimize(C0, eta=eta, tau=10.0, tol=1e-14, max_iter=500)
    assert status == 0
    tolr = 1e-5 if precision == "fp32" else 1e-10
    assert abs(solver.energy() - E_ref) <= tolr * abs(E_ref)
    if precision == "fp64":
        ref = oracle.minimize(H, S, T, C0, eta, 10.0, 0.0, 3)
        np.testing.assert_allclose(solver.energy_trace()[:4], ref.energies[:4], rtol=1e-10)
    solver.close()


@pytest.mark.parametrize("M", [37, 40])
@pytest.mark.parametrize("refine", [True, False])
def test_direct_to_lds_tile_matches_register_tile(lib_ok, M, refine, monkeypatch):
    """The 256 x 256 BF16 tile fed by direct-to-LDS loads (tile 5) sums the same products in the
    same order as the register-staged tile (tile 4): trajectories agree bit for bit. N = 200
    leaves a partial K stage and partial row tiles; M = 40 also takes the gradient (two K
    segments) through the direct loads, M = 37 makes it fall back to the register path."""
    rng = np.random.default_rng(50 + M)
    pos = lattice_positions((5, 5, 2), 2.5)
    pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    s = make_system(pos, 4, 6.0, M, rng, name="dma", eta=0.5, tau=10.0, seed=50 + M)
    C0 = start_coefficients(s.S, s.M, 51)
    _say(f"tile 5 vs tile 4 N={s.N} M={s.M} refine={refine}")
    traces = []
    for tile in ("4", "5"):
        monkeypatch.setenv("OMM_TILE", tile)
        solver, _ = _run(lib_ok, s, C0, 0.5, 10.0, 0.0, 30, precision="bf16x3", refine=refine)
        traces.append(solver.energy_trace())
        solver.close()
    assert len(traces[0]) == 31
    assert np.array_equal(traces[0], traces[1])
    assert traces[1][-1] < traces[1][0]


@pytest.mark.parametrize("M", [37, 40])
def test_stream_k_tile_converges_like_direct_tile(lib_ok, M, monkeypatch):
    """Tile 6 (the direct-to-LDS tile on a stream-K schedule) on a problem far smaller than the
    256 persistent workgroups: every tile is cut into several K parts summed by the fix-up
    kernel. The minimum matches the closed form and the tile-5 run."""
    rng = np.random.default_rng(50 + M)
    pos = lattice_positions((5, 5, 2), 2.5)
    pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    s = make_system(pos, 4, 6.0, M, rng, name="dma", eta=0.5, tau=10.0, seed=50 + M)
    C0 = start_coefficients(s.S, s.M, 51)
    w = brute.generalized_eigh_lapack(s.H, s.S)[0]
    E_ref = brute.closed_form_energy(w, s.M, 0.5)
    _say(f"tile 6 vs tile 5 N={s.N} M={s.M}")
    E = {}
    for tile in ("5", "6"):
        monkeypatch.setenv("OMM_TILE", tile)
        solver, status = _run(lib_ok, s, C0, 0.5, 10.0, 1e-12, 5000, precision="bf16x3",
                              refine=True)
        assert status == 0
        E[tile] = solver.energy()
        solver.close()
    # Trajectories are not compared: the FP32 sums of cut tiles round differently, and a
    # different last bit can flip the bf16 rounding of a direction element, so the paths part
    # at the 1e-5 level within a few line searches while reaching the same minimum.
    # Eq. 18 with tol 1e-12 bounds the last decrease, not the distance to the minimum: a slow
    # final approach can stop a few 1e-10 (relative) above it.
    print(f"rel err tile 5 {(E['5'] - E_ref) / abs(E_ref):.2e} tile 6 {(E['6'] - E_ref) / abs(E_ref):.2e}")
    assert abs(E["5"] - E_ref) <= 1e-9 * abs(E_ref)
    assert abs(E["6"] - E_ref) <= 1e-9 * abs(E_ref)


@pytest.mark.parametrize("tile,refine", [("4", True), ("5", True), ("5", False), ("6", True),
                                         (None, True)])
def test_fused_planes_match_separate_splits(lib_ok, c2, tile, refine, monkeypatch):
    """The bf16 planes written by the GEMM epilogues (G, HD, SD: register tile, direct-to-LDS
    tile, stream-K fix-up, or whatever the autotuner picks) and by the fused update kernel (HC,
    SC and their transposes) equal those of the separate split passes (OMM_FUSE=0): energy
    trajectories and C agree bit for bit."""
    if tile is None:
        s, C0, _ = c2
    else:
        rng = np.random.default_rng(60)
        pos = lattice_positions((5, 5, 2), 2.5)
        pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
        s = make_system(pos, 4, 6.0, 37, rng, name="fuse", eta=0.5, tau=10.0, seed=60)
        C0 = start_coefficients(s.S, s.M, 61)
        monkeypatch.setenv("OMM_TILE", tile)
    _say(f"fused vs separate planes N={s.N} M={s.M} tile={tile} refine={refine}")
    out = []
    for fuse in ("1", "0"):
        monkeypatch.setenv("OMM_FUSE", fuse)
        solver, _ = _run(lib_ok, s, C0, 0.5, 10.0, 0.0, 40, precision="bf16x3", refine=refine)
        out.append((solver.energy_trace(), solver.get_C()))
        solver.close()
    assert len(out[0][0]) == 41
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("tile", ["0", "2", "3"])
def test_symmetric_projections_on_every_tile_shape(lib_ok, c2, tile, monkeypatch):
    """H'' and S'' (Eq. 15) are computed on their upper block triangle and mirrored. With square
    (128 x 128) and non-square (256 x 128, 128 x 256) macro tiles pinned, the FP64 trajectory at
    2048-orbital lattice (M = 384) still follows the oracle's line search for line search."""
    s, C0, _ = c2
    monkeypatch.setenv("OMM_TILE", tile)
    _say(f"symmetric projections, fp64 c2, tile {tile}")
    solver, _ = _run(lib_ok, s, C0, 0.5, 10.0, 0.0, 8)
    ref = oracle.minimize(s.H, s.S, s.T, C0, 0.5, 10.0, 0.0, 8)
    np.testing.assert_allclose(solver.energy_trace(), ref.energies, rtol=1e-11, atol=0)


def test_fully_occupied_limit(lib_ok):
    """M = N: every eigenvector is occupied; with eta above the whole spectrum the minimum is
    2 sum_i (eps_i - eta) and SW = I (C^T C = S^-1 in row form)."""
    rng = np.random.default_rng(40)
    pos = lattice_positions((2, 2, 2), 2.5)
    pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    s = make_system(pos, 4, 6.0, 32, rng, name="full", eta=0.0, tau=10.0, seed=40)
    w = brute.generalized_eigh_lapack(s.H, s.S)[0]
    eta = w[-1] + 1.0
    C0 = start_coefficients(s.S, s.M, 41)
    _say(f"fully occupied N={s.N} M={s.M}")
    solver, status = _run(lib_ok, s, C0, eta, math.inf, 1e-14, 5000)
    E_ref = brute.closed_form_energy(w, s.M, eta)
    assert abs(solver.energy() - E_ref) <= 1e-10 * abs(E_ref)
    C = solver.get_C()
    np.testing.assert_allclose(C.T @ C, np.linalg.inv(s.S), rtol=0, atol=1e-6)


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_graph_replay_matches_eager_launches(lib_ok, c2, precision, monkeypatch):
    """Line searches replayed from the captured hipGraph give the eager trajectory bit for bit
    (many replays, with host synchronizations between them)."""
    s, C0, _ = c2
    _say(f"graph vs eager {precision} c2")
    traces = []
    for flag in ("0", "1"):
        monkeypatch.setenv("OMM_GRAPH", flag)
        solver, _ = _run(lib_ok, s, C0, 0.5, 10.0, 0.0, 90, precision=precision, refine=True)
        traces.append(solver.energy_trace())
        solver.close()
    assert len(traces[0]) == len(traces[1]) == 91
    assert np.array_equal(traces[0], traces[1])
    # the same in chunks: odd chunk lengths change the parity of the captured pair, and every
    # call grows the trace buffer (its reallocation must drop the graph that points at it)
    traces = []
    for flag in ("0", "1"):
        monkeypatch.setenv("OMM_GRAPH", flag)
        solver, _ = _run(lib_ok, s, C0, 0.5, 10.0, 0.0, 7, precision=precision, refine=True)
        for n in (13, 31, 39):
            solver.iterate(n, 0.0)
        traces.append(solver.energy_trace())
        solver.close()
    assert len(traces[0]) == len(traces[1]) == 91
    assert np.array_equal(traces[0], traces[1])


def test_error_paths(lib_ok, c1):
    from paper_1312_1549_amd import OMMError

    s, C0, _ = c1
    _say("error paths")
    solver = lib_ok(s.N, s.M)
    with pytest.raises(OMMError) as e:
        solver.minimize(C0, eta=0.5, tau=10.0)
    assert e.value.code == -2  # no H/S yet
    H = s.H.copy()
    H[0, 1] += 1e-3
    with pytest.raises(OMMError) as e:
        solver.set_HS(H, s.S, s.T)
    assert e.value.code == -9
    H = s.H.copy()
    H[3, 3] = np.nan
    with pytest.raises(OMMError) as e:
        solver.set_HS(H, s.S, s.T)
    assert e.value.code == -5
    solver.set_HS(s.H, s.S, None)
    with pytest.raises(OMMError) as e:
        solver.minimize(C0, eta=0.5, tau=10.0)  # finite tau needs T
    assert e.value.code == -1
    with pytest.raises(OMMError) as e:
        solver.minimize(None, eta=0.5, tau=0.0)  # nothing to resume from
    assert e.value.code == -2
    with pytest.raises(OMMError) as e:
        solver.iterate(3)
    assert e.value.code == -2
    # a start far outside the basin: the line search runs out of minima or diverges
    solver.set_HS(s.H, s.S, s.T)
    big = 30.0 * C0 / np.linalg.norm(C0) * math.sqrt(s.M)
    with pytest.raises(OMMError) as e:
        solver.minimize(big, eta=0.0, tau=0.0, tol=1e-14, max_iter=500)
    assert e.value.code in (-7, -8)


def test_resume_and_iterate(lib_ok, c1):
    s, C0, w = c1
    _say("resume / iterate")
    solver, _ = _run(lib_ok, s, C0, 0.5, 10.0, 0.0, 10)
    e10 = solver.energy_trace()
    st = solver.iterate(10)
    assert st == 1
    e20 = solver.energy_trace()
    ref = oracle.minimize(s.H, s.S, s.T, C0, 0.5, 10.0, 0.0, 20)
    np.testing.assert_allclose(e20[:21], ref.energies[:21], rtol=1e-10, atol=0)
    assert np.array_equal(e10[:11], e20[:11])
    # warm start from the converged C reaches the minimum in a few line searches
    solver.minimize(C0, eta=0.5, tau=10.0, tol=1e-14, max_iter=5000)
    solver.minimize(None, eta=0.5, tau=10.0, tol=1e-12, max_iter=5000)
    assert solver.stats()[0] <= 5


def test_profiling_counts_stages(lib_ok, c1):
    s, C0, _ = c1
    _say("profiling")
    solver, _ = _run(lib_ok, s, C0, 0.5, 10.0, 0.0, 2)
    solver.set_profiling(True)
    solver.iterate(6)
    t, n = solver.stage_times()
    assert n == 6 and all(v >= 0 for v in t.values()) and t["operator_products"] > 0
