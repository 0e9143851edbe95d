"""GPU tests of the remaining rows of the path: derivatives (autograd backward), batched
systems, and the full-size N=13000 workload in the launch configuration the benchmark uses."""

import json
import math
import sys
from pathlib import Path

import numpy as np
import pytest

from oracle import brute, omm as oracle
from synth import batched_systems, config_system, perturb_hamiltonian, start_coefficients

pytestmark = pytest.mark.gpu
ROOT = Path(__file__).resolve().parents[1]


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def c5():
    s = config_system("c5", 0)
    return s, start_coefficients(s.S, s.M, 1)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_autograd_backward_c5(torch, c5):
    """dE/dH = rho and dE/dS = -EDM - eta rho through torch.autograd, against the
    eigendecomposition gradient (oracle, LAPACK) and central differences of the GPU minimum."""
    from paper_1312_1549_amd import OMM, omm_energy

    s, C0 = c5
    eta, tau = s.eta, s.tau
    _say(f"autograd c5 N={s.N} M={s.M}")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    H = dev(s.H).requires_grad_(True)
    S = dev(s.S).requires_grad_(True)
    T, C0d = dev(s.T), dev(C0)
    gH_ref, gS_ref = brute.eigen_gradients(s.H, s.S, s.M)

    # FP32 forward with FP64 refinement: gradients of the converged minimum. The derivatives are
    # first order in the error of C, the energy second order: an energy error dE leaves
    # ~sqrt(dE / gap) of unoccupied components in C, and with a gap of 1.3e-3 at the Fermi level
    # a stop at tol 1e-14 (dE ~ 1e-14 |E|) would leave ~1e-5 in the derivatives. tol 1e-15 stops
    # at the FP64 noise floor of the energy.
    solver = OMM(s.N, s.M, precision="fp32", refine=True)
    E = omm_energy(H, S, T, C0d, eta, tau, 1e-15, 6000, solver)
    E.backward()
    gH, gS = H.grad.cpu().numpy(), S.grad.cpu().numpy()
    print(f"refined: rel err dE/dH {_rel(gH, gH_ref):.2e} dE/dS {_rel(gS, gS_ref):.2e} "
          f"after {solver.stats()[0]} line searches")
    assert _rel(gH, gH_ref) < 1e-5 and _rel(gS, gS_ref) < 1e-5

    # FP32 forward alone: gradients at the FP32 minimizer (error set by the 1.3e-3 gap)
    H.grad = None
    S.grad = None
    solver32 = OMM(s.N, s.M, precision="fp32", refine=False)
    E32 = omm_energy(H, S, T, C0d, eta, tau, 1e-9, 5000, solver32)
    E32.backward()
    e1, e2 = _rel(H.grad.cpu().numpy(), gH_ref), _rel(S.grad.cpu().numpy(), gS_ref)
    print(f"fp32 only: rel err dE/dH {e1:.2e} dE/dS {e2:.2e}")
    assert e1 < 5e-2 and e2 < 5e-2

    # central differences (h = 1e-4) of the FP64 minimum along random symmetric directions
    fd_solver = OMM(s.N, s.M, precision="fp64")
    fd_solver.set_HS(s.H, s.S, s.T)
    fd_solver.minimize(C0, eta=eta, tau=tau, tol=1e-14, max_iter=5000)
    Cstar = fd_solver.get_C()
    h = 1e-4
    # Error of each directional derivative relative to the gradient's norm (Z has unit norm, so
    # |<g, Z>| <= |g|): a direction nearly orthogonal to g has a tiny <g, Z>, and relative to that
    # the finite-difference noise of two converged minima (~1e-12 |E| / 2h) is not small.
    scale = {"H": float(np.linalg.norm(gH)), "S": float(np.linalg.norm(gS))}
    worst = 0.0
    for d in range(32):  # unit-Frobenius symmetric directions from seeds 300 .. 331
        Z = np.random.default_rng(300 + d).standard_normal((s.N, s.N))
        Z = np.triu(Z)
        Z = Z + np.triu(Z, 1).T
        Z /= np.linalg.norm(Z)
        for which, g in (("H", gH), ("S", gS)):
            Es = []
            for sign in (1.0, -1.0):
                Hp = s.H + sign * h * Z if which == "H" else s.H
                Sp = s.S + sign * h * Z if which == "S" else s.S
                fd_solver.set_HS(Hp, Sp, s.T)
                fd_solver.minimize(Cstar, eta=eta, tau=tau, tol=1e-15, max_iter=3000)
                Es.append(fd_solver.energy())
            fd = (Es[0] - Es[1]) / (2 * h)
            an = float(np.sum(g * Z))
            print(f"  {which} direction {d}: fd {fd:.10e} analytic {an:.10e}")
            worst = max(worst, abs(fd - an) / scale[which])
    print(f"finite differences: worst error / |g| {worst:.2e}")
    assert worst < 1e-6


def test_batched_systems_match_closed_forms(torch):
    from paper_1312_1549_amd import OMMBatch

    systems = batched_systems(count=4)
    _say("batch " + ",".join(str(x.N) for x in systems))
    b = OMMBatch([x.N for x in systems], [x.M for x in systems])
    C0s = []
    for i, x in enumerate(systems):
        b.set_HS(i, x.H, x.S, x.T)
        C0s.append(start_coefficients(x.S, x.M, 1000 + i))
    st = b.minimize(C0s, [x.eta for x in systems], [x.tau for x in systems], 1e-10, 5000)
    E = b.energies()
    for x, e in zip(systems, E):
        w = brute.generalized_eigh_lapack(x.H, x.S, x.M + 1)[0]
        ref = brute.closed_form_energy(w, x.M, x.eta)
        assert abs(e - ref) <= 1e-5 * abs(ref), (x.N, e, ref)
    # SCF-like warm start: perturbed H, start from the previous C
    it_cold = b.iterations()
    warm = []
    for i, x in enumerate(systems):
        Hp = perturb_hamiltonian(x.H, 200 + i)
        b.set_HS(i, Hp, x.S, x.T)
        warm.append(b.get_C(i))
    b.minimize(warm, [x.eta for x in systems], [x.tau for x in systems], 1e-10, 5000)
    it_warm = b.iterations()
    assert np.all(it_warm < it_cold)


def test_grouped_batch_matches_single_system_runs(torch):
    """The grouped launches (persistent GEMMs over all systems' tiles, hipGraph replays) give
    the energies of independent single-system FP32 runs, and a second call (a new graph)
    reproduces the first."""
    from paper_1312_1549_amd import OMM, OMMBatch

    systems = batched_systems(count=6, first_seed=120)
    _say("grouped batch vs single " + ",".join(str(x.N) for x in systems))
    b = OMMBatch([x.N for x in systems], [x.M for x in systems])
    C0s = [start_coefficients(x.S, x.M, 2000 + i) for i, x in enumerate(systems)]
    for i, x in enumerate(systems):
        b.set_HS(i, x.H, x.S, x.T)
    b.minimize(C0s, [x.eta for x in systems], [x.tau for x in systems], 1e-11, 4000)
    E1, it1 = b.energies(), b.iterations()
    b.minimize(C0s, [x.eta for x in systems], [x.tau for x in systems], 1e-11, 4000)
    E2 = b.energies()
    assert np.array_equal(E1, E2)
    for i, x in enumerate(systems):
        single = OMM(x.N, x.M, precision="fp32", refine=False)
        single.set_HS(x.H, x.S, x.T)
        single.minimize(C0s[i], eta=x.eta, tau=x.tau, tol=1e-11, max_iter=4000)
        assert abs(single.energy() - E1[i]) <= 1e-6 * abs(E1[i])
        w = brute.generalized_eigh_lapack(x.H, x.S, x.M + 1)[0]
        ref = brute.closed_form_energy(w, x.M, x.eta)
        assert abs(E1[i] - ref) <= 1e-5 * abs(ref)


def test_full_size_first_line_searches_match_oracle(torch):
    """N=13000, M=2000: the first line search and the state it leaves (C, SW) against the oracle
    in FP64, then the benchmark's BF16 scheme with the FP64 state in its launch configuration:
    the step against the oracle's element by element, HW and SW after the resynchronization
    against C Hs C^T and C S C^T on sampled rows (any-size properties)."""
    from paper_1312_1549_amd import OMM

    s = config_system("c3", 0)
    C0 = start_coefficients(s.S, s.M, 1)
    _say(f"full size c3 N={s.N} M={s.M} fp64 1 line search")
    dev = {k: torch.from_numpy(v).cuda() for k, v in (("H", s.H), ("S", s.S), ("T", s.T), ("C0", C0))}
    solver = OMM(s.N, s.M, precision="fp64")
    solver.set_HS(dev["H"], dev["S"], dev["T"])
    solver.minimize(dev["C0"], eta=s.eta, tau=s.tau, tol=0.0, max_iter=1)
    tr = solver.energy_trace()
    C = solver.get_C()
    HW, SW = solver.subspace()
    ref = oracle.minimize(s.H, s.S, s.T, C0, s.eta, s.tau, 0.0, 1)
    np.testing.assert_allclose(tr[:2], ref.energies[:2], rtol=1e-11, atol=0)
    assert np.max(np.abs(C - ref.C)) <= 1e-10 * np.max(np.abs(ref.C))
    rows = np.random.default_rng(0).choice(s.M, 16, replace=False)
    SW_rows = (C[rows] @ s.S) @ C.T
    assert np.max(np.abs(SW[rows] - SW_rows)) <= 1e-10 * np.max(np.abs(SW_rows))
    # mixed precision in the same launch shape: energies near the FP64 ones
    bf = OMM(s.N, s.M, precision="bf16x3", refine=False)
    bf.set_HS(dev["H"], dev["S"], dev["T"])
    bf.minimize(dev["C0"], eta=s.eta, tau=s.tau, tol=0.0, max_iter=1)
    tb = bf.energy_trace()
    assert abs(tb[1] - tr[1]) <= 1e-4 * abs(tr[1])
    # the benchmark's scheme (BF16 products on the FP64 state, FP32 G, PG, HD, SD, autotuned
    # stream-K tiles): one line search, which the call closes with an FP64 resynchronization
    _say(f"full size c3 N={s.N} M={s.M} bf16x3 with fp64 state, 1 line search")
    mx = OMM(s.N, s.M, precision="bf16x3", refine=True)
    mx.set_HS(dev["H"], dev["S"], dev["T"])
    mx.minimize(dev["C0"], eta=s.eta, tau=s.tau, tol=0.0, max_iter=1)
    tm = mx.energy_trace()
    Cm = mx.get_C()
    HWm, SWm = mx.subspace()
    assert abs(tm[0] - tr[0]) <= 1e-11 * abs(tr[0])  # initial products in FP64
    # D is rounded to bf16 and PG = G~ P~ is the product of the bf16 roundings of G and P, so
    # the step x D follows the FP64 step to a few parts in a thousand (a CPU emulation of exactly
    # those roundings at this size, FP64 arithmetic otherwise, gives 2.4e-3 in Frobenius norm and
    # 4.5e-3 of the largest element; with G unrounded 2.0e-3 and 4.2e-3)
    step_ref, step = ref.C - C0, Cm - C0
    assert np.linalg.norm(step - step_ref) <= 5e-3 * np.linalg.norm(step_ref)
    assert np.max(np.abs(step - step_ref)) <= 1e-2 * np.max(np.abs(step_ref))
    assert tm[1] < tm[0]
    assert abs(tm[1] - ref.energies[1]) <= 1e-3 * abs(tr[0] - ref.energies[1])
    # after the resynchronization HW, SW and the energy are the FP64 functions of the returned C
    Hs = oracle.shifted_hamiltonian(s.H, s.S, s.eta)
    HW_rows = (Cm[rows] @ Hs) @ Cm.T
    SW_rows = (Cm[rows] @ s.S) @ Cm.T
    assert np.max(np.abs(HWm[rows] - HW_rows)) <= 1e-10 * np.max(np.abs(HW_rows))
    assert np.max(np.abs(SWm[rows] - SW_rows)) <= 1e-10 * np.max(np.abs(SW_rows))
    assert abs(mx.energy() - oracle.functional(HWm, SWm)) <= 1e-12 * abs(mx.energy())
    assert abs(tm[1] - mx.energy()) <= 1e-12 * abs(mx.energy())
    ref_E = json.loads((ROOT / "tests" / "golden" / "c3_reference.json").read_text())["E_min"]
    assert tr[1] > ref_E  # variational: never below the closed-form minimum
