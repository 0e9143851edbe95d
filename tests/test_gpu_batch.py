"""Batched systems at the mixed-precision bar: the FP32 grouped phase followed by the FP64 grouped
phase reaches each system's closed-form minimum 2 sum_{i<=M} min(eps_i - eta, 0) (Secs. 2.1-2.2)
to 1e-8, the FP64-only batch to 1e-10, and an SCF-like warm start (H perturbed, C0 = the previous
minimizer; Sec. 3 reuses the previous step's coefficients) needs fewer line searches in both
phases than the cold start."""

import sys

import numpy as np
import pytest

from oracle import brute
from synth import batched_systems, perturb_hamiltonian, start_coefficients

pytestmark = pytest.mark.gpu


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
def systems():
    # uneven sizes (first seeds 140..145): N from a few hundred to ~2000
    xs = batched_systems(count=6, first_seed=140)
    refs = []
    for x in xs:
        w = brute.generalized_eigh_lapack(x.H, x.S, x.M + 1)[0]
        refs.append(brute.closed_form_energy(w, x.M, x.eta))
    return xs, np.array(refs)


def _errors(E, refs):
    return np.abs(E - refs) / np.abs(refs)


def test_fp32_then_fp64_batch_reaches_closed_forms(torch, systems):
    from paper_1312_1549_amd import OMMBatch

    xs, refs = systems
    _say("batch fp32+fp64 refine N=" + ",".join(str(x.N) for x in xs))
    b = OMMBatch([x.N for x in xs], [x.M for x in xs], precision="fp32", refine=True)
    for i, x in enumerate(xs):
        b.set_HS(i, x.H, x.S, x.T)
    C0s = [start_coefficients(x.S, x.M, 3000 + i) for i, x in enumerate(xs)]
    etas, taus = [x.eta for x in xs], [x.tau for x in xs]
    st = b.minimize(C0s, etas, taus, 1e-13, 5000)
    err = _errors(b.energies(), refs)
    it32, it64 = b.phase_iterations()
    print(f"  status {st}; rel err {np.array2string(err, precision=2)}; fp32 {it32}; fp64 {it64}")
    assert st == 0
    assert np.all(err <= 1e-8)
    assert np.all(it32 > 0) and np.all(it64 > 0)
    assert np.array_equal(b.iterations(), it32 + it64)
    # SCF-like warm start from the previous minimizer after H += 1e-3 sym(N(0,1)); system 0
    # also gets a new S (scaled by 1.001), so its preconditioner is rebuilt while the others
    # keep theirs
    Cs = [b.get_C(i) for i in range(len(xs))]
    refs_w = []
    for i, x in enumerate(xs):
        Hp = perturb_hamiltonian(x.H, 400 + i)
        Sp = x.S * 1.001 if i == 0 else x.S
        b.set_HS(i, Hp, Sp, x.T)
        w = brute.generalized_eigh_lapack(Hp, Sp, x.M + 1)[0]
        refs_w.append(brute.closed_form_energy(w, x.M, x.eta))
    st = b.minimize(Cs, etas, taus, 1e-13, 5000)
    err_w = _errors(b.energies(), np.array(refs_w))
    w32, w64 = b.phase_iterations()
    print(f"  warm: status {st}; rel err {np.array2string(err_w, precision=2)}; fp32 {w32}; "
          f"fp64 {w64}")
    assert st == 0
    assert np.all(err_w <= 1e-8)
    assert np.all(w32 + w64 < it32 + it64)
    b.close()


def test_fp64_batch_matches_closed_forms_and_single_systems(torch, systems):
    from paper_1312_1549_amd import OMM, OMMBatch

    xs, refs = systems
    xs, refs = xs[:3], refs[:3]
    _say("batch fp64 N=" + ",".join(str(x.N) for x in xs))
    b = OMMBatch([x.N for x in xs], [x.M for x in xs], precision="fp64")
    for i, x in enumerate(xs):
        b.set_HS(i, x.H, x.S, x.T)
    C0s = [start_coefficients(x.S, x.M, 3100 + i) for i, x in enumerate(xs)]
    st = b.minimize(C0s, [x.eta for x in xs], [x.tau for x in xs], 1e-14, 6000)
    E = b.energies()
    err = _errors(E, refs)
    it32, it64 = b.phase_iterations()
    print(f"  status {st}; rel err {np.array2string(err, precision=2)}; fp64 line searches {it64}")
    assert st == 0 and np.all(it32 == 0)
    assert np.all(err <= 1e-10)
    # the grouped FP64 minimization is the single-system FP64 minimization
    for i, x in enumerate(xs):
        single = OMM(x.N, x.M, precision="fp64")
        single.set_HS(x.H, x.S, x.T)
        single.minimize(C0s[i], eta=x.eta, tau=x.tau, tol=1e-14, max_iter=6000)
        assert abs(single.energy() - E[i]) <= 1e-10 * abs(E[i])
        single.close()
    b.close()


def test_batch_precision_arguments_are_checked(torch):
    from paper_1312_1549_amd import OMMBatch, OMMError

    xs = batched_systems(count=1, first_seed=150)
    b = OMMBatch([xs[0].N], [xs[0].M])
    with pytest.raises(OMMError) as e:
        b.set_precision("bf16x3", True)
    assert e.value.code == -1
    b.close()


def test_device_inputs_match_host_inputs(torch, systems):
    """omm_batch_set_HS_device: the same systems handed over as CUDA tensors give bit for bit the
    energies and line-search counts of host inputs; device inputs are validated on the device
    (an asymmetric H or a non-finite S is refused), and a refused call leaves the system's
    previous inputs in place."""
    from paper_1312_1549_amd import OMMBatch, OMMError

    xs, refs = systems
    xs, refs = xs[:3], refs[:3]
    _say("batch fp64 device inputs N=" + ",".join(str(x.N) for x in xs))
    C0s = [start_coefficients(x.S, x.M, 3200 + i) for i, x in enumerate(xs)]
    etas, taus = [x.eta for x in xs], [x.tau for x in xs]
    out = []
    for device in (False, True):
        b = OMMBatch([x.N for x in xs], [x.M for x in xs], precision="fp64")
        for i, x in enumerate(xs):
            if device:
                b.set_HS(i, *(torch.from_numpy(m).cuda() for m in (x.H, x.S, x.T)))
            else:
                b.set_HS(i, x.H, x.S, x.T)
        st = b.minimize(C0s, etas, taus, 1e-13, 6000)
        assert st == 0
        out.append((b.energies(), b.iterations()))
        if device:
            x = xs[0]
            Ha = x.H.copy()
            Ha[0, 1] += 1e-3
            with pytest.raises(OMMError) as e:
                b.set_HS(0, *(torch.from_numpy(m).cuda() for m in (Ha, x.S, x.T)))
            assert e.value.code == -9
            Sn = x.S.copy()
            Sn[2, 2] = np.nan
            with pytest.raises(OMMError) as e:
                b.set_HS(0, *(torch.from_numpy(m).cuda() for m in (x.H, Sn, x.T)))
            assert e.value.code == -5
            # the refused calls changed nothing: the same minimum again
            assert b.minimize(C0s, etas, taus, 1e-13, 6000) == 0
            assert np.array_equal(b.energies(), out[1][0])
        b.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.all(_errors(out[1][0], refs) <= 1e-10)
