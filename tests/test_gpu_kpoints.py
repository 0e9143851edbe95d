"""GPU tests of k-point batches: several complex Hermitian systems (one per Bloch vector k)
minimized together through their real embeddings, against the generalized Hermitian
eigenvalues (closed form of the minimum) and against single-system complex runs."""

import ctypes
import sys

import numpy as np
import pytest
import scipy.linalg

from synth import bloch_system, complex_start_coefficients

pytestmark = pytest.mark.gpu

KS = (0.0, 0.15, 0.3, 0.55)


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1312_1549_amd as p

    return p


def _closed_form(s, eta):
    w = scipy.linalg.eigh(s.H, s.S, eigvals_only=True, subset_by_index=[0, s.M])
    return 2.0 * float(np.sum(np.minimum(w[: s.M] - eta, 0.0)))


def _systems(ks, Ms=None):
    return [bloch_system("c1", k, 0, None if Ms is None else Ms[i]) for i, k in enumerate(ks)]


def test_kpoint_batch_matches_closed_forms_and_single_runs(lib):
    systems = _systems(KS, Ms=(24, 20, 24, 16))
    _say("k-point batch c1 k=" + ",".join(str(k) for k in KS))
    b = lib.OMMBatchComplex([x.N for x in systems], [x.M for x in systems])
    C0s = [complex_start_coefficients(x.S, x.M, 40 + i) for i, x in enumerate(systems)]
    for i, x in enumerate(systems):
        b.set_HS(i, x.H, x.S, x.T)
    etas, taus = [0.5] * len(systems), [10.0] * len(systems)
    b.minimize(C0s, etas, taus, 1e-11, 5000)
    E = b.energies()
    for i, x in enumerate(systems):
        ref = _closed_form(x, 0.5)
        assert abs(E[i] - ref) <= 1e-5 * abs(ref), (KS[i], E[i], ref)
        single = lib.OMMComplex(x.N, x.M, precision="fp32", refine=False)
        single.set_HS(x.H, x.S, x.T)
        single.minimize(C0s[i], eta=0.5, tau=10.0, tol=1e-11, max_iter=5000)
        assert abs(single.energy() - E[i]) <= 1e-6 * abs(E[i]), (KS[i], single.energy(), E[i])
        # the iterates keep the pair structure of the embedding exactly (half-row products)
        Cr = b.get_C(i)
        Mc, Nc = x.M, x.N
        pair = np.concatenate([-Cr[:Mc, Nc:], Cr[:Mc, :Nc]], axis=1)
        assert np.array_equal(Cr[Mc:], pair)
        # the returned Wannier functions are S(k)-orthonormal at the minimum (to FP32 products)
        C = b.get_C_complex(i)
        SW = (C @ x.S) @ C.conj().T
        assert np.abs(SW - np.eye(x.M)).max() < 1e-3


def test_kpoint_batch_warm_start_along_k(lib):
    """Moving every k-point by a small dk and starting from the previous minimizers takes fewer
    line searches than the cold start did (the k-path analogue of an SCF warm start)."""
    systems = _systems(KS)
    _say("k-point batch warm start along k")
    b = lib.OMMBatchComplex([x.N for x in systems], [x.M for x in systems])
    for i, x in enumerate(systems):
        b.set_HS(i, x.H, x.S, x.T)
    C0s = [complex_start_coefficients(x.S, x.M, 60 + i) for i, x in enumerate(systems)]
    etas, taus = [0.5] * len(systems), [10.0] * len(systems)
    b.minimize(C0s, etas, taus, 1e-10, 5000)
    it_cold = b.iterations()
    moved = _systems([k + 0.01 for k in KS])
    warm = []
    for i, x in enumerate(moved):
        warm.append(b.get_C_complex(i))
        b.set_HS(i, x.H, x.S, x.T)
    b.minimize(warm, etas, taus, 1e-10, 5000)
    it_warm = b.iterations()
    E = b.energies()
    for i, x in enumerate(moved):
        ref = _closed_form(x, 0.5)
        assert abs(E[i] - ref) <= 1e-5 * abs(ref)
    print(f"cold {it_cold.tolist()} warm {it_warm.tolist()}")
    assert np.all(it_warm < it_cold)


def test_kpoint_batch_error_paths(lib):
    s = bloch_system("c1", 0.3, 0)
    _say("k-point batch error paths")
    b = lib.OMMBatchComplex([s.N], [s.M])
    H = s.H.copy()
    H[2, 5] += 1e-3j  # no longer Hermitian
    with pytest.raises(lib.OMMError) as e:
        b.set_HS(0, H, s.S, s.T)
    assert e.value.code == -9
    L = b._L
    z = np.zeros((s.N, s.N))
    zp = z.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.omm_batch_set_HS_complex(b._h, 1, zp, None, zp, None, None, None) == -1  # index
    assert L.omm_batch_set_HS_complex(b._h, 0, None, zp, zp, None, None, None) == -1  # no H_re
    real = lib.OMMBatch([s.N], [s.M])
    r = L.omm_batch_set_HS_complex(real._h, 0, zp, None, zp, None, None, None)
    assert r == -2  # OMM_E_STATE: a real batch refuses the complex entry points
