"""GPU parity of complex Hermitian problems (k-points) against the complex oracle, the
generalized Hermitian eigenvalues, and the real path at k = 0."""

import math
import sys

import numpy as np
import pytest
import scipy.linalg

from oracle import omm_complex as oc
from synth import bloch_system, complex_start_coefficients

pytestmark = pytest.mark.gpu


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


def _complex_rows(Creal, Mc, Nc):
    """The complex Wannier functions held in the first Mc rows of the real embedding, and the
    deviation of the second Mc rows from the pair structure [-Im c, Re c]."""
    C = Creal[:Mc, :Nc] + 1j * Creal[:Mc, Nc:]
    pair = np.concatenate([-Creal[:Mc, Nc:], Creal[:Mc, :Nc]], axis=1)
    return C, float(np.abs(Creal[Mc:] - pair).max())


def test_fp64_trajectory_density_and_minimum(lib):
    s = bloch_system("c1", 0.7, 0)
    C0 = complex_start_coefficients(s.S, s.M, 1)
    eta, tau = 0.5, 10.0
    _say(f"complex fp64 c1 k=0.7 N={s.N} M={s.M}")
    solver = lib.OMMComplex(s.N, s.M, precision="fp64")
    solver.set_HS(s.H, s.S, s.T)
    status = solver.minimize(C0, eta=eta, tau=tau, tol=1e-14, max_iter=5000)
    assert status == 0
    ref = oc.minimize(s.H, s.S, s.T, C0, eta, tau, 1e-14, 5000)
    tr = solver.energy_trace()
    n = min(30, len(tr), len(ref.energies))
    np.testing.assert_allclose(tr[:n], ref.energies[:n], rtol=1e-10, atol=0)
    E_ref = _closed_form(s, eta)
    assert abs(solver.energy() - E_ref) <= 1e-10 * abs(E_ref)
    # the real iterates keep the pair structure of the embedding exactly (the second row of each
    # pair of every product is the rotation of the first); the density at the GPU's C
    C, dev = _complex_rows(solver.get_C(), s.M, s.N)
    assert dev == 0.0
    SW = (C @ s.S) @ C.conj().T
    rho_ref = oc.density(C, SW)
    rho = solver.density()
    assert np.abs(rho - rho_ref).max() <= 1e-11 * np.abs(rho_ref).max()


@pytest.mark.parametrize("precision,refine,flavour", [("bf16x3", True, "dense"),
                                                      ("fp32", True, "dense"),
                                                      ("fp64", True, "cholesky"),
                                                      ("bf16x3", True, "cholesky")])
def test_mixed_and_cholesky_reach_the_minimum(lib, precision, refine, flavour):
    s = bloch_system("c2", 1.1, 0)
    C0 = complex_start_coefficients(s.S, s.M, 2)
    eta = 0.5
    _say(f"complex {precision} {flavour} c2 k=1.1 N={s.N} M={s.M}")
    solver = lib.OMMComplex(s.N, s.M, precision=precision, refine=refine, flavour=flavour)
    solver.set_HS(s.H, s.S, s.T)
    solver.minimize(C0, eta=eta, tau=10.0, tol=1e-13, max_iter=6000)
    E_ref = _closed_form(s, eta)
    err = abs(solver.energy() - E_ref) / abs(E_ref)
    print(f"rel err {err:.2e}, line searches {solver.stats()[0]}")
    assert err < 1e-8


def test_k0_equals_the_real_path(lib):
    s = bloch_system("c1", 0.0, 0)
    assert np.abs(s.S.imag).max() == 0.0
    C0 = complex_start_coefficients(s.S, s.M, 3).real.copy()
    _say("complex at k=0 vs real path")
    cs = lib.OMMComplex(s.N, s.M, precision="fp64")
    cs.set_HS(s.H, s.S, s.T)
    cs.minimize(C0, eta=0.5, tau=10.0, tol=0.0, max_iter=40)
    rs = lib.OMM(s.N, s.M, precision="fp64")
    rs.set_HS(s.H.real.copy(), s.S.real.copy(), s.T.real.copy())
    rs.minimize(C0, eta=0.5, tau=10.0, tol=0.0, max_iter=40)
    np.testing.assert_allclose(cs.energy_trace(), rs.energy_trace(), rtol=1e-11, atol=0)


def test_non_hermitian_input_is_refused(lib):
    s = bloch_system("c1", 0.7, 0)
    _say("complex error paths")
    solver = lib.OMMComplex(s.N, s.M)
    H = s.H.copy()
    H[0, 1] += 1e-3j  # breaks H = H^H
    with pytest.raises(lib.OMMError) as e:
        solver.set_HS(H, s.S, s.T)
    assert e.value.code == -9
