"""The allocation-free backward entry point against the allocating one, through the C-ABI: two
calls in a row, the second on a smaller problem, each checked element by element; and the size
limit and flavour errors."""

import ctypes as ct
import math
import sys

import numpy as np
import pytest

from synth import config_system, start_coefficients

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


def _grads(torch, solver, fn, gE):
    n = solver.N
    dH = torch.empty((n, n), dtype=torch.float64, device="cuda")
    dS = torch.empty_like(dH)
    torch.cuda.synchronize()
    r = fn(solver._h, ct.c_double(gE), ct.c_void_p(dH.data_ptr()), ct.c_void_p(dS.data_ptr()))
    torch.cuda.synchronize()
    return r, dH.cpu().numpy(), dS.cpu().numpy()


def test_noalloc_backward_matches_backward(torch):
    from paper_1312_1549_amd import OMM
    from paper_1312_1549_amd._lib import lib

    L = lib()
    # the larger problem first, then a smaller one: the scratch keeps the first call's contents
    # 4096 x 768 takes two chunks of rows (2^21 / 4096 = 512 < 768); 128 x 24 one
    for name, prec, gE in (("c5", "fp64", 1.0), ("c1", "bf16x3", -0.75)):
        s = config_system(name, 0)
        C0 = start_coefficients(s.S, s.M, 1)
        _say(f"noalloc backward {name} N={s.N} M={s.M} {prec}")
        solver = OMM(s.N, s.M, precision=prec, refine=True, use_torch_stream=False)
        solver.set_HS(s.H, s.S, s.T)
        solver.minimize(C0, eta=s.eta, tau=s.tau, tol=0.0, max_iter=30)
        r1, gH1, gS1 = _grads(torch, solver, L.omm_backward_device, gE)
        r2, gH2, gS2 = _grads(torch, solver, L.omm_backward_device_noalloc, gE)
        assert r1 == 0 and r2 == 0, L.omm_last_error(solver._h)
        for got, ref in ((gH2, gH1), (gS2, gS1)):
            err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            print(f"  max |noalloc - backward| / max |backward| = {err:.2e}")
            assert err <= 1e-12
        solver.close()


def test_noalloc_backward_rejects_what_it_cannot_do(torch):
    from paper_1312_1549_amd import OMM
    from paper_1312_1549_amd._lib import lib

    L = lib()
    _say("noalloc backward error paths")
    big = ct.c_void_p()
    # M = 64 rows per chunk need N <= 2^21 / 64 = 32768
    assert L.omm_create(40000, 64, ct.byref(big)) == 0  # allocates nothing yet
    dummy = torch.empty(1, dtype=torch.float64, device="cuda")
    p = ct.c_void_p(dummy.data_ptr())
    q = ct.c_void_p(dummy.data_ptr() + 8)
    assert L.omm_backward_device_noalloc(big, ct.c_double(1.0), p, q) == -1
    assert b"exceeds its scratch" in L.omm_last_error(big)
    L.omm_destroy(big)
    s = config_system("c1", 0)
    solver = OMM(s.N, s.M, precision="fp64", flavour="cholesky", use_torch_stream=False)
    solver.set_HS(s.H, s.S, s.T)
    solver.minimize(start_coefficients(s.S, s.M, 1), eta=s.eta, tau=math.inf, tol=0.0,
                    max_iter=5)
    assert L.omm_backward_device_noalloc(solver._h, ct.c_double(1.0), p, q) == -2
    solver.close()
