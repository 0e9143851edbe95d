"""Block-sparse operator products: [HD | SD] = D [Hs | S] over the non-zero 32-deep K blocks of
each 256-column tile only. Skipped blocks contribute exact zeros, so every iterate must equal
the dense run's bit for bit (np.array_equal treats -0 and +0 alike) when both use the same
macro tile and K order: the sparse products always run tile 5 without split-K, and OMM_TILE=5
pins the dense run (and every other BF16 product of both runs) to the same."""

import sys

import numpy as np
import pytest

from oracle import brute
from synth import config_system, lattice_positions, make_system, start_coefficients

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def same_tile(monkeypatch):
    monkeypatch.setenv("OMM_TILE", "5")


@pytest.fixture(scope="module")
def OMM():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1312_1549_amd import OMM

    return OMM


def _pair(OMM, s, C0, eta, tau, iters, refine, H=None, S=None, T=None):
    H = s.H if H is None else H
    S = s.S if S is None else S
    T = s.T if T is None else T
    out = []
    for sparse in (False, True):
        solver = OMM(s.N, s.M, precision="bf16x3", refine=refine, sparse=sparse)
        solver.set_HS(H, S, T)
        solver.minimize(C0, eta=eta, tau=tau, tol=0.0, max_iter=iters)
        out.append((solver.energy_trace(), solver.get_C(), solver))
    return out


@pytest.mark.parametrize("refine", [True, False])
def test_c2_sparse_equals_dense(OMM, refine):
    s = config_system("c2", 0)
    C0 = start_coefficients(s.S, s.M, 1)
    _say(f"sparse vs dense c2 refine={refine}")
    (t0, C_0, _), (t1, C_1, sp) = _pair(OMM, s, C0, 0.5, 10.0, 100, refine)
    dens = sp.sparse_density()
    print(f"K-block density Hs {dens[0]:.3f} S {dens[1]:.3f}")
    assert 0.0 < dens[0] < 1.0 and 0.0 < dens[1] < 1.0
    assert len(t0) == len(t1) == 101
    print("max rel diff", float(np.max(np.abs(t0 - t1) / np.abs(t0))))
    assert np.array_equal(t0, t1)
    assert np.array_equal(C_0, C_1)


@pytest.mark.parametrize("M", [37, 40])
def test_ragged_sparse_equals_dense(OMM, M):
    """N = 200: a partial last K block, partial column and row tiles; then convergence to the
    closed form with the sparse products."""
    rng = np.random.default_rng(60 + M)
    pos = lattice_positions((5, 5, 2), 2.5)
    pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    s = make_system(pos, 4, 6.0, M, rng, name="sparse", eta=0.5, tau=10.0, seed=60 + M)
    C0 = start_coefficients(s.S, s.M, 61)
    _say(f"sparse vs dense ragged N={s.N} M={s.M}")
    (t0, _, _), (t1, _, sp) = _pair(OMM, s, C0, 0.5, 10.0, 60, True)
    assert np.array_equal(t0, t1)
    w = brute.generalized_eigh_lapack(s.H, s.S)[0]
    E_ref = brute.closed_form_energy(w, s.M, 0.5)
    sp.minimize(None, eta=0.5, tau=10.0, tol=1e-13, max_iter=4000)
    assert abs(sp.energy() - E_ref) <= 1e-9 * abs(E_ref)


def test_zero_blocks_and_all_zero_tiles(OMM):
    """An overlap with whole zero stripes (two decoupled halves of the basis, the second one
    diagonal): the second column tile lists only its diagonal blocks; results still match
    dense."""
    rng = np.random.default_rng(70)
    pos = lattice_positions((8, 8, 2), 2.5)
    pos = pos + rng.uniform(-0.2, 0.2, size=pos.shape)
    s = make_system(pos, 4, 6.0, 96, rng, name="blocks", eta=0.5, tau=10.0, seed=70)
    N = s.N
    H, S, T = s.H.copy(), s.S.copy(), s.T.copy()
    h = N // 2
    for X in (H, S, T):
        X[:h, h:] = 0.0
        X[h:, :h] = 0.0
    for X in (S, T):
        X[h:, h:] = np.diag(np.diag(X[h:, h:]))
    C0 = start_coefficients(S, s.M, 71)
    _say(f"sparse vs dense with zero stripes N={N} M={s.M}")
    (t0, _, _), (t1, _, sp) = _pair(OMM, s, C0, 0.5, 10.0, 40, True, H=H, S=S, T=T)
    assert np.array_equal(t0, t1)
    assert sp.sparse_density()[1] <= 0.5


def test_c3_first_line_searches(OMM):
    import torch

    s = config_system("c3", 0)
    C0 = start_coefficients(s.S, s.M, 1)
    _say(f"sparse vs dense c3 N={s.N} M={s.M}, 4 line searches")
    dev = {k: torch.from_numpy(v).cuda() for k, v in (("H", s.H), ("S", s.S), ("T", s.T), ("C0", C0))}
    traces = []
    for sparse in (False, True):
        solver = OMM(s.N, s.M, precision="bf16x3", refine=True, sparse=sparse)
        solver.set_HS(dev["H"], dev["S"], dev["T"])
        solver.minimize(dev["C0"], eta=s.eta, tau=s.tau, tol=0.0, max_iter=4)
        traces.append(solver.energy_trace())
        if sparse:
            print("c3 K-block density", solver.sparse_density())
        solver.close()
    assert np.array_equal(traces[0], traces[1])
