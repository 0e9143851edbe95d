"""Python binding of libomm: argument marshalling around the C-ABI of include/omm.h.

Host inputs are NumPy FP64 arrays; device inputs are FP64 ``torch`` tensors on the GPU (PyTorch
supplies device memory and the current stream only). Every step of the minimization runs in the
library's HIP kernels.
"""

from __future__ import annotations

import ctypes as ct
import math
from typing import Optional, Sequence

import numpy as np

from ._lib import lib

OK = 0
W_MAXITER = 1
ERRORS = {
    -1: "OMM_E_ARG", -2: "OMM_E_STATE", -3: "OMM_E_ALLOC", -4: "OMM_E_HIP",
    -5: "OMM_E_NONFINITE", -6: "OMM_E_PRECON", -7: "OMM_E_NO_LINE_MIN", -8: "OMM_E_DIVERGED",
    -9: "OMM_E_ASYMMETRIC",
}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
FLAVOURS = {"dense": 0, "cholesky": 1}


class OMMError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _host_ptr(a: np.ndarray, shape) -> ct.c_void_p:
    if a.dtype != np.float64 or not a.flags.c_contiguous or a.shape != tuple(shape):
        raise ValueError(f"expected a C-contiguous float64 array of shape {tuple(shape)}")
    return ct.c_void_p(a.ctypes.data)


def _dev_ptr(t, shape) -> ct.c_void_p:
    import torch

    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected a contiguous float64 GPU tensor of shape {tuple(shape)}")
    return ct.c_void_p(t.data_ptr())


class OMM:
    """One dense OMM problem (N basis orbitals, M Wannier functions) on the current GPU."""

    def __init__(self, N: int, M: int, precision: str = "fp64", refine: bool = True,
                 mixed_tol: Optional[float] = None, use_torch_stream: bool = True,
                 resync: Optional[int] = None, flavour: str = "dense", sparse: bool = False):
        self._L = lib()
        self.N, self.M = int(N), int(M)
        h = ct.c_void_p()
        r = self._L.omm_create(self.N, self.M, ct.byref(h))
        if r != OK:
            raise OMMError(r, f"omm_create(N={N}, M={M}) failed")
        self._h = h
        self.set_precision(precision, refine)
        if mixed_tol is not None:
            self._check(self._L.omm_set_mixed_tol(self._h, float(mixed_tol)))
        if resync is not None:
            self._check(self._L.omm_set_resync(self._h, int(resync)))
        self.set_flavour(flavour)
        self._check(self._L.omm_set_sparse(self._h, 1 if sparse else 0))
        self._use_torch_stream = use_torch_stream

    # -- plumbing --------------------------------------------------------------------------
    def _check(self, r: int) -> int:
        if r < 0:
            msg = self._L.omm_last_error(self._h)
            raise OMMError(r, msg.decode() if msg else "")
        return r

    def _bind_stream(self):
        if self._use_torch_stream:
            import torch

            if torch.cuda.is_available():
                s = torch.cuda.current_stream().cuda_stream
                self._check(self._L.omm_set_stream(self._h, ct.c_void_p(s)))

    def close(self):
        if getattr(self, "_h", None):
            self._L.omm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- API ---------------------------------------------------------------------------------
    def set_precision(self, precision: str = "fp64", refine: bool = True):
        self._check(self._L.omm_set_precision(self._h, PRECISIONS[precision], 1 if refine else 0))

    def set_flavour(self, flavour: str):
        """"dense" (the generalized problem, preconditioner from tau) or "cholesky" (the
        Cholesky-reduced problem; tau is ignored, outputs are in the original basis)."""
        if flavour not in FLAVOURS:
            raise ValueError(f"flavour must be one of {sorted(FLAVOURS)}")
        self._check(self._L.omm_set_flavour(self._h, FLAVOURS[flavour]))

    def sparse_density(self):
        """Fractions of K blocks the block-sparse products visit for (Hs, S)."""
        d = (ct.c_double * 2)()
        self._check(self._L.omm_sparse_density(self._h, d))
        return float(d[0]), float(d[1])

    def set_HS(self, H, S, T=None):
        n = (self.N, self.N)
        if _is_torch(H):
            self._bind_stream()
            self._check(self._L.omm_set_HS_device(
                self._h, _dev_ptr(H, n), _dev_ptr(S, n), _dev_ptr(T, n) if T is not None else None))
        else:
            self._check(self._L.omm_set_HS(
                self._h, _host_ptr(H, n), _host_ptr(S, n), _host_ptr(T, n) if T is not None else None))

    def minimize(self, C0=None, eta: float = 0.0, tau: float = 10.0, tol: float = 1e-10,
                 max_iter: int = 1000) -> int:
        """Returns 0 (converged) or 1 (max_iter reached); raises OMMError on errors."""
        mn = (self.M, self.N)
        if C0 is not None and _is_torch(C0):
            self._bind_stream()
            return self._check(self._L.omm_minimize_device(
                self._h, _dev_ptr(C0, mn), float(eta), float(tau), float(tol), int(max_iter)))
        self._bind_stream()
        ptr = _host_ptr(C0, mn) if C0 is not None else None
        return self._check(self._L.omm_minimize(self._h, ptr, float(eta), float(tau), float(tol),
                                                int(max_iter)))

    def iterate(self, count: int, tol: float = 0.0) -> int:
        """Continue the last minimization for up to `count` line searches (no setup)."""
        self._bind_stream()
        return self._check(self._L.omm_iterate(self._h, int(count), float(tol)))

    STAGES = ("gradient", "precondition", "direction", "operator_products", "projections",
              "line_search", "update")

    def set_profiling(self, on: bool = True):
        self._check(self._L.omm_set_profiling(self._h, 1 if on else 0))

    def stage_times(self):
        """(dict stage -> accumulated ms, profiled line searches)."""
        buf = (ct.c_double * 7)()
        it = ct.c_int()
        self._check(self._L.omm_stage_times(self._h, buf, 7, ct.byref(it)))
        return dict(zip(self.STAGES, list(buf))), it.value

    def energy(self) -> float:
        e = ct.c_double()
        self._check(self._L.omm_energy(self._h, ct.byref(e)))
        return e.value

    def density(self, out=None):
        if out is not None and _is_torch(out):
            self._bind_stream()
            self._check(self._L.omm_density_device(self._h, _dev_ptr(out, (self.N, self.N))))
            return out
        out = np.empty((self.N, self.N)) if out is None else out
        self._check(self._L.omm_density(self._h, _host_ptr(out, (self.N, self.N))))
        return out

    def edm(self, out=None):
        if out is not None and _is_torch(out):
            self._bind_stream()
            self._check(self._L.omm_edm_device(self._h, _dev_ptr(out, (self.N, self.N))))
            return out
        out = np.empty((self.N, self.N)) if out is None else out
        self._check(self._L.omm_edm(self._h, _host_ptr(out, (self.N, self.N))))
        return out

    def backward(self, gE: float, dH, dS):
        self._bind_stream()
        n = (self.N, self.N)
        self._check(self._L.omm_backward_device(self._h, float(gE), _dev_ptr(dH, n), _dev_ptr(dS, n)))

    def get_C(self) -> np.ndarray:
        out = np.empty((self.M, self.N))
        self._check(self._L.omm_get_C(self._h, _host_ptr(out, (self.M, self.N))))
        return out

    def subspace(self):
        HW = np.empty((self.M, self.M))
        SW = np.empty((self.M, self.M))
        self._check(self._L.omm_get_subspace(self._h, _host_ptr(HW, HW.shape), _host_ptr(SW, SW.shape)))
        return HW, SW

    def preconditioner(self) -> np.ndarray:
        out = np.empty((self.N, self.N))
        self._check(self._L.omm_get_preconditioner(self._h, _host_ptr(out, out.shape)))
        return out

    def stats(self):
        it = ct.c_int()
        rel = ct.c_double()
        self._check(self._L.omm_stats(self._h, ct.byref(it), ct.byref(rel)))
        return it.value, rel.value

    def checkpoints(self):
        """(line-search indices, FP64-exact energies) of the BF16x3 + FP64-state scheme."""
        n = ct.c_int()
        self._check(self._L.omm_checkpoints(self._h, None, None, 0, ct.byref(n)))
        it = (ct.c_int * max(n.value, 1))()
        E = (ct.c_double * max(n.value, 1))()
        self._check(self._L.omm_checkpoints(self._h, it, E, n.value, ct.byref(n)))
        return np.array(list(it)[: n.value]), np.array(list(E)[: n.value])

    def phase_stats(self):
        """(mixed-precision line searches, FP64 line searches) of the last minimize call."""
        a, b = ct.c_int(), ct.c_int()
        self._check(self._L.omm_phase_stats(self._h, ct.byref(a), ct.byref(b)))
        return a.value, b.value

    def energy_trace(self) -> np.ndarray:
        n = ct.c_int()
        self._check(self._L.omm_energy_trace(self._h, None, 0, ct.byref(n)))
        buf = np.empty(max(n.value, 1))
        self._check(self._L.omm_energy_trace(self._h, buf.ctypes.data_as(ct.POINTER(ct.c_double)),
                                             n.value, ct.byref(n)))
        return buf[: n.value]


class OMMComplex(OMM):
    """One complex Hermitian problem (a k-point): N orbitals, M Wannier functions, held by the
    library as its exact real embedding. Inputs are complex NumPy arrays (host)."""

    def __init__(self, N: int, M: int, precision: str = "fp64", refine: bool = True,
                 mixed_tol: Optional[float] = None, resync: Optional[int] = None,
                 flavour: str = "dense", sparse: bool = False):
        self._L = lib()
        self.Nc, self.Mc = int(N), int(M)
        self.N, self.M = 2 * self.Nc, 2 * self.Mc
        h = ct.c_void_p()
        r = self._L.omm_create_complex(self.Nc, self.Mc, ct.byref(h))
        if r != OK:
            raise OMMError(r, f"omm_create_complex(N={N}, M={M}) failed")
        self._h = h
        self.set_precision(precision, refine)
        if mixed_tol is not None:
            self._check(self._L.omm_set_mixed_tol(self._h, float(mixed_tol)))
        if resync is not None:
            self._check(self._L.omm_set_resync(self._h, int(resync)))
        self.set_flavour(flavour)
        self._check(self._L.omm_set_sparse(self._h, 1 if sparse else 0))
        self._use_torch_stream = False

    @staticmethod
    def _parts(X, shape):
        X = np.asarray(X)
        if X.shape != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {X.shape}")
        re = np.ascontiguousarray(X.real, dtype=np.float64)
        im = np.ascontiguousarray(X.imag, dtype=np.float64) if np.iscomplexobj(X) else None
        return re, im

    @staticmethod
    def _p(a):
        return None if a is None else a.ctypes.data_as(ct.POINTER(ct.c_double))

    def set_HS(self, H, S, T=None):
        n = (self.Nc, self.Nc)
        Hr, Hi = self._parts(H, n)
        Sr, Si = self._parts(S, n)
        Tr, Ti = self._parts(T, n) if T is not None else (None, None)
        self._check(self._L.omm_set_HS_complex(self._h, self._p(Hr), self._p(Hi), self._p(Sr),
                                               self._p(Si), self._p(Tr), self._p(Ti)))

    def minimize(self, C0=None, eta: float = 0.0, tau: float = 10.0, tol: float = 1e-10,
                 max_iter: int = 1000) -> int:
        if C0 is None:
            return self._check(self._L.omm_minimize_complex(self._h, None, None, float(eta),
                                                            float(tau), float(tol), int(max_iter)))
        Cr, Ci = self._parts(C0, (self.Mc, self.Nc))
        return self._check(self._L.omm_minimize_complex(self._h, self._p(Cr), self._p(Ci),
                                                        float(eta), float(tau), float(tol),
                                                        int(max_iter)))

    def density(self, out=None):
        re = np.empty((self.Nc, self.Nc))
        im = np.empty((self.Nc, self.Nc))
        self._check(self._L.omm_density_complex(self._h, self._p(re), self._p(im)))
        return re + 1j * im


class OMMBatch:
    """Many independent systems of uneven size (FP32 or FP64 products, FP64 reductions).

    ``precision="fp32"`` with ``refine=True`` runs an FP64 phase after the FP32 one (both in
    grouped launches); ``mixed_tol`` is the FP32 phase's stopping threshold."""

    def __init__(self, Ns: Sequence[int], Ms: Sequence[int], precision: str = "fp32",
                 refine: bool = False, mixed_tol: Optional[float] = None):
        self._L = lib()
        self.Ns = [int(n) for n in Ns]
        self.Ms = [int(m) for m in Ms]
        k = len(self.Ns)
        h = ct.c_void_p()
        Na = (ct.c_int64 * k)(*self.Ns)
        Ma = (ct.c_int64 * k)(*self.Ms)
        r = self._L.omm_batch_create(k, Na, Ma, ct.byref(h))
        if r != OK:
            raise OMMError(r, "omm_batch_create failed")
        self._h = h
        self.set_precision(precision, refine)
        if mixed_tol is not None:
            self._check(self._L.omm_batch_set_mixed_tol(self._h, float(mixed_tol)))

    def set_precision(self, precision: str = "fp32", refine: bool = False):
        self._check(self._L.omm_batch_set_precision(self._h, PRECISIONS[precision],
                                                    1 if refine else 0))

    def phase_iterations(self):
        """(line searches of the FP32 phase, of the FP64 phase) per system."""
        k = len(self.Ns)
        a = np.zeros(k, dtype=np.int32)
        b = np.zeros(k, dtype=np.int32)
        self._check(self._L.omm_batch_phase_iterations(
            self._h, a.ctypes.data_as(ct.POINTER(ct.c_int)), b.ctypes.data_as(ct.POINTER(ct.c_int))))
        return a, b

    def _check(self, r: int) -> int:
        if r < 0:
            msg = self._L.omm_batch_last_error(self._h)
            raise OMMError(r, msg.decode() if msg else "")
        return r

    def close(self):
        if getattr(self, "_h", None):
            self._L.omm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_HS(self, i: int, H, S, T=None):
        n = (self.Ns[i], self.Ns[i])
        if _is_torch(H):
            import torch

            # the batch copies on its own stream: the producers of H, S, T must have finished
            torch.cuda.current_stream().synchronize()
            self._check(self._L.omm_batch_set_HS_device(
                self._h, i, _dev_ptr(H, n), _dev_ptr(S, n), _dev_ptr(T, n) if T is not None else None))
        else:
            self._check(self._L.omm_batch_set_HS(self._h, i, _host_ptr(H, n), _host_ptr(S, n),
                                                 _host_ptr(T, n) if T is not None else None))

    def minimize(self, C0s, etas, taus, tol: float, max_iter: int) -> int:
        k = len(self.Ns)
        keep = []
        ptrs = (ct.c_void_p * k)()
        for i in range(k):
            if C0s is None or C0s[i] is None:
                ptrs[i] = None
            else:
                a = np.ascontiguousarray(C0s[i], dtype=np.float64)
                keep.append(a)
                ptrs[i] = _host_ptr(a, (self.Ms[i], self.Ns[i])).value
        e = (ct.c_double * k)(*[float(x) for x in etas])
        t = (ct.c_double * k)(*[float(x) for x in taus])
        return self._check(self._L.omm_batch_minimize(self._h, ptrs, e, t, float(tol), int(max_iter)))

    def energies(self) -> np.ndarray:
        out = np.empty(len(self.Ns))
        self._check(self._L.omm_batch_energy(self._h, out.ctypes.data_as(ct.POINTER(ct.c_double))))
        return out

    def iterations(self) -> np.ndarray:
        out = np.zeros(len(self.Ns), dtype=np.int32)
        self._check(self._L.omm_batch_iterations(self._h, out.ctypes.data_as(ct.POINTER(ct.c_int))))
        return out

    def get_C(self, i: int) -> np.ndarray:
        out = np.empty((self.Ms[i], self.Ns[i]))
        self._check(self._L.omm_batch_get_C(self._h, i, _host_ptr(out, out.shape)))
        return out


class OMMBatchComplex(OMMBatch):
    """k-point batch: complex Hermitian systems (complex sizes Ns, Ms) solved together through
    their real embeddings. Inputs are complex NumPy arrays."""

    def __init__(self, Ns: Sequence[int], Ms: Sequence[int], precision: str = "fp32",
                 refine: bool = False, mixed_tol: Optional[float] = None):
        self._L = lib()
        self.Nc = [int(n) for n in Ns]
        self.Mc = [int(m) for m in Ms]
        self.Ns = [2 * n for n in self.Nc]
        self.Ms = [2 * m for m in self.Mc]
        k = len(self.Nc)
        h = ct.c_void_p()
        r = self._L.omm_batch_create_complex(k, (ct.c_int64 * k)(*self.Nc),
                                             (ct.c_int64 * k)(*self.Mc), ct.byref(h))
        if r != OK:
            raise OMMError(r, "omm_batch_create_complex failed")
        self._h = h
        self.set_precision(precision, refine)
        if mixed_tol is not None:
            self._check(self._L.omm_batch_set_mixed_tol(self._h, float(mixed_tol)))

    def set_HS(self, i: int, H, S, T=None):
        n = (self.Nc[i], self.Nc[i])
        parts = [OMMComplex._parts(X, n) if X is not None else (None, None) for X in (H, S, T)]
        p = OMMComplex._p
        self._check(self._L.omm_batch_set_HS_complex(self._h, i, p(parts[0][0]), p(parts[0][1]),
                                                     p(parts[1][0]), p(parts[1][1]),
                                                     p(parts[2][0]), p(parts[2][1])))

    def minimize(self, C0s, etas, taus, tol: float, max_iter: int) -> int:
        k = len(self.Nc)
        keep = []
        re = (ct.c_void_p * k)()
        im = (ct.c_void_p * k)()
        for i in range(k):
            if C0s is None or C0s[i] is None:
                re[i] = im[i] = None
                continue
            r, j = OMMComplex._parts(C0s[i], (self.Mc[i], self.Nc[i]))
            keep += [r, j]
            re[i] = r.ctypes.data
            im[i] = j.ctypes.data if j is not None else None
        e = (ct.c_double * k)(*[float(x) for x in etas])
        t = (ct.c_double * k)(*[float(x) for x in taus])
        return self._check(self._L.omm_batch_minimize_complex(self._h, re, im, e, t, float(tol),
                                                              int(max_iter)))

    def get_C_complex(self, i: int) -> np.ndarray:
        """The complex Wannier functions held in the first M rows of system i's embedding."""
        C = self.get_C(i)
        m, n = self.Mc[i], self.Nc[i]
        return C[:m, :n] + 1j * C[:m, n:]


def _energy_function():
    import torch

    class OMMEnergy(torch.autograd.Function):
        """E(H, S) = min_C of Eq. 8 for H - eta S; backward returns (gE rho, gE (-EDM - eta rho)).

        ``solver`` is an :class:`OMM` of matching size; it keeps C between calls (warm starts).
        """

        @staticmethod
        def forward(ctx, H, S, T, C0, eta, tau, tol, max_iter, solver):
            solver.set_HS(H, S, T)
            solver.minimize(C0, eta=eta, tau=tau, tol=tol, max_iter=max_iter)
            ctx.solver = solver
            ctx.shape = H.shape
            return torch.tensor(solver.energy(), dtype=torch.float64, device=H.device)

        @staticmethod
        def backward(ctx, gE):
            dH = torch.empty(ctx.shape, dtype=torch.float64, device=gE.device)
            dS = torch.empty_like(dH)
            ctx.solver.backward(float(gE.item()), dH, dS)
            return dH, dS, None, None, None, None, None, None, None

    return OMMEnergy


_OMMEnergy = None


def omm_energy(H, S, T, C0, eta: float, tau: float, tol: float, max_iter: int, solver: OMM):
    """Differentiable minimum energy (see OMMEnergy)."""
    global _OMMEnergy
    if _OMMEnergy is None:
        _OMMEnergy = _energy_function()
    return _OMMEnergy.apply(H, S, T, C0, eta, tau, tol, max_iter, solver)


def flops_per_iteration(N: int, M: int, preconditioned: bool = True) -> float:
    """Algorithmic flops of one line search: 2 (M x N x N) operator products (+1 for P),
    gradient 2 (M x M x N), 4 projections (M x N x M) -- the direct-coefficient column of the
    paper's operation-count table (Sec. 2.3)."""
    big = (3 if preconditioned else 2) * 2.0 * M * N * N
    return big + 2 * 2.0 * M * M * N + 4 * 2.0 * M * M * N


def inf() -> float:
    return math.inf
