"""Python face of libcola: operator handle, solve, and the autograd Function.

PyTorch supplies device memory and the stream; every step of the MVM, the
CG iteration, the refinement and the gradients runs in the HIP library.
Vectors are packed: system s with n_s unknowns and nrhs right-hand sides
occupies nrhs * n_s consecutive float64 entries (right-hand side r at
offset r * n_s), systems one after another.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_f64(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return t.detach().to(torch.float64).contiguous()


@dataclass
class SystemSpec:
    """One system: factors[j][k] (n_k x n_k float64 device tensors), optional diag, sigma2."""
    factors: List[List[torch.Tensor]]
    sigma2: float = 0.0
    diag: Optional[torch.Tensor] = None

    @property
    def dims(self):
        return tuple(int(f.shape[0]) for f in self.factors[0])

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))


class KronOperator:
    """A = sum_j kron(factors[j]) + diag(d) + sigma2 I for each system (cola_op_create)."""

    def __init__(self, systems: Sequence[SystemSpec], prec: str = "fp32", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("KronOperator needs a ROCm GPU; there is no CPU path")
        self.lib = L.lib()
        self.prec = L.PREC_BY_NAME[prec]
        self.systems = list(systems)
        self._keep = []
        descs = (L.SystemDesc * len(self.systems))()
        for i, s in enumerate(self.systems):
            J, F = len(s.factors), len(s.factors[0])
            fac = [_dev_f64(f) for row in s.factors for f in row]
            self._keep += fac
            arr = (ctypes.c_void_p * (J * F))(*[f.data_ptr() for f in fac])
            self._keep.append(arr)
            d = descs[i]
            d.nterms, d.nfactors = J, F
            for k in range(F):
                d.dims[k] = int(s.factors[0][k].shape[0])
            d.factors = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
            if s.diag is not None:
                dg = _dev_f64(s.diag).reshape(-1)
                self._keep.append(dg)
                d.diag = dg.data_ptr()
            else:
                d.diag = None
            d.sigma2 = float(s.sigma2)
        self._descs = descs
        h = ctypes.c_void_p()
        L.check("cola_op_create", self.lib.cola_op_create(descs, len(self.systems), self.prec,
                                                           _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        torch.cuda.current_stream().synchronize()
        self._keep = []          # the library holds its own copies now
        self.sizes = [s.n for s in self.systems]
        self.n_total = int(sum(self.sizes))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.cola_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- packing helpers -------------------------------------------------
    def pack(self, per_system: Sequence[torch.Tensor]) -> torch.Tensor:
        """(nrhs, n_s) tensors per system -> one packed float64 device vector."""
        return torch.cat([t.to(torch.float64).reshape(-1) for t in per_system]).contiguous()

    def unpack(self, packed: torch.Tensor, nrhs: int) -> List[torch.Tensor]:
        out, off = [], 0
        for n in self.sizes:
            out.append(packed[off:off + nrhs * n].view(nrhs, n))
            off += nrhs * n
        return out

    # ---- entry points ----------------------------------------------------
    def matvec(self, X: torch.Tensor, nrhs: int, prec: Optional[str] = None) -> torch.Tensor:
        p = self.prec if prec is None else L.PREC_BY_NAME[prec]
        dtype = L.COLA_F64 if p == L.COLA_PREC_FP64 else L.COLA_F32
        tdt = torch.float64 if dtype == L.COLA_F64 else torch.float32
        if X.dtype != tdt or not X.is_contiguous():
            raise ValueError(f"X must be a contiguous {tdt} device tensor")
        Y = torch.empty_like(X)
        L.check("cola_kron_matvec", self.lib.cola_kron_matvec(self.handle, X.data_ptr(), Y.data_ptr(), nrhs,
                                                              dtype, p, _stream_ptr()))
        return Y

    def matvec_noalloc(self, X: torch.Tensor, Y: torch.Tensor, nrhs: int, prec: Optional[str] = None) -> torch.Tensor:
        """Y = A X into the caller's Y (cola_kron_matvec_noalloc): no device memory is allocated by
        the library or here; the intermediates use the library's static scratch (see cola.h)."""
        p = self.prec if prec is None else L.PREC_BY_NAME[prec]
        dtype = L.COLA_F64 if p == L.COLA_PREC_FP64 else L.COLA_F32
        tdt = torch.float64 if dtype == L.COLA_F64 else torch.float32
        for t in (X, Y):
            if t.dtype != tdt or not t.is_contiguous():
                raise ValueError(f"X and Y must be contiguous {tdt} device tensors")
        L.check("cola_kron_matvec_noalloc", self.lib.cola_kron_matvec_noalloc(
            self.handle, X.data_ptr(), Y.data_ptr(), nrhs, dtype, p, _stream_ptr()))
        return Y

    def _opts(self, tol, max_iters, prec, inner_tol, max_sweeps, check_every, refine="reliable",
              precond="none", x0_given=False, hist=None, hist_stride=0) -> L.SolveOpts:
        o = L.SolveOpts()
        o.x0_given = 1 if x0_given else 0
        if hist is not None:
            if hist.dtype != torch.float64 or not hist.is_contiguous() or hist.dim() != 2:
                raise ValueError("hist must be a contiguous float64 device tensor (nsys * nrhs, length)")
            o.hist = hist.data_ptr()
            o.hist_len = int(hist.shape[1])
            o.hist_stride = int(hist_stride)
        o.refine = L.REFINE_BY_NAME[refine]
        o.precond = L.PRECOND_BY_NAME[precond]
        o.tol = float(tol)
        o.max_iters = int(max_iters)
        o.prec = self.prec if prec is None else L.PREC_BY_NAME[prec]
        o.inner_tol = float(inner_tol)
        o.max_sweeps = int(max_sweeps)
        o.check_every = int(check_every)
        return o

    def solve(self, B: torch.Tensor, nrhs: int, tol: float = 1e-6, max_iters: int = 10000,
              prec: Optional[str] = None, inner_tol: float = 0.1, max_sweeps: int = 20,
              check_every: int = 32, info: Optional[torch.Tensor] = None, refine: str = "reliable",
              precond: str = "none", x0: Optional[torch.Tensor] = None, hist: Optional[torch.Tensor] = None,
              hist_stride: int = 1):
        """X = A^{-1} B (cola_cg_solve); returns (X, info tensor on device).  precond ("none",
        "jacobi", "kron_eig") selects preconditioned CG, FP64 solves only.  x0: warm start (packed like
        B).  hist: (nsys * nrhs, length) float64 device tensor receiving the recursive relative residual
        every hist_stride iterations (NaN where none was recorded)."""
        if B.dtype != torch.float64 or not B.is_contiguous():
            raise ValueError("B must be a contiguous float64 device tensor")
        if x0 is not None:
            if x0.shape != B.shape or x0.dtype != torch.float64:
                raise ValueError("x0 must be a float64 device tensor shaped like B")
            X = x0.detach().clone().contiguous()
        else:
            X = torch.empty_like(B)
        if info is None:
            info = torch.empty(len(self.sizes) * nrhs * L.INFO_WORDS, dtype=torch.int32, device=B.device)
        o = self._opts(tol, max_iters, prec, inner_tol, max_sweeps, check_every, refine, precond,
                       x0_given=x0 is not None, hist=hist, hist_stride=hist_stride)
        L.check("cola_cg_solve", self.lib.cola_cg_solve(self.handle, B.data_ptr(), X.data_ptr(), nrhs,
                                                        ctypes.byref(o), info.data_ptr(), _stream_ptr()))
        return X, info

    def _grad_buffers(self, dev, want_factors=True, want_diag=True):
        """Per-system gradient outputs and the host pointer arrays the C ABI takes."""
        dfac, ptrs = [], []
        for s in self.systems:
            rows = []
            for row in s.factors:
                r = []
                for f in row:
                    t = torch.empty(f.shape, dtype=torch.float64, device=dev)
                    r.append(t)
                    ptrs.append(t.data_ptr())
                rows.append(r)
            dfac.append(rows)
        ddiag, dptrs = [], []
        for s in self.systems:
            if s.diag is not None and want_diag:
                t = torch.empty(s.n, dtype=torch.float64, device=dev)
                ddiag.append(t)
                dptrs.append(t.data_ptr())
            else:
                ddiag.append(None)
                dptrs.append(None)
        ds2 = torch.empty(len(self.systems), dtype=torch.float64, device=dev)
        fa = (ctypes.c_void_p * max(1, len(ptrs)))(*ptrs) if want_factors else None
        da = (ctypes.c_void_p * len(dptrs))(*dptrs)
        fap = ctypes.cast(fa, ctypes.POINTER(ctypes.c_void_p)) if fa is not None else None
        dap = ctypes.cast(da, ctypes.POINTER(ctypes.c_void_p))
        return dfac, ddiag, ds2, (fa, da, fap, dap)

    def solve_backward(self, X: torch.Tensor, G: torch.Tensor, nrhs: int, tol: float = 1e-6,
                       max_iters: int = 10000, prec: Optional[str] = None, inner_tol: float = 0.1,
                       max_sweeps: int = 20, check_every: int = 32, want_factors: bool = True,
                       want_diag: bool = True, refine: str = "reliable", precond: str = "none"):
        """Adjoint backward (cola_cg_solve_backward): Lambda, dfactors, ddiag, dsigma2, info."""
        dev = X.device
        Lam = torch.empty_like(X)
        dfac, ddiag, ds2, (fa, da, fap, dap) = self._grad_buffers(dev, want_factors, want_diag)
        info = torch.empty(len(self.sizes) * nrhs * L.INFO_WORDS, dtype=torch.int32, device=dev)
        o = self._opts(tol, max_iters, prec, inner_tol, max_sweeps, check_every, refine, precond)
        L.check("cola_cg_solve_backward", self.lib.cola_cg_solve_backward(
            self.handle, X.data_ptr(), G.data_ptr(), nrhs, ctypes.byref(o), Lam.data_ptr(), fap, dap,
            ds2.data_ptr(), info.data_ptr(), _stream_ptr()))
        return Lam, (dfac if want_factors else None), ddiag, ds2, info

    def diagonal(self) -> torch.Tensor:
        """Exact Diag(A) of every system, packed (cola_op_diagonal)."""
        out = torch.empty(self.n_total, dtype=torch.float64, device="cuda")
        L.check("cola_op_diagonal", self.lib.cola_op_diagonal(self.handle, out.data_ptr(), _stream_ptr()))
        return out

    def diag_estimate(self, Z: torch.Tensor, nprobes: int, mode: str = "hutchinson") -> torch.Tensor:
        """Probe estimate of Diag(A) (cola_diag_estimate).  Z: float64 probes, packed per system as
        nprobes vectors ("hutchinson") or nterms * nprobes vectors, term-major ("doubly")."""
        if Z.dtype != torch.float64 or not Z.is_contiguous():
            raise ValueError("Z must be a contiguous float64 device tensor")
        per = [nprobes * n if mode == "hutchinson" else nprobes * len(s.factors) * n
               for s, n in zip(self.systems, self.sizes)]
        if Z.numel() != sum(per):
            raise ValueError(f"Z has {Z.numel()} entries; {sum(per)} expected")
        out = torch.empty(sum(self.sizes), dtype=torch.float64, device=Z.device)
        L.check("cola_diag_estimate", self.lib.cola_diag_estimate(
            self.handle, Z.data_ptr(), nprobes, L.DIAG_MODE_BY_NAME[mode], out.data_ptr(), _stream_ptr()))
        return out

    def eig_solve(self, B: torch.Tensor, nrhs: int) -> torch.Tensor:
        """X = A^{-1} B for single-term Kronecker + sigma2 I systems by the Kronecker eigen rules
        (cola_eig_solve); the factors' eigendecomposition is computed on the first call."""
        if B.dtype != torch.float64 or not B.is_contiguous():
            raise ValueError("B must be a contiguous float64 device tensor")
        X = torch.empty_like(B)
        L.check("cola_eig_solve", self.lib.cola_eig_solve(self.handle, B.data_ptr(), X.data_ptr(), nrhs,
                                                           _stream_ptr()))
        return X

    def logdet(self, Z: torch.Tensor, nprobes: int, tol: float = 1e-8, max_iters: int = 200,
               want_solution: bool = False):
        """Stochastic Lanczos quadrature estimate of log det A per system (cola_slq_logdet).

        Z: packed float64 probes (nprobes per system, e.g. +-1 entries).  Returns (logdet per
        system, per-probe estimates, A^{-1} Z or None, info tensor)."""
        if Z.dtype != torch.float64 or not Z.is_contiguous():
            raise ValueError("Z must be a contiguous float64 device tensor")
        nsys = len(self.systems)
        ld = torch.empty(nsys, dtype=torch.float64, device=Z.device)
        est = torch.empty(nsys * nprobes, dtype=torch.float64, device=Z.device)
        X = torch.empty_like(Z) if want_solution else None
        info = torch.empty(len(self.sizes) * nprobes * L.INFO_WORDS, dtype=torch.int32, device=Z.device)
        L.check("cola_slq_logdet", self.lib.cola_slq_logdet(
            self.handle, Z.data_ptr(), nprobes, tol, max_iters, X.data_ptr() if X is not None else None,
            ld.data_ptr(), est.data_ptr(), info.data_ptr(), _stream_ptr()))
        return ld, est, X, info

    def logdet_grad(self, Z: torch.Tensor, nprobes: int, tol: float = 1e-8, max_iters: int = 10000,
                    x0: Optional[torch.Tensor] = None):
        """Hutchinson estimate of d log det A / d(factors, diagonal, sigma2) (cola_logdet_grad): the mean
        over probes of (A^{-1} z)^T (dA/dtheta) z.  x0: a warm start for A^{-1} Z (e.g. logdet's X)."""
        if Z.dtype != torch.float64 or not Z.is_contiguous():
            raise ValueError("Z must be a contiguous float64 device tensor")
        dev = Z.device
        Lam = x0.detach().clone().contiguous() if x0 is not None else torch.empty_like(Z)
        dfac, ddiag, ds2, (fa, da, fap, dap) = self._grad_buffers(dev)
        info = torch.empty(len(self.sizes) * nprobes * L.INFO_WORDS, dtype=torch.int32, device=dev)
        o = self._opts(tol, max_iters, "fp64", 0.1, 20, 32, x0_given=x0 is not None)
        L.check("cola_logdet_grad", self.lib.cola_logdet_grad(
            self.handle, Z.data_ptr(), nprobes, ctypes.byref(o), Lam.data_ptr(), fap, dap, ds2.data_ptr(),
            info.data_ptr(), _stream_ptr()))
        return dfac, ddiag, ds2, info

    def autotune(self, nrhs: int, cache: Optional[str] = None) -> bool:
        """Tune the tile shapes of the general contraction passes for nrhs right-hand sides.

        cache: a JSON file mapping a shape signature (working precision, nrhs, every system's
        modes and term count) to the table cola_autotune_export writes.  A hit loads the table
        (cola_autotune_import applies only the entries recorded on this device) instead of timing
        the candidates; a miss tunes and adds the table.  Returns True on a hit."""
        sig = None
        if cache is not None:
            sig = json.dumps({"prec": int(self.prec), "nrhs": int(nrhs),
                              "systems": [[list(map(int, s.dims)), len(s.factors), s.diag is not None]
                                          for s in self.systems]}, sort_keys=True)
            table = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    table = json.load(fh)
            if sig in table:
                L.check("cola_autotune_import", self.lib.cola_autotune_import(self.handle, table[sig].encode()))
                return True
        L.check("cola_autotune", self.lib.cola_autotune(self.handle, nrhs, _stream_ptr()))
        if cache is not None:
            n = ctypes.c_int64()
            L.check("cola_autotune_export", self.lib.cola_autotune_export(self.handle, None, 0, ctypes.byref(n)))
            buf = ctypes.create_string_buffer(int(n.value) + 1)
            L.check("cola_autotune_export", self.lib.cola_autotune_export(self.handle, buf, n.value + 1,
                                                                          ctypes.byref(n)))
            table = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    table = json.load(fh)
            table[sig] = buf.value.decode()
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return False

    def set_engine(self, name: str, enable: bool):
        """Switch one kernel engine on or off ("fused_cg", "gemm2", "gemm3", "slab", "resident", "small64",
        "gemm64")."""
        if name not in L.ENGINE_BY_NAME:
            raise ValueError(f"unknown engine {name!r}; one of {sorted(L.ENGINE_BY_NAME)}")
        L.check("cola_op_set_engine",
                self.lib.cola_op_set_engine(self.handle, L.ENGINE_BY_NAME[name], 1 if enable else 0))

    def memory(self, reset_peak: bool = False):
        """(live, peak) bytes of device memory held by this operator (cola_op_memory)."""
        live, peak = ctypes.c_int64(), ctypes.c_int64()
        L.check("cola_op_memory", self.lib.cola_op_memory(self.handle, ctypes.byref(live), ctypes.byref(peak),
                                                          1 if reset_peak else 0))
        return live.value, peak.value

    @staticmethod
    def trace_enable(on: bool = True):
        """Process-wide roctx ranges around the library's calls (cola_trace_enable), for
        rocprofv3 --marker-trace."""
        L.check("cola_trace_enable", L.lib().cola_trace_enable(1 if on else 0))

    def profile_enable(self, on: bool = True):
        L.check("cola_profile_enable", self.lib.cola_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self, kernel: str):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        L.check("cola_profile_read", self.lib.cola_profile_read(self.handle, kernel.encode(), ctypes.byref(ms),
                                                                ctypes.byref(cnt)))
        return ms.value, cnt.value


def decode_info(info: torch.Tensor, count: int):
    """Device info buffer -> list of dicts (status, iters, sweeps, relres_recursive, relres_true, and
    relres = the FP64 true residual of the returned X)."""
    raw = info.detach().cpu().numpy().view(np.uint8)[: count * 4 * L.INFO_WORDS]
    rec = np.frombuffer(raw.tobytes(), dtype=np.dtype([("status", "<i4"), ("iters", "<i4"), ("sweeps", "<i4"),
                                                        ("reserved", "<i4"), ("relres_recursive", "<f8"),
                                                        ("relres_true", "<f8")]))
    return [dict(status=int(r["status"]), iters=int(r["iters"]), sweeps=int(r["sweeps"]),
                 relres_recursive=float(r["relres_recursive"]), relres_true=float(r["relres_true"]),
                 relres=float(r["relres_true"])) for r in rec]


class KronSolve(torch.autograd.Function):
    """x = A^{-1} b with the adjoint backward of App. B.2 (rule 1).

    forward(meta, B_packed, sigma2 (nsys), *tensors) where tensors are every
    factor (system, term, factor order) followed by every diagonal present.
    The backward runs a second solve for Lambda and the factor contractions
    inside libcola; gradients flow on to whatever built the factors (e.g. an
    RBF lengthscale) through torch's autograd.
    """

    @staticmethod
    def forward(ctx, meta, B, sigma2, *tensors):
        specs, opts = meta["specs"], meta["opts"]
        it = iter(tensors)
        systems = []
        for i, (J, F, has_diag) in enumerate(specs):
            facs = [[next(it) for _ in range(F)] for _ in range(J)]
            systems.append([facs, has_diag])
        diags = [next(it) if has_diag else None for (_, _, has_diag) in specs]
        sys_specs = [SystemSpec(factors=f, sigma2=float(sigma2[i]), diag=diags[i])
                     for i, (f, _) in enumerate(systems)]
        op = KronOperator(sys_specs, prec=opts.get("prec", "fp32"))
        nrhs = meta["nrhs"]
        X, info = op.solve(B.detach().to(torch.float64).contiguous(), nrhs, **opts)
        ctx.op = op
        ctx.meta = meta
        ctx.save_for_backward(X)
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, gX):
        (X,) = ctx.saved_tensors
        op, meta = ctx.op, ctx.meta
        opts = dict(meta["opts"])
        opts.update(meta.get("backward_opts", {}))
        Lam, dfac, ddiag, ds2, info = op.solve_backward(X, gX.contiguous().to(torch.float64), meta["nrhs"], **opts)
        ctx.backward_info = info
        ctx.device_peak_bytes = op.memory()[1]     # the operator's buffers over forward and backward
        grads = [None, Lam, ds2]
        for s in dfac:
            for row in s:
                grads.extend(row)
        for (J, F, has_diag), dd in zip(meta["specs"], ddiag):
            if has_diag:
                grads.append(dd)
        op.close()
        return tuple(grads)


def kron_cg_solve(systems: Sequence[SystemSpec], B: torch.Tensor, nrhs: int, **opts) -> torch.Tensor:
    """Differentiable packed solve X = A^{-1} B over all systems."""
    specs = [(len(s.factors), len(s.factors[0]), s.diag is not None) for s in systems]
    backward_opts = opts.pop("backward_opts", {})
    meta = {"specs": specs, "opts": opts, "nrhs": nrhs, "backward_opts": backward_opts}
    sig = [s.sigma2 for s in systems]
    sigma2 = torch.stack([torch.as_tensor(v, dtype=torch.float64, device=B.device) for v in sig])
    tensors = [f for s in systems for row in s.factors for f in row]
    tensors += [s.diag for s in systems if s.diag is not None]
    return KronSolve.apply(meta, B, sigma2, *tensors)
