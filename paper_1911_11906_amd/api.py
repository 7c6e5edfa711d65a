"""Python front end of the fraclap HIP library.

PyTorch supplies device memory and the stream; every computation happens in
the HIP kernels behind the C ABI (include/fraclap.h).  Dense matrices are
column-major: a torch tensor X of shape (n, m) is accepted when
X.stride(0) == 1 (e.g. ``torch.empty(m, n).t()``); helpers below produce that
layout.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import torch

from . import _lib
from ._lib import FlEigInfo, FlEigOpts, FlGemmChoice, FlSliceInfo, FraclapError

# kept at import: module globals (sys included) may already be None when a
# destructor runs during interpreter shutdown
_finalizing = sys.is_finalizing

P = ctypes.c_void_p


def colmajor(x, device=None) -> torch.Tensor:
    """float64 CUDA tensor with column-major storage (stride(0) == 1)."""
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float64).T)).t()
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a numpy array or a torch tensor")
    if x.dim() == 1:
        x = x[:, None]
    dev = device if device is not None else (x.device if x.is_cuda else torch.device("cuda", 0))
    x = x.to(device=dev, dtype=torch.float64)
    if x.stride(0) != 1 or (x.shape[1] > 1 and x.stride(1) < x.shape[0]):
        x = x.t().contiguous().t()
    return x


def empty_colmajor(n: int, m: int, device) -> torch.Tensor:
    return torch.empty((m, n), dtype=torch.float64, device=device).t()


def _ld(x: torch.Tensor) -> int:
    return max(int(x.stride(1)) if x.shape[1] > 1 else int(x.shape[0]), 1)


def _ptr(x: torch.Tensor):
    return P(x.data_ptr())


class Context:
    """One device and the torch stream work is queued on."""

    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        self.device = torch.device("cuda", device)
        self.ptr = P()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        rc = self.lib.fl_ctx_create(device, P(stream), ctypes.byref(self.ptr))
        if rc != 0:
            raise FraclapError(rc, "fl_ctx_create failed")

    def _sync_stream(self):
        self.lib.fl_ctx_set_stream(self.ptr, P(torch.cuda.current_stream(self.device).cuda_stream))

    def check(self, rc: int):
        if rc != 0:
            raise FraclapError(rc, self.lib.fl_last_error(self.ptr).decode())

    def close(self):
        if self.ptr:
            self.lib.fl_ctx_destroy(self.ptr)
            self.ptr = P()

    def __del__(self):
        # no library calls while the interpreter (and the HIP runtime) shut down
        if _finalizing is None or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------ kernel timers
    def kernel_timing(self, enable: bool):
        """Record HIP events around the timed kernels ("q2_apply", "sb2st",
        "scaled_gemm") on the stream each is launched on."""
        self.check(self.lib.fl_kernel_timing(1 if enable else 0))

    def kernel_time(self, name: str):
        """(launches, total ms) accumulated for `name` since the last call."""
        cnt, tot = ctypes.c_int64(0), ctypes.c_double(0.0)
        self.check(self.lib.fl_kernel_time(name.encode(), ctypes.byref(cnt), ctypes.byref(tot)))
        return cnt.value, tot.value

    def measure_peaks(self, copy_bytes: int = 1 << 30) -> dict:
        """Measured FP64 / FP32 matrix-core TFLOP/s and copy GB/s."""
        f64, f32, bw = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._sync_stream()
        self.check(self.lib.fl_measure_peaks(self.ptr, ctypes.byref(f64), ctypes.byref(f32), ctypes.byref(bw),
                                             copy_bytes))
        return {"fp64_mfma_tflops": f64.value, "fp32_mfma_tflops": f32.value, "copy_gbs": bw.value,
                "copy_bytes": copy_bytes}

    # ---------------------------------------------------- launch-shape tuner
    def gemm_tune(self, kind: str, m: int, n: int, k: int, ta: bool = False, tb: bool = False,
                  reps: int = 3) -> dict:
        """Time every launch shape of a product on this device and record the
        fastest (kind "f64", "f32" or "scaled", the spectral product with
        k == m); returns the chosen entry."""
        kd = {"f64": _lib.FL_TUNE_F64, "f32": _lib.FL_TUNE_F32, "scaled": _lib.FL_TUNE_SCALED}[kind]
        out = FlGemmChoice()
        self._sync_stream()
        self.check(self.lib.fl_gemm_tune(self.ptr, kd, int(ta), int(tb), m, n, k, reps, ctypes.byref(out)))
        return out.as_dict()

    def tuning_table(self) -> list:
        out = []
        for i in range(int(self.lib.fl_gemm_tuning_count())):
            c = FlGemmChoice()
            self.check(self.lib.fl_gemm_tuning_get(i, ctypes.byref(c)))
            out.append(c.as_dict())
        return out

    def set_tuning(self, entries) -> None:
        for e in entries:
            c = FlGemmChoice(**{f: e[f] for f, _ in FlGemmChoice._fields_})
            rc = self.lib.fl_gemm_tuning_set(ctypes.byref(c))
            if rc != 0:
                raise FraclapError(rc, f"malformed tuning entry {e}")

    def save_tuning(self, path: str) -> None:
        """JSON file keyed by the device architecture."""
        import json
        arch = torch.cuda.get_device_properties(self.device).gcnArchName
        with open(path, "w") as f:
            json.dump({"arch": arch, "entries": self.tuning_table()}, f, indent=1)

    def load_tuning(self, path: str) -> int:
        """Installs the entries of a JSON tuning file written for this
        device's architecture; returns how many (0 for another architecture)."""
        import json
        with open(path) as f:
            d = json.load(f)
        arch = torch.cuda.get_device_properties(self.device).gcnArchName
        if d.get("arch", "").split(":")[0] != arch.split(":")[0]:
            return 0
        self.set_tuning(d["entries"])
        return len(d["entries"])

    def eigensolve_batched(self, ops, precision: str = "fp64"):
        """Solve every Operator in `ops` in one persistent launch (FP64,
        each n <= 1024); returns the per-problem info dicts."""
        ops = list(ops)
        prec = {"fp64": _lib.FL_FP64, "mixed": _lib.FL_MIXED}[precision]
        arr = (P * len(ops))(*[o.ptr for o in ops])
        infos = (FlEigInfo * max(len(ops), 1))()
        self._sync_stream()
        rc = self.lib.fl_eigensolve_batched(self.ptr, len(ops), ctypes.cast(arr, P), prec,
                                            ctypes.cast(infos, P))
        out = [infos[i].as_dict() for i in range(len(ops))]
        for o, d in zip(ops, out):
            o.info = d
        if rc != 0:
            raise FraclapError(rc, self.lib.fl_last_error(self.ptr).decode())
        return out

    def eigensolve_batched_begin(self, ops, precision: str = "fp64") -> "BatchedSolve":
        """Queue the batched solve of `ops` on the current stream and return
        at once; `wait()` on the result waits for it and returns the
        per-problem info dicts.  The operators are not to be used until
        then."""
        ops = list(ops)
        prec = {"fp64": _lib.FL_FP64, "mixed": _lib.FL_MIXED}[precision]
        arr = (P * max(len(ops), 1))(*[o.ptr for o in ops])
        h = P()
        self._sync_stream()
        rc = self.lib.fl_eigensolve_batched_begin(self.ptr, len(ops), ctypes.cast(arr, P), prec, ctypes.byref(h))
        if rc != 0:
            raise FraclapError(rc, self.lib.fl_last_error(self.ptr).decode())
        return BatchedSolve(self, ops, h)

    # ---------------------------------------------------------- stage calls
    def dgemm(self, A, B, C=None, ta=False, tb=False, alpha=1.0, beta=0.0):
        A, B = colmajor(A, self.device), colmajor(B, self.device)
        m = A.shape[1] if ta else A.shape[0]
        k = A.shape[0] if ta else A.shape[1]
        n = B.shape[0] if tb else B.shape[1]
        if C is None:
            C = empty_colmajor(m, n, self.device)
            beta = 0.0
        self._sync_stream()
        self.check(self.lib.fl_dgemm(self.ptr, int(ta), int(tb), m, n, k, alpha, _ptr(A), _ld(A), _ptr(B), _ld(B),
                                     beta, _ptr(C), _ld(C)))
        return C

    def dpotrf(self, A):
        """Lower Cholesky factor of A (returns a new column-major tensor)."""
        A = colmajor(A, self.device).clone()
        n = A.shape[0]
        info = ctypes.c_int64(0)
        self._sync_stream()
        rc = self.lib.fl_dpotrf(self.ptr, n, _ptr(A), _ld(A), ctypes.byref(info))
        if rc == _lib.FL_ENOTSPD:
            raise FraclapError(rc, f"not positive definite at pivot {info.value}")
        self.check(rc)
        return torch.tril(A)

    def dsygst(self, L, K):
        L, K = colmajor(L, self.device), colmajor(K, self.device).clone()
        self._sync_stream()
        self.check(self.lib.fl_dsygst(self.ptr, K.shape[0], _ptr(L), _ld(L), _ptr(K), _ld(K)))
        return K

    def dstedc(self, d, e):
        d = torch.as_tensor(d, dtype=torch.float64).to(self.device).clone()
        e = torch.as_tensor(e, dtype=torch.float64).to(self.device).clone()
        n = d.numel()
        Z = empty_colmajor(n, n, self.device)
        self._sync_stream()
        self.check(self.lib.fl_dstedc(self.ptr, n, _ptr(d), _ptr(e), _ptr(Z), _ld(Z)))
        return d, Z

    def dsytrd_2stage(self, A, band=0, want_q=True):
        A = colmajor(A, self.device).clone()
        n = A.shape[0]
        d = torch.empty(n, dtype=torch.float64, device=self.device)
        e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=self.device)
        Q = empty_colmajor(n, n, self.device) if want_q else None
        self._sync_stream()
        self.check(self.lib.fl_dsytrd_2stage(self.ptr, n, _ptr(A), _ld(A), band, _ptr(d), _ptr(e),
                                             _ptr(Q) if want_q else None, _ld(Q) if want_q else n))
        return d, e[: n - 1], Q

    def dsyevd(self, A, band=0):
        A = colmajor(A, self.device).clone()
        n = A.shape[0]
        w = torch.empty(n, dtype=torch.float64, device=self.device)
        Z = empty_colmajor(n, n, self.device)
        self._sync_stream()
        self.check(self.lib.fl_dsyevd(self.ptr, n, _ptr(A), _ld(A), band, _ptr(w), _ptr(Z), _ld(Z)))
        return w, Z


class BatchedSolve:
    """A batched solve in flight (from Context.eigensolve_batched_begin)."""

    def __init__(self, ctx: "Context", ops, handle):
        self.ctx, self.ops, self.h = ctx, ops, handle

    def wait(self):
        infos = (FlEigInfo * max(len(self.ops), 1))()
        h, self.h = self.h, None
        if h is None:
            raise FraclapError(_lib.FL_ESTATE, "batched solve already waited for")
        rc = self.ctx.lib.fl_eigensolve_batched_wait(h, ctypes.cast(infos, P))
        out = [infos[i].as_dict() for i in range(len(self.ops))]
        for o, d in zip(self.ops, out):
            o.info = d
        if rc != 0:
            raise FraclapError(rc, self.ctx.lib.fl_last_error(self.ctx.ptr).decode())
        return out


class Operator:
    """A discretised domain (K, M) and, after ``eigensolve``, its eigenbasis."""

    def __init__(self, ctx: Context, ptr: P, dof_of_node=None):
        self.ctx = ctx
        self.ptr = ptr
        self.dof_of_node = dof_of_node
        self.n = int(ctx.lib.fl_op_n(ptr))
        self.info = None

    @classmethod
    def assemble(cls, ctx: Context, mesh, sparse: bool = False) -> "Operator":
        """sparse: keep only the CSR pencil (for n beyond dense storage)."""
        xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
        conn = np.ascontiguousarray(mesh.conn, dtype=np.int32)
        dirichlet = np.ascontiguousarray(mesh.dirichlet, dtype=np.uint8)
        out = P()
        n = ctypes.c_int64(0)
        dof = np.zeros(xy.shape[0], dtype=np.int64)
        ctx._sync_stream()
        fn = ctx.lib.fl_assemble_sparse if sparse else ctx.lib.fl_assemble
        ctx.check(fn(ctx.ptr, int(mesh.elem), xy.shape[0], xy.ctypes.data_as(P), conn.shape[0],
                                      conn.ctypes.data_as(P), dirichlet.ctypes.data_as(P), ctypes.byref(out),
                                      ctypes.byref(n), dof.ctypes.data_as(P)))
        return cls(ctx, out, dof)

    @classmethod
    def from_dense(cls, ctx: Context, K, M) -> "Operator":
        K = np.asfortranarray(K, dtype=np.float64)
        M = np.asfortranarray(M, dtype=np.float64)
        out = P()
        ctx._sync_stream()
        ctx.check(ctx.lib.fl_op_from_dense(ctx.ptr, K.shape[0], K.ctypes.data_as(P), M.ctypes.data_as(P),
                                           K.shape[0], 0, ctypes.byref(out)))
        return cls(ctx, out)

    @classmethod
    def load(cls, ctx: Context, path: str) -> "Operator":
        """An operator (pencil and, when saved, eigenpairs) from fl_op_save."""
        out = P()
        ctx._sync_stream()
        ctx.check(ctx.lib.fl_op_load(ctx.ptr, path.encode(), ctypes.byref(out)))
        return cls(ctx, out)

    def save(self, path: str) -> None:
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_op_save(self.ptr, path.encode()))

    def describe(self) -> dict:
        n, he, pr, it, rr = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self.ctx.check(self.ctx.lib.fl_op_info(self.ptr, ctypes.byref(n), ctypes.byref(he), ctypes.byref(pr),
                                               ctypes.byref(it), ctypes.byref(rr)))
        prec = {_lib.FL_FP64: "fp64", _lib.FL_MIXED: "mixed"}.get(pr.value)
        return {"n": n.value, "has_eig": bool(he.value), "precision": prec, "refine_iters": it.value,
                "refine_resid": rr.value}

    def close(self):
        if self.ptr:
            self.ctx.lib.fl_op_destroy(self.ptr)
            self.ptr = P()

    def __del__(self):
        if _finalizing is None or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def matrices(self):
        K = empty_colmajor(self.n, self.n, self.ctx.device)
        M = empty_colmajor(self.n, self.n, self.ctx.device)
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_op_matrices(self.ptr, _ptr(K), _ptr(M), _ld(K), 1))
        return K, M

    def eigensolve(self, precision: str = "fp64", band: int = 0, leaf: int = 0, refine_max_iters: int = -1,
                   refine_tol: float = 0.0, fp32_band: bool = False) -> dict:
        """precision "fp64" or "mixed" (FP32 back-transforms + FP64
        refinement); fp32_band also runs the band reduction in FP32."""
        prec = {"fp64": _lib.FL_FP64, "mixed": _lib.FL_MIXED}[precision]
        opts = FlEigOpts(band, leaf, refine_max_iters, refine_tol, _lib.FL_MIXED_FP32_BAND if fp32_band else 0)
        info = FlEigInfo()
        self.ctx._sync_stream()
        rc = self.ctx.lib.fl_eigensolve(self.ptr, prec, ctypes.byref(opts), ctypes.byref(info))
        self.info = info.as_dict()
        if rc != 0:
            raise FraclapError(rc, self.ctx.lib.fl_last_error(self.ctx.ptr).decode() + f" (index {info.index})")
        return self.info

    def eigenpairs(self, want_vectors: bool = True):
        theta = torch.empty(self.n, dtype=torch.float64, device=self.ctx.device)
        V = empty_colmajor(self.n, self.n, self.ctx.device) if want_vectors else None
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_eigenpairs(self.ptr, _ptr(theta), _ptr(V) if V is not None else None,
                                                  _ld(V) if V is not None else self.n, 1))
        return theta, V

    def set_eigenpairs(self, theta, V):
        theta = torch.as_tensor(np.asarray(theta) if isinstance(theta, np.ndarray) else theta,
                                dtype=torch.float64).to(self.ctx.device).contiguous()
        V = colmajor(V, self.ctx.device)
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_op_set_eigenpairs(self.ptr, _ptr(theta), _ptr(V), _ld(V), 1))

    def apply(self, F, alpha, paired: bool = False, out=None) -> torch.Tensor:
        """u = sum_k theta_k^(-alpha/2) (phi_k^T M f) phi_k.  Columns j + i*nf
        (all pairs) or b (paired)."""
        F = colmajor(F, self.ctx.device)
        al = np.ascontiguousarray(np.atleast_1d(np.asarray(alpha, dtype=np.float64)))
        nf, na = F.shape[1], al.size
        ncol = nf if paired else nf * na
        U = out if out is not None else empty_colmajor(self.n, ncol, self.ctx.device)
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_apply_fractional(self.ptr, nf, _ptr(F), _ld(F), na, al.ctypes.data_as(P),
                                                        int(paired), _ptr(U), _ld(U)))
        return U

    def inertia(self, sigma):
        """Number of eigenvalues below each shift (Sylvester inertia of
        K - sigma M on the device); returns (counts, bandwidth)."""
        sg = np.ascontiguousarray(np.atleast_1d(np.asarray(sigma, dtype=np.float64)))
        cnt = np.zeros(sg.size, dtype=np.int64)
        bw = ctypes.c_int64(0)
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_inertia_count(self.ptr, sg.size, sg.ctypes.data_as(P), cnt.ctypes.data_as(P),
                                                     ctypes.byref(bw)))
        return cnt, bw.value

    def eigensolve_interval(self, lo: float, hi: float, max_per_slice: int = 128, tol: float = 1e-11,
                            cap: int = None):
        """All eigenpairs with lo <= theta < hi by spectrum slicing; returns
        (theta, V, info) with V n x count (M-orthonormal)."""
        if cap is None:
            cnt, _ = self.inertia([lo, hi])
            cap = max(int(cnt[1] - cnt[0]), 0)
        theta = torch.empty(max(cap, 1), dtype=torch.float64, device=self.ctx.device)
        V = empty_colmajor(self.n, max(cap, 1), self.ctx.device)
        info = FlSliceInfo()
        self.ctx._sync_stream()
        rc = self.ctx.lib.fl_eigensolve_interval(self.ptr, float(lo), float(hi), int(max_per_slice), float(tol),
                                                 int(cap), _ptr(theta), _ptr(V), _ld(V), ctypes.byref(info))
        d = info.as_dict()
        if rc != 0:
            err = FraclapError(rc, self.ctx.lib.fl_last_error(self.ctx.ptr).decode())
            err.info = d
            raise err
        return theta[:d["count"]], V[:, :d["count"]], d

    def apply_graph(self, F, alpha, paired: bool = False, out=None) -> torch.Tensor:
        """Same as ``apply`` (bitwise), captured once per argument set into a
        HIP graph and replayed afterwards (F and out must keep their storage)."""
        F = colmajor(F, self.ctx.device)
        al = np.ascontiguousarray(np.atleast_1d(np.asarray(alpha, dtype=np.float64)))
        nf, na = F.shape[1], al.size
        ncol = nf if paired else nf * na
        U = out if out is not None else empty_colmajor(self.n, ncol, self.ctx.device)
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_apply_graph(self.ptr, nf, _ptr(F), _ld(F), na, al.ctypes.data_as(P),
                                                   int(paired), _ptr(U), _ld(U)))
        return U

    def diffuse(self, U0, alpha, t, mu=1.0, paired: bool = False, out=None) -> torch.Tensor:
        """u(t) = sum_k exp(-mu theta_k^(alpha/2) t) (phi_k^T M u0) phi_k.
        alpha, t, mu: one value per parameter set (t and mu broadcast)."""
        U0 = colmajor(U0, self.ctx.device)
        al = np.ascontiguousarray(np.atleast_1d(np.asarray(alpha, dtype=np.float64)))
        tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), al.shape))
        mu_ = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), al.shape))
        nf, na = U0.shape[1], al.size
        U = out if out is not None else empty_colmajor(self.n, nf if paired else nf * na, self.ctx.device)
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_apply_diffusion(self.ptr, nf, _ptr(U0), _ld(U0), na, al.ctypes.data_as(P),
                                                       tt.ctypes.data_as(P), mu_.ctypes.data_as(P), int(paired),
                                                       _ptr(U), _ld(U)))
        return U

    def grad_diffusion(self, U0, alpha, t, mu, GU, want_u0: bool = True, want_params: bool = True):
        """Adjoint of the paired diffusion map: (GU0, galpha, gt, gmu)."""
        U0 = colmajor(U0, self.ctx.device)
        GU = colmajor(GU, self.ctx.device)
        nb = GU.shape[1]
        al = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha, dtype=np.float64), (nb,)))
        tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), (nb,)))
        mu_ = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (nb,)))
        GU0 = empty_colmajor(self.n, nb, self.ctx.device) if want_u0 else None
        ga, gt, gm = (np.zeros(nb), np.zeros(nb), np.zeros(nb)) if want_params else (None, None, None)
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_grad_diffusion(
            self.ptr, nb, _ptr(U0), _ld(U0), al.ctypes.data_as(P), tt.ctypes.data_as(P), mu_.ctypes.data_as(P),
            _ptr(GU), _ld(GU), _ptr(GU0) if want_u0 else None, _ld(GU0) if want_u0 else self.n,
            ga.ctypes.data_as(P) if want_params else None, gt.ctypes.data_as(P) if want_params else None,
            gm.ctypes.data_as(P) if want_params else None))
        if not want_params:
            return GU0, None, None, None
        return GU0, torch.from_numpy(ga), torch.from_numpy(gt), torch.from_numpy(gm)

    def grad(self, F, alpha, GU, want_f: bool = True, want_alpha: bool = True):
        F = colmajor(F, self.ctx.device)
        GU = colmajor(GU, self.ctx.device)
        al = np.ascontiguousarray(np.atleast_1d(np.asarray(alpha, dtype=np.float64)))
        nb = GU.shape[1]
        GF = empty_colmajor(self.n, nb, self.ctx.device) if want_f else None
        ga = np.zeros(nb) if want_alpha else None
        self.ctx._sync_stream()
        self.ctx.check(self.ctx.lib.fl_grad_apply(
            self.ptr, nb, _ptr(F), _ld(F), al.ctypes.data_as(P), _ptr(GU), _ld(GU),
            _ptr(GF) if want_f else None, _ld(GF) if want_f else self.n,
            ga.ctypes.data_as(P) if want_alpha else None))
        return GF, (torch.from_numpy(ga) if want_alpha else None)


class FracApply(torch.autograd.Function):
    """u_b = v(alpha_b, f_b) for paired columns; backward through the
    hand-written adjoint (fl_grad_apply)."""

    @staticmethod
    def forward(ctx, op: Operator, F: torch.Tensor, alpha: torch.Tensor):
        ctx.op = op
        Fc = colmajor(F.detach(), op.ctx.device)
        ctx.save_for_backward(Fc, alpha.detach())
        U = op.apply(Fc, alpha.detach().cpu().numpy(), paired=True)
        return U

    @staticmethod
    def backward(ctx, gU):
        F, alpha = ctx.saved_tensors
        op = ctx.op
        GF, ga = op.grad(F, alpha.cpu().numpy(), gU, want_f=ctx.needs_input_grad[1],
                         want_alpha=ctx.needs_input_grad[2])
        ga_t = ga.to(alpha.device, alpha.dtype) if ga is not None else None
        return None, GF, ga_t


class FracDiffusion(torch.autograd.Function):
    """u_b(t_b) of the fractional diffusion equation for paired columns
    (u0_b, alpha_b, t_b, mu_b); backward through the hand-written adjoint
    (fl_grad_diffusion)."""

    @staticmethod
    def forward(ctx, op: Operator, U0: torch.Tensor, alpha: torch.Tensor, t: torch.Tensor, mu: torch.Tensor):
        ctx.op = op
        U0c = colmajor(U0.detach(), op.ctx.device)
        ctx.save_for_backward(U0c, alpha.detach(), t.detach(), mu.detach())
        return op.diffuse(U0c, alpha.detach().cpu().numpy(), t.detach().cpu().numpy(), mu.detach().cpu().numpy(),
                          paired=True)

    @staticmethod
    def backward(ctx, gU):
        U0, alpha, t, mu = ctx.saved_tensors
        op = ctx.op
        want_params = any(ctx.needs_input_grad[2:5])
        GU0, ga, gt, gm = op.grad_diffusion(U0, alpha.cpu().numpy(), t.cpu().numpy(), mu.cpu().numpy(), gU,
                                            want_u0=ctx.needs_input_grad[1], want_params=want_params)

        def back(g, like, need):
            return g.to(like.device, like.dtype) if (need and g is not None) else None
        return (None, GU0, back(ga, alpha, ctx.needs_input_grad[2]), back(gt, t, ctx.needs_input_grad[3]),
                back(gm, mu, ctx.needs_input_grad[4]))
