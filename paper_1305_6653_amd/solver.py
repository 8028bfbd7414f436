"""Python face of the C ABI: a thin wrapper that marshals arrays into ``libfdebvm.so``.

Host arrays are numpy FP64 arrays; device arrays are torch CUDA (ROCm/HIP) FP64 tensors,
passed by pointer (torch is only the allocator and stream owner).  Every computation
happens in the HIP library; nothing here does arithmetic on the data.
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref
from typing import Optional

import numpy as np

from . import _native as N
from .devmem import DeviceArray

_KINDS = {"trapezoidal": N.FDE_BVM_TRAPEZOIDAL, "gbdf3": N.FDE_BVM_GBDF3, "gam5": N.FDE_BVM_GAM5}
_PREC = {"fp64": N.FDE_FP64, "mixed": N.FDE_MIXED_C32, "c32": N.FDE_MIXED_C32}
_PC = {"strang": N.FDE_PC_STRANG, "bccb": N.FDE_PC_BCCB, "bccb_shifted": N.FDE_PC_BCCB_SHIFTED,
       "none": N.FDE_PC_NONE}
_SIDE = {"right": N.FDE_SIDE_RIGHT, "left": N.FDE_SIDE_LEFT}
_BLOCKS = {"lu": N.FDE_BLOCKS_LU, "hessenberg": N.FDE_BLOCKS_HESSENBERG, "band": N.FDE_BLOCKS_BAND,
           "auto": N.FDE_BLOCKS_AUTO}


_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    """Destroy the handles still open at interpreter exit while the HIP runtime is fully up
    (a destructor run during interpreter teardown could free device memory after the
    runtime's own exit handlers)."""
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


def _is_torch_cuda(x) -> bool:
    return hasattr(x, "is_cuda") and bool(x.is_cuda) and not isinstance(x, DeviceArray)


def _sync_torch_producers(stream_ptr, *arrays):
    """Device tensors are read on the library's stream.  Unless that stream is torch's current
    one, wait until torch's current stream has finished the work that produced them."""
    if not any(_is_torch_cuda(a) for a in arrays if a is not None):
        return
    import torch
    cs = torch.cuda.current_stream()
    if not (stream_ptr and stream_ptr == cs.cuda_stream):
        cs.synchronize()


def _arg(x, count: int, name: str, writable: bool = False):
    """Return (pointer, mem_space, keepalive) for a host numpy array or a device FP64 array
    (torch CUDA tensor or ``DeviceArray``)."""
    if isinstance(x, DeviceArray):
        if x.numel() != count:
            raise ValueError(f"{name}: expected {count} elements, got {x.numel()}")
        return C.c_void_p(x.data_ptr()), N.FDE_MEM_DEVICE, x
    if _is_torch_cuda(x):
        import torch
        if x.dtype != torch.float64 or not x.is_contiguous():
            raise TypeError(f"{name}: device tensor must be contiguous float64")
        if x.numel() != count:
            raise ValueError(f"{name}: expected {count} elements, got {x.numel()}")
        return C.c_void_p(x.data_ptr()), N.FDE_MEM_DEVICE, x
    a = np.asarray(x)
    if writable:
        if a.dtype != np.float64 or not a.flags.c_contiguous or not a.flags.writeable:
            raise TypeError(f"{name}: host output must be a writable C-contiguous float64 array")
    else:
        a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != count:
        raise ValueError(f"{name}: expected {count} elements, got {a.size}")
    return C.c_void_p(a.ctypes.data), N.FDE_MEM_HOST, a


def _same_space(*spaces):
    sp = {s for s in spaces if s is not None}
    if len(sp) > 1:
        raise ValueError("all arrays of one call must be either host arrays or device tensors")
    return sp.pop() if sp else N.FDE_MEM_HOST


class BvmSolver:
    """One all-at-once BVM system: ``setup`` on construction, then ``factor`` and ``solve``.

    problem: any object with alpha, m, s, d_plus, d_minus, bvm ('trapezoidal'|'gbdf3'|'gam5')
    and optional xL, xR, t0, T (a ``workloads.Problem`` works).
    """

    def __init__(self, problem, stream=None, formula=None):
        """formula: a custom mu-step BVM (FDE_BVM_CUSTOM) given as any object with nu, mu,
        alpha, beta [mu+1], alpha_init, beta_init [nu-1][mu+1] and alpha_fin, beta_fin
        [mu-nu][mu+1]; it replaces the problem's named BVM."""
        L = N.lib()
        self.m = int(problem.m)
        self.s = int(problem.s)
        self._dp = np.ascontiguousarray(problem.d_plus, dtype=np.float64)
        self._dm = np.ascontiguousarray(problem.d_minus, dtype=np.float64)
        if self._dp.size != self.m or self._dm.size != self.m:
            raise ValueError("d_plus and d_minus must have m entries")
        kind = getattr(problem, "bvm", "gbdf3")
        custom = None
        if formula is not None:
            custom = self._custom_formula(formula)
            code = N.FDE_BVM_CUSTOM
        elif kind in _KINDS:
            code = _KINDS[kind]
        else:
            raise ValueError(f"unknown BVM {kind!r}")
        p = N.FdeProblem(float(problem.alpha), float(getattr(problem, "xL", 0.0)),
                         float(getattr(problem, "xR", 2.0)), float(getattr(problem, "t0", 0.0)),
                         float(getattr(problem, "T", 1.0)), self.m, self.s,
                         self._dp.ctypes.data_as(N._dp), self._dm.ctypes.data_as(N._dp),
                         code, C.pointer(custom) if custom is not None else None)
        h = C.c_void_p()
        N.check(L.fde_bvm_setup(C.byref(p), C.byref(h)))
        self._h = h
        dims = (C.c_int * 6)()
        N.check(L.fde_get_dims(h, dims))
        self.mu, self.nu, self.nb, self.mp = dims[2], dims[3], dims[4], dims[5]
        self.n = self.m * self.s
        self._stream_ptr = 0
        _LIVE.add(self)
        if stream is not None:
            self.set_stream(stream)

    def _custom_formula(self, F):
        nu, mu = int(F.nu), int(F.mu)
        arrs = []

        def dp(x, rows):
            if rows == 0:
                return None
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(rows, mu + 1))
            arrs.append(a)
            return a.ctypes.data_as(N._dp)
        f = N.FdeBvmFormula(nu, mu - nu, dp(F.alpha, 1), dp(F.beta, 1),
                            dp(F.alpha_init, nu - 1), dp(F.beta_init, nu - 1),
                            dp(F.alpha_fin, mu - nu), dp(F.beta_fin, mu - nu))
        self._formula_keep = arrs  # the library copies the tables during setup
        return f

    # ---- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            N.lib().fde_bvm_destroy(self._h)
            self._h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_option(self, option: int, value: int):
        N.check(N.lib().fde_bvm_set_option(self._h, int(option), int(value)))

    def get_option(self, option: int) -> int:
        v = C.c_int()
        N.check(N.lib().fde_bvm_get_option(self._h, int(option), C.byref(v)))
        return v.value

    def set_stream(self, stream):
        ptr = getattr(stream, "cuda_stream", stream)
        N.check(N.lib().fde_set_stream(self._h, C.c_void_p(ptr or 0)))
        self._stream_ptr = int(ptr or 0)

    # ---- the three calls
    def factor(self, precision: str = "fp64", preconditioner: Optional[str] = None,
               blocks: Optional[str] = None):
        """Build the preconditioner: "strang" (block LUs), "bccb" or "bccb_shifted" (2-D DFT),
        or "none".  blocks: "lu", "hessenberg", "band" or "auto" (how the blocks of "strang" are
        factored); None keeps the handle's setting."""
        if blocks is not None:
            kind = _BLOCKS[blocks]
            if self.get_option(N.FDE_OPT_BLOCKS) != kind:
                self.set_option(N.FDE_OPT_BLOCKS, kind)
        if preconditioner is not None:
            kind = _PC[preconditioner]
            if self.get_option(N.FDE_OPT_PRECOND) != kind:
                self.set_option(N.FDE_OPT_PRECOND, kind)
        N.check(N.lib().fde_precond_factor(self._h, _PREC[precision]))

    def solve(self, u0, f, x0=None, out=None, rtol: float = 1e-10, restart: int = 20,
              maxit: int = 1000, raise_on_noconv: bool = True, x0_kind: int = N.FDE_X0_SOLUTION,
              side: Optional[str] = None):
        """Returns (u [s][m], info dict).  u0 [m], f [s+1][m], x0 [s][m] or None
        (x0_kind: FDE_X0_SOLUTION, or FDE_X0_LOWRANK for a guess of (S - M) u).  side: "right"
        or "left" sets the handle's preconditioning side (None keeps it)."""
        if side is not None:
            if self.get_option(N.FDE_OPT_SIDE) != _SIDE[side]:
                self.set_option(N.FDE_OPT_SIDE, _SIDE[side])
        pu0, s1, k1 = _arg(u0, self.m, "u0")
        pf, s2, k2 = _arg(f, (self.s + 1) * self.m, "f")
        sx = None
        px0 = None
        if x0 is not None:
            px0, sx, k3 = _arg(x0, self.n, "x0")
        space = _same_space(s1, s2, sx)
        if out is None:
            out = self._alloc_like(space, (self.s, self.m), u0)
        pu, so, k4 = _arg(out, self.n, "out", writable=True)
        _same_space(space, so)
        _sync_torch_producers(self._stream_ptr, u0, f, x0, out)
        opts = N.FdeSolveOpts(float(rtol), int(restart), int(maxit), px0, space, int(x0_kind))
        info = N.FdeSolveInfo()
        st = N.lib().fde_bvm_solve(self._h, pu0, pf, pu, C.byref(opts), C.byref(info))
        if st != N.FDE_OK and (st != N.FDE_ENOCONV or raise_on_noconv):
            N.check(st)
        return out, info.as_dict()

    # ---- single steps
    def rhs(self, u0, f, out=None):
        pu0, s1, _a = _arg(u0, self.m, "u0")
        pf, s2, _b = _arg(f, (self.s + 1) * self.m, "f")
        space = _same_space(s1, s2)
        out = self._alloc_like(space, (self.s, self.m), u0) if out is None else out
        pb, _, _c = _arg(out, self.n, "out", writable=True)
        _sync_torch_producers(self._stream_ptr, u0, f, out)
        N.check(N.lib().fde_build_rhs(self._h, pu0, pf, pb, space))
        return out

    def matvec(self, z, out=None):
        pz, space, _a = _arg(z, self.n, "z")
        out = self._alloc_like(space, (self.s, self.m), z) if out is None else out
        pw, _, _b = _arg(out, self.n, "out", writable=True)
        _sync_torch_producers(self._stream_ptr, z, out)
        N.check(N.lib().fde_apply_matvec(self._h, pz, pw, space))
        return out

    def strang_apply(self, z, out=None):
        """w = S z (forward Strang block-circulant)."""
        return self._band_op(N.lib().fde_bvm_strang_apply, z, out)

    def lowrank_correction(self, z, out=None):
        """c = (S - M) z, supported on the boundary time rows."""
        return self._band_op(N.lib().fde_bvm_lowrank_correction, z, out)

    def _band_op(self, fn, z, out):
        pz, space, _a = _arg(z, self.n, "z")
        out = self._alloc_like(space, (self.s, self.m), z) if out is None else out
        pw, _, _b = _arg(out, self.n, "out", writable=True)
        _sync_torch_producers(self._stream_ptr, z, out)
        N.check(fn(self._h, pz, pw, space))
        return out

    def set_coefficients(self, alpha: float, d_plus, d_minus):
        dp = np.ascontiguousarray(d_plus, dtype=np.float64)
        dm = np.ascontiguousarray(d_minus, dtype=np.float64)
        N.check(N.lib().fde_bvm_set_coefficients(self._h, float(alpha), dp.ctypes.data_as(N._dp),
                                                  dm.ctypes.data_as(N._dp)))

    def precond(self, v, out=None):
        pv, space, _a = _arg(v, self.n, "v")
        out = self._alloc_like(space, (self.s, self.m), v) if out is None else out
        pz, _, _b = _arg(out, self.n, "out", writable=True)
        _sync_torch_producers(self._stream_ptr, v, out)
        N.check(N.lib().fde_apply_precond(self._h, pv, pz, space))
        return out

    def toeplitz(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        count = x.size // self.m
        y = np.empty_like(x)
        N.check(N.lib().fde_toeplitz_apply(self._h, C.c_void_p(x.ctypes.data),
                                            C.c_void_p(y.ctypes.data), count, N.FDE_MEM_HOST))
        return y

    def time_rfft(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        out = np.empty((self.s // 2 + 1, self.m), dtype=np.complex128)
        N.check(N.lib().fde_time_rfft(self._h, C.c_void_p(v.ctypes.data),
                                       C.c_void_p(out.ctypes.data), N.FDE_MEM_HOST))
        return out

    def hessenberg(self):
        """(H, Q) of J = Q H Q^T from a FDE_BLOCKS_HESSENBERG factorization."""
        H = np.empty((self.m, self.m))
        Q = np.empty((self.m, self.m))
        N.check(N.lib().fde_get_hessenberg(self._h, C.c_void_p(H.ctypes.data), C.c_void_p(Q.ctypes.data)))
        return H, Q

    def factor_block(self, k: int) -> np.ndarray:
        out = np.empty((self.m, self.m), dtype=np.complex128)
        N.check(N.lib().fde_get_factor_block(self._h, int(k), C.c_void_p(out.ctypes.data)))
        return out

    # ---- timing
    def profile(self, enable: bool = True):
        N.check(N.lib().fde_profile_enable(self._h, 1 if enable else 0))

    def profile_query(self, name: str):
        ms, cnt, work = C.c_double(), C.c_int(), C.c_double()
        N.check(N.lib().fde_profile_query(self._h, name.encode(), C.byref(ms), C.byref(cnt),
                                           C.byref(work)))
        return {"total_ms": ms.value, "count": cnt.value, "work": work.value}

    @staticmethod
    def _alloc_like(space, shape, like):
        if isinstance(like, DeviceArray):
            return DeviceArray(shape)
        if space == N.FDE_MEM_DEVICE:
            import torch
            return torch.empty(shape, dtype=torch.float64, device=like.device)
        return np.empty(shape, dtype=np.float64)


def autotune_report() -> str:
    """The autotuner's choices so far, "shape=W;...;shape/tfft=cols;..."."""
    buf = C.create_string_buffer(1 << 20)
    N.check(N.lib().fde_autotune_report(buf, len(buf)))
    return buf.value.decode()


def factor_batch(solvers, precision: str = "fp64"):
    """fde_precond_factor_batch: one launch per LU phase over the blocks of all solvers."""
    count = len(solvers)
    hs = (C.c_void_p * count)(*[s.handle for s in solvers])
    N.check(N.lib().fde_precond_factor_batch(hs, count, _PREC[precision]))


def solve_batch(solvers, u0s, fs, rtol: float = 1e-10, restart: int = 20, maxit: int = 1000,
                outs=None, x0s=None, raise_on_noconv: bool = True, x0_kind: int = N.FDE_X0_SOLUTION):
    """fde_bvm_solve_batch (or _x0 when x0s is given) over factored solvers; returns (outs, infos)."""
    count = len(solvers)
    if outs is None:
        outs = [BvmSolver._alloc_like(_arg(u, s.m, "u0")[1], (s.s, s.m), u)
                for s, u in zip(solvers, u0s)]
    keep = []
    hs = (C.c_void_p * count)(*[s.handle for s in solvers])
    pu0 = (C.c_void_p * count)()
    pf = (C.c_void_p * count)()
    pu = (C.c_void_p * count)()
    px0 = (C.c_void_p * count)()
    spaces = []
    for i, s in enumerate(solvers):
        a, sa, ka = _arg(u0s[i], s.m, "u0")
        b, sb, kb = _arg(fs[i], (s.s + 1) * s.m, "f")
        c, sc, kc = _arg(outs[i], s.n, "out", writable=True)
        keep += [ka, kb, kc]
        spaces += [sa, sb, sc]
        pu0[i], pf[i], pu[i] = a, b, c
        if x0s is not None and x0s[i] is not None:
            d, sd, kd = _arg(x0s[i], s.n, "x0")
            keep.append(kd)
            spaces.append(sd)
            px0[i] = d
    space = _same_space(*spaces)
    _sync_torch_producers(solvers[0]._stream_ptr if count else 0, *keep)
    opts = N.FdeSolveOpts(float(rtol), int(restart), int(maxit), None, space, int(x0_kind))
    infos = (N.FdeSolveInfo * count)()
    if x0s is None:
        st = N.lib().fde_bvm_solve_batch(hs, count, pu0, pf, pu, C.byref(opts), infos)
    else:
        st = N.lib().fde_bvm_solve_batch_x0(hs, count, pu0, pf, px0, pu, C.byref(opts), infos)
    if st != N.FDE_OK and (st != N.FDE_ENOCONV or raise_on_noconv):
        N.check(st)
    return outs, [i.as_dict() for i in infos]
