"""Learned warm start for the all-at-once solve: data generation with the solver itself,
training with the library's own GPU forward/backward kernels, and evaluation of the
iterations and time it saves against zero-start GMRES.

Tensors are torch device buffers (allocation only); every computation runs in
libfdebvm.so.  The trained network only proposes x0; the solve still stops on the true
FP64 residual, so the warm start changes cost, never the answer.
"""
from __future__ import annotations

import ctypes as C
import sys
import time
from typing import Optional, Sequence

import numpy as np

from . import _native as N
from .solver import BvmSolver, factor_batch, solve_batch


class WarmStartNet:
    """ctypes wrapper of fde_nn_* (see the warm-start section of include/fdebvm.h)."""

    def __init__(self, m: int = 255, s: int = 128, max_batch: int = 64, conv_ch=(96, 96, 64),
                 fc=(768, 512), nx: int = 32, nt: int = 16, seed: int = 0):
        L = N.lib()
        self.cfg = N.FdeNnConfig(m, s, max_batch, (C.c_int * 3)(*conv_ch), (C.c_int * 2)(*fc), nx, nt, seed)
        self.m, self.s, self.max_batch = m, s, max_batch
        self.cin = s + 4
        h = C.c_void_p()
        N.check_nn(L.fde_nn_create(C.byref(self.cfg), C.byref(h)))
        self._h = h
        cnt = C.c_longlong()
        N.check_nn(L.fde_nn_num_params(h, C.byref(cnt)))
        self.num_params = cnt.value

    def close(self):
        if getattr(self, "_h", None):
            N.lib().fde_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # ---- parameters and optimiser state (host FP32 arrays)
    def get(self, which: int = 0) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        N.check_nn(N.lib().fde_nn_get_params(self._h, C.c_void_p(out.ctypes.data), which))
        return out

    def set_params(self, theta: np.ndarray):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        assert theta.size == self.num_params
        N.check_nn(N.lib().fde_nn_set_params(self._h, C.c_void_p(theta.ctypes.data)))

    def set_state(self, m1: np.ndarray, m2: np.ndarray, step: int):
        m1 = np.ascontiguousarray(m1, dtype=np.float32)
        m2 = np.ascontiguousarray(m2, dtype=np.float32)
        N.check_nn(N.lib().fde_nn_set_state(self._h, C.c_void_p(m1.ctypes.data),
                                            C.c_void_p(m2.ctypes.data), int(step)))

    @property
    def step(self) -> int:
        v = C.c_int()
        N.check_nn(N.lib().fde_nn_get_step(self._h, C.byref(v)))
        return v.value

    def checkpoint(self) -> dict:
        return {"params": self.get(0), "m1": self.get(2), "m2": self.get(3), "step": self.step}

    def restore(self, ck: dict):
        self.set_params(ck["params"])
        self.set_state(ck["m1"], ck["m2"], ck["step"])

    # ---- device work
    def features(self, fs, dps, dms, alphas, X, rms, row0: int = 0):
        """Features of len(fs) instances into rows row0.. of X [N][256][cin] and rms [N]
        (torch float32 device tensors); fs/dps/dms are FP64 device tensors."""
        B = len(fs)
        arr = lambda ts: (C.c_void_p * B)(*[t.data_ptr() for t in ts])
        al = np.ascontiguousarray(alphas, dtype=np.float64)
        N.check_nn(N.lib().fde_nn_features(
            self._h, B, arr(fs), arr(dps), arr(dms), al.ctypes.data_as(N._dp),
            C.c_void_p(X.data_ptr() + row0 * X.stride(0) * 4), C.c_void_p(rms.data_ptr() + row0 * 4)))

    def loss_grad(self, X, T, rms, idx: Optional[np.ndarray], B: int) -> float:
        loss = C.c_float()
        pidx = None
        if idx is not None:
            idx = np.ascontiguousarray(idx, dtype=np.int32)
            pidx = idx.ctypes.data_as(C.POINTER(C.c_int))
        N.check_nn(N.lib().fde_nn_loss_grad(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                            C.c_void_p(rms.data_ptr()), pidx, int(B), C.byref(loss)))
        return loss.value

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        N.check_nn(N.lib().fde_nn_adam(self._h, lr, beta1, beta2, eps))

    def predict(self, X, rms, idx: Optional[np.ndarray], outs):
        B = len(outs)
        pidx = None
        if idx is not None:
            idx = np.ascontiguousarray(idx, dtype=np.int32)
            pidx = idx.ctypes.data_as(C.POINTER(C.c_int))
        po = (C.c_void_p * B)(*[o.data_ptr() for o in outs])
        N.check_nn(N.lib().fde_nn_predict(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(rms.data_ptr()),
                                          pidx, B, po))

    def set_basis(self, basis: np.ndarray):
        basis = np.ascontiguousarray(basis, dtype=np.float32)
        assert basis.shape == (self.cfg.nx * self.cfg.nt, self.s * self.m)
        N.check_nn(N.lib().fde_nn_set_basis(self._h, C.c_void_p(basis.ctypes.data)))

    def use_boundary_rows(self, rows: Sequence[int]):
        """Output = scatter of nt = len(rows) rows of nx = m values onto those time rows."""
        assert self.cfg.nt == len(rows) and self.cfg.nx == self.m
        basis = np.zeros((len(rows) * self.m, self.s * self.m), dtype=np.float32)
        for q, r in enumerate(rows):
            for p in range(self.m):
                basis[q * self.m + p, r * self.m + p] = 1.0
        self.set_basis(basis)

    def output(self, B: int) -> np.ndarray:
        out = np.empty((B, self.s * self.m), dtype=np.float32)
        N.check_nn(N.lib().fde_nn_output(self._h, C.c_void_p(out.ctypes.data), B))
        return out


class InstancePool:
    """A fixed set of solver handles (same m, s, formula) re-targeted per instance with
    fde_bvm_set_coefficients, so that many instances reuse one allocation."""

    def __init__(self, template, size: int):
        self.solvers = [BvmSolver(template) for _ in range(size)]

    def load(self, problems):
        for S, p in zip(self.solvers, problems):
            dp = np.ascontiguousarray(p.d_plus, dtype=np.float64)
            dm = np.ascontiguousarray(p.d_minus, dtype=np.float64)
            N.check(N.lib().fde_bvm_set_coefficients(S.handle, float(p.alpha), dp.ctypes.data_as(N._dp),
                                                      dm.ctypes.data_as(N._dp)))
        return self.solvers[:len(problems)]

    def close(self):
        for S in self.solvers:
            S.close()


def _device(arr, torch, dev):
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64)).to(dev)


def boundary_rows(nu: int, mu: int, s: int):
    """Time rows (s-form) where S and M differ: the nu initial and mu - nu final rows."""
    return list(range(nu)) + list(range(s - (mu - nu), s))


def build_dataset(seeds: Sequence[int], net: WarmStartNet, make_problem, batch: int = 64,
                  precision: str = "fp64", log=None, target: str = "solution"):
    """Solve every seeded instance with the plain method (zero start) and build the features.
    target "solution": T = u; target "lowrank": T = c = (S - M) u (boundary rows only).
    Returns dict(X, rms, T (FP64 [N][s][m]), iters, seconds)."""
    import torch
    dev = torch.device("cuda:0")
    n = len(seeds)
    X = torch.zeros((n, 256, net.cin), dtype=torch.float32, device=dev)
    rms = torch.zeros(n, dtype=torch.float32, device=dev)
    T = torch.zeros((n, net.s, net.m), dtype=torch.float64, device=dev)
    iters = np.zeros(n, dtype=np.int32)
    pool = InstancePool(make_problem(seeds[0]), min(batch, n))
    t0 = time.perf_counter()
    for b0 in range(0, n, batch):
        ps = [make_problem(sd) for sd in seeds[b0:b0 + batch]]
        Ss = pool.load(ps)
        factor_batch(Ss, precision)
        u0s = [_device(p.u0, torch, dev) for p in ps]
        fs = [_device(p.f, torch, dev) for p in ps]
        outs = [T[b0 + i] for i in range(len(ps))]
        _, infos = solve_batch(Ss, u0s, fs, outs=outs)
        if target == "lowrank":
            for S_, o in zip(Ss, outs):
                S_.lowrank_correction(o, out=o)
        iters[b0:b0 + len(ps)] = [i["iters"] for i in infos]
        net.features(fs, [_device(p.d_plus, torch, dev) for p in ps],
                     [_device(p.d_minus, torch, dev) for p in ps], [p.alpha for p in ps], X, rms, row0=b0)
        if log and (b0 // batch) % 50 == 0:
            log(f"dataset {b0 + len(ps)}/{n} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    pool.close()
    return {"X": X, "rms": rms, "T": T, "iters": iters, "seconds": time.perf_counter() - t0}


def train(net: WarmStartNet, data: dict, epochs: int = 20, batch: int = 64, lr: float = 1e-3,
          seed: int = 0, log=None, lr_decay: float = 0.9):
    """Adam on the relative-MSE loss; returns the per-epoch mean training loss."""
    rng = np.random.default_rng(seed)
    n = data["X"].shape[0]
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(n).astype(np.int32)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            tot += net.loss_grad(data["X"], data["T"], data["rms"], idx, batch)
            net.adam(lr)
            cnt += 1
        hist.append(tot / max(cnt, 1))
        lr *= lr_decay
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return hist


def evaluate(net: WarmStartNet, seeds: Sequence[int], make_problem, batch: int = 64,
             precision: str = "fp64", target: str = "solution", gate: Optional[int] = None):
    """GMRES iterations and solve time to rel-res 1e-10 with zero start and with the network's
    guess (inference time included), per instance, on the same batched solver.  With target
    "lowrank" the guess is c ~ (S - M) u and the solve starts from S^{-1}(b + c).  gate: the
    solver's FDE_OPT_X0_GATE for the warm-started solves (None: the library default; 0 keeps
    every guess); x0_kept records which guesses passed it."""
    import torch
    dev = torch.device("cuda:0")
    n = len(seeds)
    pool = InstancePool(make_problem(seeds[0]), min(batch, n))
    X = torch.zeros((min(batch, n), 256, net.cin), dtype=torch.float32, device=dev)
    rms = torch.zeros(min(batch, n), dtype=torch.float32, device=dev)
    res = {"iters_zero": [], "iters_warm": [], "ms_zero": 0.0, "ms_warm": 0.0, "ms_nn": 0.0,
           "rel_err_x0": [], "relres_warm": [], "relres_zero": [], "x0_kept": []}
    for b0 in range(0, n, batch):
        ps = [make_problem(sd) for sd in seeds[b0:b0 + batch]]
        Ss = pool.load(ps)
        if gate is not None:
            for S in Ss:
                S.set_option(N.FDE_OPT_X0_GATE, gate)
        factor_batch(Ss, precision)
        u0s = [_device(p.u0, torch, dev) for p in ps]
        fs = [_device(p.f, torch, dev) for p in ps]
        outs0 = [torch.empty((p.s, p.m), dtype=torch.float64, device=dev) for p in ps]
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, inf0 = solve_batch(Ss, u0s, fs, outs=outs0)
        torch.cuda.synchronize()
        res["ms_zero"] += (time.perf_counter() - t) * 1e3
        dps = [_device(p.d_plus, torch, dev) for p in ps]
        dms = [_device(p.d_minus, torch, dev) for p in ps]
        x0s = [torch.empty((p.s, p.m), dtype=torch.float64, device=dev) for p in ps]
        outs1 = [torch.empty((p.s, p.m), dtype=torch.float64, device=dev) for p in ps]
        torch.cuda.synchronize()
        t = time.perf_counter()
        net.features(fs, dps, dms, [p.alpha for p in ps], X, rms)
        net.predict(X, rms, None, x0s)
        torch.cuda.synchronize()
        t_nn = time.perf_counter()
        kind = N.FDE_X0_LOWRANK if target == "lowrank" else N.FDE_X0_SOLUTION
        _, inf1 = solve_batch(Ss, u0s, fs, outs=outs1, x0s=x0s, x0_kind=kind)
        torch.cuda.synchronize()
        res["ms_warm"] += (time.perf_counter() - t) * 1e3
        res["ms_nn"] += (t_nn - t) * 1e3
        for i in range(len(ps)):
            res["iters_zero"].append(inf0[i]["iters"])
            res["iters_warm"].append(inf1[i]["iters"])
            res["relres_zero"].append(inf0[i]["true_relres"])
            res["relres_warm"].append(inf1[i]["true_relres"])
            res["x0_kept"].append(Ss[i].get_option(N.FDE_OPT_X0_KEPT))
            ref = outs0[i]
            if target == "lowrank":
                ref = Ss[i].lowrank_correction(ref)
            u = ref.cpu().numpy()
            x0 = x0s[i].cpu().numpy()
            res["rel_err_x0"].append(float(np.linalg.norm(x0 - u) / np.linalg.norm(u)))
    pool.close()
    return res
