#!/usr/bin/env python3
"""Benchmark: ms per all-at-once solve to true rel-res 1e-10 (reported as solves/s).

One step = fde_precond_factor + fde_bvm_solve on the 4,095 x 256 GBDF3 workload
(alpha = 1.3, seeded smooth random data, 1,048,320 unknowns) with u0 and f already
resident in HBM.  Prints ONE JSON line.  The plain FP64 form is the headline value;
the mixed form (complex-FP32 blocks inside flexible GMRES) is reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c2|c3|c4|ex41]
                    [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per all-at-once solve to rel-res 1e-10 (solves/s); mixed vs plain FP64"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (separate runs),
# each scaled by the same counter's reading for a plain device-to-device copy of known size.
# Keyed by (workload, precision, kernel).  A figure is valid only while the sources of its
# kernel's group hash to the value recorded with it; otherwise "traffic" is reported as null.
PMC_GROUPS = {
    "factor": ("k_factor.hip", "common.hpp", "batch.hpp"),
    "spacetime": ("k_spacetime.hip", "fft_lds.hpp", "common.hpp", "batch.hpp"),
    "krylov": ("k_krylov.hip", "common.hpp", "batch.hpp"),
    "hessenberg": ("k_hessenberg.hip", "common.hpp", "batch.hpp"),
    "band": ("k_band.hip", "common.hpp", "batch.hpp"),
}
PMC_KERNEL_GROUP = {
    "assemble": "factor", "lu_diag": "factor", "lu_panel": "factor", "lu_update": "factor",
    "trsv": "factor", "hess_uinv": "factor",
    "bvm_matvec": "spacetime", "time_rfft": "spacetime", "time_irfft": "spacetime",
    "bccb_solve": "spacetime", "rhs": "spacetime",
    "mgs": "krylov", "cgs": "krylov", "arnoldi": "krylov", "normalize": "krylov", "residual": "krylov",
    "update_x": "krylov", "dot": "krylov",
    "hess_reduce": "hessenberg", "hess_lu": "hessenberg", "qgemm": "hessenberg",
    "hess_lsolve": "hessenberg",
    "band_panel": "band", "band_update": "band", "band_init": "band", "band_finish": "band",
    "band_lu_panel": "factor", "band_lu_rows": "factor", "band_lu_step": "factor", "band_lsolve": "factor",
}
# Per measured workload: the source hashes of every kernel group when its counters were taken,
# and the bytes per launch.  Workload keys: the bench workload, plus a route letter for the
# routes compared beside the headline ("c2h": Hessenberg route at 1023x512, "c3l": block-LU
# route at 4095x256; "c3" itself is the band route, the default there).
PMC_MEASURED = {
    "c2": {"hash": {"factor": "c53d9b1c3810c0bd", "spacetime": "41b6c6d79eb78c42", "krylov": "a336f5b3ef0ee3cb"},
           "bytes": {
               ("fp64", "assemble"): 1.0112e+09, ("fp64", "bccb_solve"): 9.3250e+06,
               ("fp64", "bvm_matvec"): 2.1818e+07, ("fp64", "lu_diag"): 6.7648e+07,
               ("fp64", "lu_panel"): 5.7406e+08, ("fp64", "lu_update"): 1.8857e+09,
               ("fp64", "mgs"): 1.5971e+07, ("fp64", "normalize"): 8.5660e+06,
               ("fp64", "time_irfft"): 8.6140e+06, ("fp64", "time_rfft"): 8.9990e+06,
               ("fp64", "trsv"): 4.4729e+09,
               ("mixed", "assemble"): 5.0574e+08, ("mixed", "lu_diag"): 3.3814e+07,
               ("mixed", "lu_panel"): 2.9044e+08, ("mixed", "lu_update"): 8.5514e+08,
               ("mixed", "trsv"): 2.6343e+09}},
    "c2h": {"hash": {"factor": "c53d9b1c3810c0bd", "hessenberg": "cf0e655e99339546"},
            "bytes": {
                ("fp64", "hess_lsolve"): 1.3739e+07, ("fp64", "hess_lu"): 2.2026e+09,
                ("fp64", "hess_reduce"): 6.8204e+09, ("fp64", "hess_uinv"): 4.2120e+08,
                ("fp64", "qgemm"): 5.2862e+07, ("fp64", "trsv"): 2.2364e+09,
                ("mixed", "hess_lsolve"): 1.3739e+07, ("mixed", "hess_lu"): 1.1253e+09,
                ("mixed", "hess_reduce"): 6.8204e+09, ("mixed", "hess_uinv"): 2.1905e+08,
                ("mixed", "qgemm"): 5.2862e+07, ("mixed", "trsv"): 1.3156e+09}},
    # profiles/hbm_traffic_m4095_s256_gbdf3.txt
    "c3": {"hash": {"factor": "da95ccf4032e6e85", "spacetime": "7d1eafc888daca2c", "krylov": "5584998f77183f5e",
                    "hessenberg": "6ab681476fb4a268", "band": "6851e166aa9f8d8b"},
           "bytes": {
               ("fp64", "trsv"): 1.7687e+10, ("fp64", "band_lu_step"): 9.8122e+08,
               ("fp64", "band_lu_rows"): 4.2619e+07, ("fp64", "band_lu_panel"): 3.4665e+07,
               ("fp64", "band_lsolve"): 1.0948e+09, ("fp64", "qgemm"): 2.1053e+08,
               ("fp64", "band_panel"): 1.4629e+07, ("fp64", "band_init"): 2.6943e+08,
               ("fp64", "mgs"): 3.1258e+07, ("fp64", "bvm_matvec"): 1.9734e+07,
               ("fp64", "time_rfft"): 1.7079e+07, ("fp64", "time_irfft"): 1.6881e+07,
               ("fp64", "normalize"): 1.6917e+07, ("mixed", "trsv"): 9.3656e+09,
               ("mixed", "band_lu_step"): 6.9877e+08, ("mixed", "band_lu_rows"): 2.1533e+07,
               ("mixed", "band_lu_panel"): 1.7741e+07, ("mixed", "band_lsolve"): 5.5800e+08,
               ("mixed", "qgemm"): 2.1053e+08, ("mixed", "band_panel"): 1.4629e+07,
               ("mixed", "band_init"): 2.6943e+08}},
    "c3l": {"hash": {"factor": "da95ccf4032e6e85", "spacetime": "7d1eafc888daca2c", "krylov": "5584998f77183f5e"},
           "bytes": {
               ("fp64", "lu_update"): 2.2898e+10, ("fp64", "trsv"): 3.5387e+10,
               ("fp64", "lu_panel"): 1.1004e+09, ("fp64", "lu_diag"): 3.4090e+07,
               ("fp64", "assemble"): 2.1333e+09, ("mixed", "lu_update"): 9.5230e+09,
               ("mixed", "trsv"): 1.8712e+10, ("mixed", "lu_panel"): 6.3364e+08,
               ("mixed", "lu_diag"): 1.7037e+07, ("mixed", "assemble"): 1.0673e+09}},
}


def group_source_hash(group: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in PMC_GROUPS[group]:
        with open(os.path.join(ROOT, "paper_1305_6653_amd", "csrc", name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, prec, kernel):
    """HBM bytes per launch of the kernel, or None when it was not measured for this workload,
    route and form, or its group's sources have changed since."""
    rec = PMC_MEASURED.get(workload_name)
    group = PMC_KERNEL_GROUP.get(kernel)
    if rec is None or group is None or rec["hash"].get(group) != group_source_hash(group):
        return None
    return rec["bytes"].get((prec, kernel))


_MFMA_PEAK = {}


def measured_mfma_peak(prec):
    """Matrix-core rate on this GPU, TFLOP/s: the library's probe of back-to-back 16x16x4 MFMAs
    (FP64, or FP32 for the mixed form; best of 5), outside the timed region."""
    if prec not in _MFMA_PEAK:
        import ctypes as C
        from paper_1305_6653_amd import _native as N
        v = C.c_double()
        N.check(N.lib().fde_mfma_peak_probe(1 if prec == "fp64" else 0, 5, C.byref(v)))
        _MFMA_PEAK[prec] = round(v.value, 2)
    return _MFMA_PEAK[prec]


FLOP_KERNELS = ("lu_diag", "lu_panel", "lu_update", "hess_lu", "hess_reduce", "hess_uinv",
                "band_panel", "band_update", "band_lu_panel", "band_lu_rows", "band_lu_step", "qgemm")


def kernel_table(prof, steps, prec):
    """Per kernel and step: time, launches, average launch, and the algorithmic rate of its
    launches (bytes or flops recorded by the library per launch) as a fraction of the roofline
    that bounds it (HBM 8 TB/s; FP64 or FP32 for the flop kernels, in the precision they run in)."""
    out = {}
    for k, v in prof.items():
        row = {"total_ms": round(v["total_ms"] / steps, 4), "count": v["count"] // steps,
               "avg_us": round(1e3 * v["total_ms"] / max(1, v["count"]), 2)}
        if v.get("work") and v["total_ms"] > 0:
            rate = v["work"] / (v["total_ms"] * 1e-3)
            if k in FLOP_KERNELS:
                fp32 = k in ("lu_diag", "lu_panel", "lu_update", "band_lu_rows", "band_lu_panel", "band_lu_step",
                             "hess_lu", "hess_uinv")
                peak = PEAK_FP32_TFLOPS if (prec == "mixed" and fp32) else PEAK_FP64_TFLOPS
                row["TFLOPs"] = round(rate / 1e12, 3)
                row["frac"] = round(rate / 1e12 / peak, 4)
            else:
                row["GBs"] = round(rate / 1e9, 1)
                row["frac"] = round(rate / 1e9 / PEAK_HBM_GBS, 4)
        out[k] = row
    return out


def measured_read_peak():
    """Achievable HBM read bandwidth on this GPU, GB/s: the library's streaming-read probe over
    4 GiB (best of 5), outside the timed region.  Context for the datasheet peak."""
    import ctypes as C
    from paper_1305_6653_amd import _native as N
    v = C.c_double()
    N.check(N.lib().fde_read_bandwidth_probe(4 << 30, 5, C.byref(v)))
    return round(v.value, 1)


class DeviceMemory:
    """Where the benchmark keeps its device arrays: torch CUDA tensors (default), or the
    library's own device buffers (``library``: no torch in the process, so a profiler that
    preloads the system HIP runtime sees the only runtime the process maps)."""

    def __init__(self, kind):
        self.kind = kind
        if kind == "library":
            os.environ["FDE_NO_TORCH"] = "1"

    def put(self, a):
        import numpy as np
        if self.kind == "library":
            from paper_1305_6653_amd.devmem import DeviceArray
            return DeviceArray.from_numpy(a)
        import torch
        return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")

    def empty(self, shape):
        if self.kind == "library":
            from paper_1305_6653_amd.devmem import DeviceArray
            return DeviceArray(shape)
        import torch
        return torch.empty(shape, dtype=torch.float64, device="cuda:0")

    def get(self, d):
        return d.numpy().copy() if self.kind == "library" else d.cpu().numpy().copy()

    def sync(self):
        if self.kind == "library":
            from paper_1305_6653_amd.devmem import synchronize
            synchronize()
        else:
            import torch
            torch.cuda.synchronize()

    def stream(self):
        if self.kind == "library":
            return None
        import torch
        return torch.cuda.current_stream()

    def calib_copy(self, mib):
        """One plain device-to-device copy of mib MiB (a blit dispatch) outside the timed region."""
        if mib <= 0:
            return
        if self.kind == "library":
            from paper_1305_6653_amd.devmem import DeviceArray
            a, b = DeviceArray(mib << 17), DeviceArray(mib << 17)   # 8-byte elements
            self.sync()
            b.copy_from(a)
            self.sync()
            a.free()
            b.free()
            return
        import torch
        a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b


DEV = DeviceMemory("torch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "ex41"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-hessenberg", action="store_true",
                    help="skip the solves with the blocks factored through a Hessenberg form of J")
    ap.add_argument("--no-bccb", action="store_true",
                    help="skip the BCCB-preconditioned solves reported beside the main one")
    ap.add_argument("--device-memory", default="torch", choices=["torch", "library"],
                    help="hold the device arrays in torch tensors or in the library's own buffers "
                         "(library: torch is not imported)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed steps, run one plain device-to-device copy of this many MiB "
                         "(the reference dispatch for scaling FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def workload(name):
    import workloads as W
    if name == "c1":
        return W.manufactured_c1()
    if name == "c2":
        return W.smooth_c2()
    return W.smooth_c3()


def workload_alt(name):
    """A second right-hand side of the same recipe and sizes (another seed)."""
    import workloads as W
    p = workload(name)
    if name == "c1":   # analytic: the same source with a scaled initial value
        q = W.manufactured_c1()
        q.u0 = 0.5 * q.u0
        q.name = p.name + "_u0x0.5"
        return q
    return W.smooth_random(p.m, p.s, p.alpha, {"c2": 2, "c3": 3}[name] + 100)


def timed_steps(S, u0, f, out, prec, steps, warmup, pc=None):
    """W warmup steps, then K timed steps (the value), then the same K steps again with every
    launch bracketed by HIP events on the library's stream (the per-kernel profile: the
    events cost a few microseconds per launch, so they are kept out of the first pass)."""
    for _ in range(warmup):
        S.factor(prec, pc)
        S.solve(u0, f, out=out, rtol=1e-10)
    DEV.sync()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        S.factor(prec, pc)
        _, info = S.solve(u0, f, out=out, rtol=1e-10)
        infos.append(info)
    DEV.sync()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    S.profile(True)
    DEV.sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        S.factor(prec, pc)
        S.solve(u0, f, out=out, rtol=1e-10)
    DEV.sync()
    ms_prof = (time.perf_counter() - t0) * 1e3 / steps
    prof = {}
    for k in ("assemble", "lu_diag", "lu_panel", "lu_update", "trsv", "bccb_solve", "time_rfft",
              "time_irfft", "bvm_matvec", "mgs", "cgs", "arnoldi", "normalize", "residual", "update_x", "rhs", "dot",
              "hess_reduce", "hess_formq", "hess_lu", "hess_uinv", "qgemm", "hess_lsolve",
              "band_init", "band_panel", "band_update", "band_finish", "band_lu_panel", "band_lu_rows",
              "band_lu_step", "band_lsolve"):
        q = S.profile_query(k)
        if q["count"]:
            prof[k] = q
    S.profile(False)
    return ms, ms_prof, infos, prof


def roofline(prof, prec, workload_name=None, read_peak=None):
    """Dominant kernel (largest total time) with its algorithmic work rate."""
    if not prof:
        return None
    name, q = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    avg_ms = q["total_ms"] / q["count"]
    traffic = measured_traffic(workload_name, prec, name)
    if name.startswith("hess_") or name in ("band_panel", "band_lu_panel"):
        # the Hessenberg reduction, the shifted LUs and the band panels: flops on the vector ALUs
        # in chains of dependent steps (latency-bound), priced against the vector peak of the
        # precision they run in (the reductions are FP64 in either form)
        achieved = q["work"] / (q["total_ms"] * 1e-3) / 1e12
        fp32 = prec == "mixed" and name in ("hess_lu", "hess_uinv", "band_lu_panel")
        peak = PEAK_FP32_TFLOPS if fp32 else PEAK_FP64_TFLOPS
        return {"kernel": name, "bound": "alu", "achieved": round(achieved, 4),
                "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 5),
                "traffic": traffic, "avg_launch_ms": round(avg_ms, 4), "launches": q["count"],
                "work_per_launch": q["work"] / q["count"]}
    if name in FLOP_KERNELS:
        achieved = q["work"] / (q["total_ms"] * 1e-3) / 1e12
        # the band reduction is FP64 in either form; the band LU runs in the factor precision
        peak = PEAK_FP64_TFLOPS if (prec == "fp64" or name in ("band_update", "qgemm")) else PEAK_FP32_TFLOPS
        out = {"kernel": name, "bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
               "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
               "avg_launch_ms": round(avg_ms, 4), "launches": q["count"],
               "work_per_launch": q["work"] / q["count"]}
        if name in ("lu_update", "lu_panel", "band_lu_rows", "band_lu_step"):
            # the work is counted as 8 real flops per complex multiply-add; the 3M form of the
            # complex GEMM issues 3 real MFMA products per complex one, i.e. 6 of those 8 flops
            out["mfma_executed_frac"] = round(0.75 * achieved / peak, 4)
            mp = measured_mfma_peak(prec)
            out["measured_mfma_peak"] = mp
            out["mfma_executed_frac_of_measured_peak"] = round(0.75 * achieved / mp, 4)
        return out
    achieved = q["work"] / (q["total_ms"] * 1e-3) / 1e9
    out = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
           "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
           "avg_launch_ms": round(avg_ms, 4), "launches": q["count"],
           "work_per_launch": q["work"] / q["count"]}
    if read_peak:
        out["measured_read_peak"] = read_peak
        out["frac_of_measured_read_peak"] = round(achieved / read_peak, 4)
    return out


def _median_time(fn, reps=3):
    import numpy as np
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def _oracle_pieces(p, nblk, reps):
    """Times of the oracle's own operations on this workload.  Block factorization: the
    expression StrangPreconditioner evaluates per block, scipy lu_factor(lambda_k I - tau mu_k J),
    on nblk blocks spread over the spectrum (mean of their medians); block solve: its lu_solve,
    taken in turn over the nblk factors so that each solve reads its factor from memory as an
    apply over all blocks does; plus the time rfft + irfft of an apply, the dense-J product
    apply_M and one dot + axpy pair of the Arnoldi step (medians of `reps`)."""
    import numpy as np
    import scipy.linalg
    import oracle as O
    J, F, tau, _ = O.problem_matrices(p)
    A, B, _, _, _ = O.s_form(F, p.s)
    lam, mu = O.strang_eigs(F, p.s)
    nb = p.s // 2 + 1
    ks = sorted({int(round(i * (nb - 1) / max(1, nblk - 1))) for i in range(nblk)})
    rng = np.random.default_rng(0)
    n = p.s * p.m
    eye = np.eye(p.m)
    t_lu, lus = [], []
    for k in ks:
        box = [None]

        def fac():
            box[0] = scipy.linalg.lu_factor(lam[k] * eye - tau * mu[k] * J, check_finite=False)
        t_lu.append(_median_time(fac, reps))
        lus.append(box[0])
    rhs = rng.standard_normal((len(ks), p.m)) + 1j * rng.standard_normal((len(ks), p.m))
    t_sol = []
    for _ in range(reps):
        t0 = time.perf_counter()
        for lu, r in zip(lus, rhs):
            scipy.linalg.lu_solve(lu, r, check_finite=False)
        t_sol.append((time.perf_counter() - t0) / len(ks))
    del lus
    V = rng.standard_normal((p.s, p.m))
    t_fft = _median_time(lambda: np.fft.irfft(np.fft.rfft(V, axis=0), n=p.s, axis=0), reps)
    t_mv = _median_time(lambda: O.apply_M(J, A, B, tau, V), reps)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    t_mgs = _median_time(lambda: y - (x @ y) * x, reps)
    return float(np.mean(t_lu)), float(np.median(t_sol)), t_fft, t_mv, t_mgs, len(ks)


def cpu_baseline(p, iters, restarts):
    """The oracle (scipy/numpy FP64, textbook GMRES with LAPACK block solves) on the host cores,
    on a bounded sample of the same workload scaled to one whole solve: its per-block LU and
    block solve timed on a sample of the s/2+1 blocks, its time FFTs, dense-J product and Arnoldi
    vector operations timed in full (median of 3 each), combined as one solve takes them:
    (s/2+1) block LUs, then per GMRES iteration one preconditioner apply (time FFT pair and
    s/2+1 block solves), one product with M and j dot/axpy pairs at step j, plus one product
    with M per restart for the true residual.  `iters` is the GPU's FP64 count (equal to the
    oracle's within one, tested).  Also the same at one BLAS thread (one sampled block)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    nb = p.s // 2 + 1
    R = 20
    steps = sum((j % R) + 1 for j in range(iters))   # Arnoldi step j (in its cycle) has j+1 pairs

    def model(t):
        t_lu, t_sol, t_fft, t_mv, t_mgs = t
        return nb * t_lu + iters * (t_fft + nb * t_sol + t_mv) + steps * t_mgs + (restarts + 1) * t_mv

    # enough sampled blocks that their factors (16 m^2 bytes each) exceed 1 GB, or all of them
    nblk = min(nb, max(3, -(-10 ** 9 // (16 * p.m * p.m))))
    t_all = time.perf_counter()
    pieces = _oracle_pieces(p, nblk, 3)
    full = model(pieces[:5])
    t_sample = time.perf_counter() - t_all
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        pieces1 = _oracle_pieces(p, 1 if p.m > 2048 else 3, 1)
        t_sample1 = time.perf_counter() - t1
    one = model(pieces1[:5])
    model_name = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model_name = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    sample = (f"oracle pieces of the m={p.m}, s={p.s} {p.bvm} workload, median of 3 each: LAPACK "
              f"block LU and block solve on {pieces[5]} of the {nb} blocks, time rfft+irfft, dense-J "
              f"product with M, Arnoldi dot/axpy; scaled to one solve of {iters} iterations, "
              f"{restarts + 1} true residuals ({t_sample:.1f} s of sampling)")
    return {"value": round(1.0 / full, 5), "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": sample, "seconds_per_solve": round(full, 3),
            "factor_seconds": round(nb * pieces[0], 3),
            "one_thread": {"value": round(1.0 / one, 6), "seconds_per_solve": round(one, 2), "cores": 1,
                           "sample": f"as above at one BLAS thread, {pieces1[5]} sampled block(s), one "
                                     f"timing each ({t_sample1:.1f} s of sampling)"},
            "cpu_model": model_name, "logical_cpus": os.cpu_count()}


def bench_batch(args):
    """64 uneven instances (seeds 4000..4063), mixed precision; one step = fde_precond_factor_batch
    + fde_bvm_solve_batch over all of them with inputs resident in HBM."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1305_6653_amd import BvmSolver, factor_batch, solve_batch
    ps = W.batch_c4(64)
    dev = torch.device("cuda:0")
    u0s = [torch.from_numpy(np.ascontiguousarray(p.u0)).to(dev) for p in ps]
    fs = [torch.from_numpy(np.ascontiguousarray(p.f)).to(dev) for p in ps]
    outs = [torch.empty((p.s, p.m), dtype=torch.float64, device=dev) for p in ps]
    Ss = [BvmSolver(p) for p in ps]
    stream = torch.cuda.current_stream()
    for S in Ss:
        S.set_stream(stream)
    for _ in range(args.warmup):
        factor_batch(Ss, "mixed")
        solve_batch(Ss, u0s, fs, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        factor_batch(Ss, "mixed")
        _, infos = solve_batch(Ss, u0s, fs, outs=outs)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    lead = Ss[0]
    lead.profile(True)
    for _ in range(args.steps):
        factor_batch(Ss, "mixed")
        solve_batch(Ss, u0s, fs, outs=outs)
    torch.cuda.synchronize()
    prof = {}
    for k in ("assemble", "lu_diag", "lu_panel", "lu_update", "trsv", "time_rfft", "time_irfft",
              "bvm_matvec", "mgs", "cgs", "arnoldi", "normalize", "residual", "update_x", "rhs", "dot", "toeplitz"):
        q = lead.profile_query(k)
        if q["count"]:
            prof[k] = q
    lead.profile(False)
    # the same 64 instances one at a time in plain FP64 (fde_precond_factor + fde_bvm_solve
    # each), once: the reference the batched mixed form is compared with
    iters_fp64 = []
    for S, u0, f, o in zip(Ss, u0s, fs, outs):   # warm every shape's autotuner entry first
        S.factor("fp64")
        S.solve(u0, f, out=o, rtol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for S, u0, f, o in zip(Ss, u0s, fs, outs):
        S.factor("fp64")
        _, inf = S.solve(u0, f, out=o, rtol=1e-10)
        iters_fp64.append(inf["iters"])
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3
    flops = sum((p.s // 2 + 1) * 8.0 * p.m ** 3 / 3.0 for p in ps)
    result = {
        "metric": METRIC, "value": round(64 * 1000.0 / ms, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c32+f64",
        "data": "synthetic (seeded random instances, workloads.batch_c4)",
        "config": {"workload": "batch of 64 uneven instances (seeds 4000..4063), GBDF3, mixed",
                   "instances": 64, "m_range": [min(p.m for p in ps), max(p.m for p in ps)],
                   "s_range": [min(p.s for p in ps), max(p.s for p in ps)],
                   "unknowns_total": sum(p.m * p.s for p in ps), "precision": "mixed", "rtol": 1e-10,
                   "step": "fde_precond_factor_batch + fde_bvm_solve_batch"},
        "iters_max": max(i["iters"] for i in infos), "iters_mean": float(np.mean([i["iters"] for i in infos])),
        "max_true_relres": max(i["true_relres"] for i in infos), "lu_flops": flops,
        "sequential_fp64_ms": round(ms_seq, 3),
        "speedup_vs_sequential_fp64": round(ms_seq / ms, 3),
        "iters_fp64_mean": float(np.mean(iters_fp64)),
        "kernels": kernel_table(prof, args.steps, "mixed"),
        "roofline": roofline(prof, "mixed", "c4"), "cpu_baseline": None,
    }
    DEV.calib_copy(args.calib_copy_mib)
    for S in Ss:
        S.close()
    print(json.dumps(result), flush=True)


def bench_example41(args):
    """Example 4.1 of Section 4 (GAM5, f = 0, Gaussian pulse): every (alpha, m, s) of Tables 1-2
    with each preconditioner (I, S, S2, S2~), left-preconditioned GMRES(20) to 1e-8 of the
    initial preconditioned residual from a zero start (the tables' convention).  One step =
    fde_precond_factor + fde_bvm_solve of one case; reported per case (ITS, ms) and as the
    rate over all 96 cases."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1305_6653_amd import BvmSolver
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    cases, total_ms = [], 0.0
    for a, m, s in W.EXAMPLE41_GRID:
        p = W.example41(a, m, s)
        u0 = torch.from_numpy(np.ascontiguousarray(p.u0)).to(dev)
        f = torch.from_numpy(np.ascontiguousarray(p.f)).to(dev)
        out = torch.empty((s, m), dtype=torch.float64, device=dev)
        S = BvmSolver(p)
        S.set_stream(stream)
        row = {"alpha": a, "m": m, "s": s}
        for pc, key in (("none", "I"), ("strang", "S"), ("bccb", "S2"), ("bccb_shifted", "S2t")):
            for _ in range(max(1, args.warmup)):
                S.factor("fp64", pc)
                S.solve(u0, f, out=out, rtol=1e-8, maxit=3000, side="left")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                S.factor("fp64", pc)
                _, info = S.solve(u0, f, out=out, rtol=1e-8, maxit=3000, side="left")
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            total_ms += ms
            row[key] = {"its": info["iters"], "ms": round(ms, 4),
                        "true_relres": float("%.3g" % info["true_relres"])}
        S.close()
        cases.append(row)
    result = {
        "metric": "Example 4.1 (Tables 1-2): factor + left-preconditioned GMRES(20) solves to 1e-8, "
                  "solves/s over all 96 (alpha, m, s, preconditioner) cases",
        "value": round(96 * 1000.0 / total_ms, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(total_ms / 96, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "analytic (Example 4.1: f = 0, d+ = 0.6, d- = 0.5, Gaussian pulse u0)",
        "config": {"workload": "Example 4.1, GAM5, alpha in {1.2, 1.5}, m in {24, 48, 96}, "
                               "s in {16, 32, 64, 128}", "precision": "fp64", "side": "left",
                   "rtol": 1e-8, "restart": 20, "step": "fde_precond_factor + fde_bvm_solve"},
        "cases": cases,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def main():
    global DEV
    args = parse()
    DEV = DeviceMemory(args.device_memory)
    if args.workload == "ex41":
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        bench_example41(args)
        return
    if args.workload == "c4":
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        bench_batch(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path shards across "
              "GPUs by frequency block, which this library does not run", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    from paper_1305_6653_amd import BvmSolver, autotune_report
    from paper_1305_6653_amd import _native as N

    p = workload(args.workload)
    prec = "fp64"
    fp64_dev = DEV.put
    u0 = fp64_dev(p.u0)
    f = fp64_dev(p.f)
    out = DEV.empty((p.s, p.m))
    S = BvmSolver(p)
    if DEV.stream() is not None:
        S.set_stream(DEV.stream())

    ms, ms_prof, infos, prof = timed_steps(S, u0, f, out, prec, args.steps, args.warmup)
    read_peak = measured_read_peak()
    u_main = DEV.get(out)
    result = {
        "metric": METRIC, "value": round(1000.0 / ms, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded smooth random Fourier modes, workloads module)",
        "config": {"workload": p.name, "m": p.m, "s": p.s, "bvm": p.bvm, "alpha": p.alpha,
                   "unknowns": p.m * p.s, "precision": prec, "rtol": 1e-10, "restart": 20,
                   "step": "fde_precond_factor + fde_bvm_solve (the library's default block solver "
                           "for this size; config.blocks)"},
        "iters": infos[-1]["iters"], "restarts": infos[-1]["restarts"],
        "true_relres": infos[-1]["true_relres"],
        "t_factor_ms": round(infos[-1]["t_factor_ms"], 3),
        "t_solve_ms": round(infos[-1]["t_solve_ms"], 3),
        "profiled_ms_per_step": round(ms_prof, 4),
        "kernels": kernel_table(prof, args.steps, prec),
        "roofline": roofline(prof, prec, args.workload, read_peak),
        "autotuned": autotune_report(),
    }
    # Every solve of a handle sizes its first stretch of Arnoldi steps from its previous solve;
    # with a right-hand side that changes from step to step that guess is not exact.  Same
    # steps, alternating between two seeded right-hand sides of the same recipe.
    q = workload_alt(args.workload)
    rhs = [(u0, f), (fp64_dev(q.u0), fp64_dev(q.f))]
    for k in range(2):
        S.factor(prec)
        S.solve(*rhs[k % 2], out=out, rtol=1e-10)
    DEV.sync()
    t0 = time.perf_counter()
    for k in range(args.steps):
        S.factor(prec)
        S.solve(*rhs[k % 2], out=out, rtol=1e-10)
    DEV.sync()
    ms_alt = (time.perf_counter() - t0) * 1e3 / args.steps
    result["changed_rhs"] = {"ms_per_step": round(ms_alt, 4), "value": round(1000.0 / ms_alt, 4),
                             "rhs": f"alternating {p.name} and {q.name}'s u0, f"}
    route_names = {N.FDE_BLOCKS_LU: "lu", N.FDE_BLOCKS_HESSENBERG: "hessenberg", N.FDE_BLOCKS_BAND: "band"}
    in_use = S.get_option(N.FDE_OPT_BLOCKS_IN_USE)  # the headline form's route (before the mixed form's)
    result["config"]["blocks"] = route_names.get(in_use, in_use)
    if not args.no_mixed:
        ms2, _, infos2, prof2 = timed_steps(S, u0, f, out, "mixed", args.steps, args.warmup)
        u_mixed = DEV.get(out)
        result["mixed"] = {
            "ms_per_step": round(ms2, 4), "value": round(1000.0 / ms2, 4), "iters": infos2[-1]["iters"],
            "true_relres": infos2[-1]["true_relres"],
            "t_factor_ms": round(infos2[-1]["t_factor_ms"], 3),
            "t_solve_ms": round(infos2[-1]["t_solve_ms"], 3),
            "rel_diff_vs_fp64": float(np.linalg.norm(u_mixed - u_main) / np.linalg.norm(u_main)),
            "speedup_vs_fp64": round(ms / ms2, 3),
            "blocks": route_names.get(S.get_option(N.FDE_OPT_BLOCKS_IN_USE)),
            "kernels": kernel_table(prof2, args.steps, "mixed"),
            "roofline": roofline(prof2, "mixed", args.workload, read_peak),
        }
    if not args.no_hessenberg:
        # the same preconditioner S with its blocks solved by the other routes: dense block LU,
        # one Hessenberg form of J (m <= 1024), one band form of J
        for key, route in (("lu", N.FDE_BLOCKS_LU), ("band", N.FDE_BLOCKS_BAND),
                           ("hessenberg", N.FDE_BLOCKS_HESSENBERG)):
            if route == in_use:
                continue
            result[key] = {}
            for form in ("fp64", "mixed"):
                S.set_option(N.FDE_OPT_BLOCKS, route)
                try:
                    ms4, _, infos4, prof4 = timed_steps(S, u0, f, out, form, args.steps, args.warmup)
                except N.FdeError as e:
                    result[key][form] = {"unsupported": str(e)}
                    continue
                u4 = DEV.get(out)
                result[key][form] = {
                    "ms_per_step": round(ms4, 4), "value": round(1000.0 / ms4, 4),
                    "iters": infos4[-1]["iters"], "true_relres": infos4[-1]["true_relres"],
                    "t_factor_ms": round(infos4[-1]["t_factor_ms"], 3),
                    "t_solve_ms": round(infos4[-1]["t_solve_ms"], 3),
                    "rel_diff_vs_headline": float(np.linalg.norm(u4 - u_main) / np.linalg.norm(u_main)),
                    "headline_speedup": round(ms4 / ms, 3),
                    "kernels": kernel_table(prof4, args.steps, form),
                    "roofline": roofline(prof4, form, args.workload + key[0], read_peak),
                }
        S.set_option(N.FDE_OPT_BLOCKS, N.FDE_BLOCKS_AUTO)
    if not args.no_bccb and args.workload == "c2":
        # the paper's other preconditioners on the same system (Section 3.1): S2 = s(A) x I -
        # tau s(B) x s(J) and its shifted form, each a 2-D FFT diagonal solve per iteration
        result["bccb"] = {}
        for pc in ("bccb", "bccb_shifted"):
            ms3, _, infos3, prof3 = timed_steps(S, u0, f, out, "fp64", max(1, args.steps // 2),
                                                1, pc)
            u3 = DEV.get(out)
            result["bccb"][pc] = {
                "ms_per_step": round(ms3, 4), "value": round(1000.0 / ms3, 4),
                "iters": infos3[-1]["iters"], "true_relres": infos3[-1]["true_relres"],
                "rel_diff_vs_strang": float(np.linalg.norm(u3 - u_main) / np.linalg.norm(u_main)),
                "kernels": {k: {"total_ms": round(v["total_ms"] / max(1, args.steps // 2), 4),
                                "avg_us": round(1e3 * v["total_ms"] / v["count"], 2)}
                            for k, v in prof3.items() if k in ("bccb_solve", "bvm_matvec", "mgs", "cgs",
                                                               "time_rfft", "time_irfft")},
                "bccb_solve_GBs": round(prof3["bccb_solve"]["work"]
                                        / (prof3["bccb_solve"]["total_ms"] * 1e-3) / 1e9, 1)
                if "bccb_solve" in prof3 else None,
            }
    S.close()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(p, result["iters"], result["restarts"])
        result["vs_cpu_baseline"] = round(result["value"] / result["cpu_baseline"]["value"], 1)
    else:
        result["cpu_baseline"] = None
    DEV.calib_copy(args.calib_copy_mib)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
