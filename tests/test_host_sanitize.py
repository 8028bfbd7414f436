"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

`python -m paper_1305_6653_amd.build --sanitize` instruments the host code (the device code is
unchanged).  A child process that preloads the sanitizer runtime loads that build and drives
every host path that runs without a GPU: the validation of every rejected problem and formula,
the host tables of setup (Grünwald weights, the BVM coefficient bands, the Strang eigenvalues,
the FFT twiddles) for the three named BVMs and a custom formula over m from 1 to 4096 and s
from 4 to 1024, the teardown of a handle whose device step failed (without a GPU, setup fails
at its first device call and destroys the half-built handle; with one, the handle is built and
destroyed), and the NULL-argument paths of the other entry points.  Any sanitizer report fails
the child and the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import ctypes as C
import numpy as np
from paper_1305_6653_amd import _native as N

L = N.lib()
OK_OR_NODEV = (N.FDE_OK, N.FDE_EDEVICE)


def setup(m, s, kind=N.FDE_BVM_GBDF3, alpha=1.5, dp=None, dm=None, custom=None, **kw):
    dp = np.ascontiguousarray(np.linspace(1.0, 2.0, m) if dp is None else dp, dtype=np.float64)
    dm = np.ascontiguousarray(np.linspace(2.0, 0.5, m) if dm is None else dm, dtype=np.float64)
    p = N.FdeProblem(alpha, kw.get("xL", 0.0), kw.get("xR", 2.0), 0.0, kw.get("T", 1.0), m, s,
                     dp.ctypes.data_as(N._dp), dm.ctypes.data_as(N._dp), kind,
                     C.pointer(custom) if custom is not None else None)
    h = C.c_void_p()
    st = L.fde_bvm_setup(C.byref(p), C.byref(h))
    if st == N.FDE_OK:
        L.fde_bvm_destroy(h)
    else:
        assert not h.value
        assert L.fde_last_error()
    return st


def formula(nu1, nu2, rows=True):
    mu1 = nu1 + nu2 + 1
    keep = []

    def arr(k):
        a = np.ascontiguousarray(np.random.default_rng(k).standard_normal(max(1, k) * mu1))
        keep.append(a)
        return a.ctypes.data_as(N._dp)
    a = np.zeros(mu1); a[nu1 - 1], a[nu1] = -1.0, 1.0
    b = np.full(mu1, 1.0 / mu1)
    keep += [a, b]
    f = N.FdeBvmFormula(nu1, nu2, a.ctypes.data_as(N._dp), b.ctypes.data_as(N._dp),
                        arr(nu1 - 1) if rows and nu1 > 1 else None, arr(nu1 - 1) if rows and nu1 > 1 else None,
                        arr(nu2) if rows and nu2 > 0 else None, arr(nu2) if rows and nu2 > 0 else None)
    return f, keep


# rejected problems: every validation branch
bad = [dict(alpha=2.0), dict(alpha=1.0), dict(alpha=float("nan")), dict(xR=0.0), dict(T=0.0),
       dict(dm=-np.ones(8)), dict(dp=np.zeros(8), dm=np.zeros(8)), dict(dp=np.full(8, np.inf)),
       dict(kind=99)]
for kw in bad:
    assert setup(8, 16, **kw) == N.FDE_EINVAL, kw
assert setup(8, 3) == N.FDE_EINVAL             # GBDF3 needs s >= 4
assert setup(8, 24) == N.FDE_EUNSUPPORTED      # not a power of two
assert setup(8, 2048) == N.FDE_EUNSUPPORTED
assert setup(4097, 16) == N.FDE_EUNSUPPORTED
assert L.fde_bvm_setup(None, None) == N.FDE_EINVAL
f, keep = formula(2, 1, rows=False)            # initial/final rows missing
assert setup(8, 16, kind=N.FDE_BVM_CUSTOM, custom=f) == N.FDE_EINVAL
f, keep = formula(9, 9)                        # nu1 + nu2 > 16
assert setup(8, 64, kind=N.FDE_BVM_CUSTOM, custom=f) == N.FDE_EINVAL
assert setup(8, 16, kind=N.FDE_BVM_CUSTOM, custom=None) == N.FDE_EINVAL

# accepted problems: host tables, then device step and teardown
count = 0
for kind in (N.FDE_BVM_TRAPEZOIDAL, N.FDE_BVM_GBDF3, N.FDE_BVM_GAM5):
    for m in (1, 2, 63, 64, 65, 130, 1023, 4095, 4096):
        for s in (8, 16, 256, 1024):
            assert setup(m, s, kind=kind, alpha=1.2 + 0.7 * ((m + s) % 7) / 7) in OK_OR_NODEV, (kind, m, s)
            count += 1
f, keep = formula(2, 2)
for m in (1, 100, 4096):
    assert setup(m, 32, kind=N.FDE_BVM_CUSTOM, custom=f) in OK_OR_NODEV
    count += 1

# NULL handles and arguments of the other entry points
v = C.c_int()
assert L.fde_precond_factor(None, N.FDE_FP64) == N.FDE_EINVAL
assert L.fde_bvm_solve(None, None, None, None, None, None) == N.FDE_EINVAL
assert L.fde_bvm_set_option(None, 0, 0) == N.FDE_EINVAL
assert L.fde_bvm_get_option(None, 0, C.byref(v)) == N.FDE_EINVAL
assert L.fde_precond_factor_batch(None, 0, N.FDE_FP64) == N.FDE_OK
assert L.fde_precond_factor_batch(None, 2, N.FDE_FP64) == N.FDE_EINVAL
L.fde_bvm_destroy(None)
buf = C.create_string_buffer(64)
L.fde_autotune_report(buf, 64)
print("sanitized host paths:", count, "setups")
'''


def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    from paper_1305_6653_amd import build as B
    rt = B.sanitizer_runtime()
    if rt is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    lib = B.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, FDE_LIB_PATH=lib, FDE_NO_TORCH="1",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:detect_odr_violation=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True,
                       timeout=600, cwd=ROOT)
    report = r.stdout[-3000:] + r.stderr[-6000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, report
    assert r.returncode == 0, report
    assert "sanitized host paths:" in r.stdout, report
