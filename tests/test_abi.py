"""C ABI checks that need no GPU: the library loads, exports every symbol that
include/fdebvm.h declares, and rejects invalid problems before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1305_6653_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdebvm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fde_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(N.LIB_PATH):
        pytest.fail("libfdebvm.so is not built (run python -m paper_1305_6653_amd.build)")
    return N.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
    bound = {n for n, _, _ in N.SIGNATURES}
    assert set(names) == bound, set(names) ^ bound


def _problem(**kw):
    m = kw.pop("m", 8)
    dp = np.ascontiguousarray(kw.pop("dp", np.ones(m)), dtype=np.float64)
    dm = np.ascontiguousarray(kw.pop("dm", np.ones(m)), dtype=np.float64)
    p = N.FdeProblem(kw.pop("alpha", 1.5), kw.pop("xL", 0.0), kw.pop("xR", 2.0), kw.pop("t0", 0.0),
                     kw.pop("T", 1.0), m, kw.pop("s", 16), dp.ctypes.data_as(N._dp),
                     dm.ctypes.data_as(N._dp), kw.pop("kind", N.FDE_BVM_GBDF3), kw.pop("custom", None))
    return p, (dp, dm)


@pytest.mark.parametrize("kw,status", [
    (dict(alpha=2.0), N.FDE_EINVAL),
    (dict(alpha=1.0), N.FDE_EINVAL),
    (dict(alpha=float("nan")), N.FDE_EINVAL),
    (dict(dm=-np.ones(8)), N.FDE_EINVAL),
    (dict(dp=np.zeros(8), dm=np.zeros(8)), N.FDE_EINVAL),
    (dict(dp=np.full(8, np.inf)), N.FDE_EINVAL),
    (dict(m=0, dp=np.ones(1), dm=np.ones(1)), N.FDE_EINVAL),
    (dict(s=3), N.FDE_EINVAL),                       # GBDF3 needs s >= mu+1 = 4
    (dict(s=24), N.FDE_EUNSUPPORTED),                # not a power of two
    (dict(s=2048), N.FDE_EUNSUPPORTED),
    (dict(xR=0.0), N.FDE_EINVAL),
    (dict(T=0.0), N.FDE_EINVAL),
    (dict(kind=7), N.FDE_EINVAL),
    (dict(kind=N.FDE_BVM_CUSTOM), N.FDE_EINVAL),     # custom without a formula
])
def test_setup_rejects_invalid_problem(lib, kw, status):
    p, keep = _problem(**kw)
    h = C.c_void_p()
    st = lib.fde_bvm_setup(C.byref(p), C.byref(h))
    assert st == status
    assert not h.value
    assert lib.fde_last_error()


def test_setup_rejects_inconsistent_custom_formula(lib):
    a = (C.c_double * 2)(-1.0, 1.0)
    b = (C.c_double * 2)(0.5, 0.6)    # rho'(1) = 1 != sigma(1) = 1.1
    f = N.FdeBvmFormula(1, 0, a, b, None, None, None, None)
    p, keep = _problem(kind=N.FDE_BVM_CUSTOM, custom=C.pointer(f))
    h = C.c_void_p()
    assert lib.fde_bvm_setup(C.byref(p), C.byref(h)) == N.FDE_EINVAL
    assert b"consistent" in lib.fde_last_error()


def test_null_arguments(lib):
    h = C.c_void_p()
    assert lib.fde_bvm_setup(None, C.byref(h)) == N.FDE_EINVAL
    assert lib.fde_precond_factor(None, 0) == N.FDE_EINVAL
    assert lib.fde_bvm_solve(None, None, None, None, None, None) == N.FDE_EINVAL
    assert lib.fde_apply_matvec(None, None, None, 0) == N.FDE_EINVAL
    assert lib.fde_read_bandwidth_probe(1 << 20, 1, None) == N.FDE_EINVAL
    assert lib.fde_mfma_peak_probe(1, 0, None) == N.FDE_EINVAL
    lib.fde_bvm_destroy(None)


def test_empty_and_negative_batches(lib):
    # an empty batch is a no-op (nothing is launched); a negative count is an error
    assert lib.fde_precond_factor_batch(None, 0, 0) == N.FDE_OK
    assert lib.fde_bvm_solve_batch(None, 0, None, None, None, None, None) == N.FDE_OK
    assert lib.fde_precond_factor_batch(None, -1, 0) == N.FDE_EINVAL
    assert lib.fde_bvm_solve_batch(None, -1, None, None, None, None, None) == N.FDE_EINVAL
