"""The allocation-free preconditioner apply (fde_apply_precond_noalloc) against the handle's own
apply (fde_apply_precond): bitwise equal on two calls in a row, the second on a smaller
problem, in FP64 and the mixed form; sizes beyond its fixed array and other block solvers are
refused."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from paper_1305_6653_amd import BvmSolver, FdeError
from paper_1305_6653_amd import _native as N

pytestmark = pytest.mark.gpu


def _noalloc(S, v, z):
    return N.lib().fde_apply_precond_noalloc(S.handle, C.c_void_p(v.data_ptr()), C.c_void_p(z.data_ptr()))


@pytest.mark.parametrize("trsv_w", [0, -1])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_apply_equals_the_handle_apply(prec, trsv_w):
    """trsv_w = -1: the handle's block solve is the ordinary one-workgroup launch, which the
    allocation-free apply then takes too."""
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(11)
    for p in (W.tiny(1000, 64, 1.6, 1, "gbdf3"), W.tiny(130, 16, 1.3, 2, "trapezoidal")):
        S = BvmSolver(p)
        S.set_option(N.FDE_OPT_TRSV_W, trsv_w)
        S.factor(prec)
        v = torch.from_numpy(rng.standard_normal((p.s, p.m))).to(dev)
        ref = S.precond(v)
        z = torch.full((p.s, p.m), float("nan"), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        assert _noalloc(S, v, z) == N.FDE_OK, N.lib().fde_last_error()
        torch.cuda.synchronize()
        assert torch.equal(z, ref), (p.name, prec)
        S.close()


def test_noalloc_apply_refuses_what_it_cannot_hold():
    import torch
    dev = torch.device("cuda:0")
    big = W.tiny(4095, 512, 1.5, 3, "gbdf3")      # 257 x 4096 x 16 bytes of frequency vector
    S = BvmSolver(big)
    v = torch.zeros((big.s, big.m), dtype=torch.float64, device=dev)
    assert _noalloc(S, v, v) == N.FDE_EUNSUPPORTED
    S.close()
    p = W.tiny(63, 16, 1.5, 4, "gbdf3")
    S = BvmSolver(p)
    v = torch.zeros((p.s, p.m), dtype=torch.float64, device=dev)
    assert _noalloc(S, v, v) == N.FDE_EINVAL             # not factored yet
    S.factor("fp64", blocks="hessenberg")
    assert _noalloc(S, v, v) == N.FDE_EUNSUPPORTED       # another block solver
    S.close()
