"""Parity at the benchmark's full sizes, in the configuration bench.py times.

* 1023 x 512 GBDF3 (seed 2): the FP64 and the mixed-form solutions, by the default route and
  by the dense block LU, against the oracle's (textbook preconditioned GMRES to 1e-11 with
  LAPACK block solves, ~10-20 s), plus the true residual with the oracle's dense operator, and
  sampled block-LU factor blocks.
* 4095 x 256 GBDF3 (seed 3), FP64 and mixed form, through the band route (the default at this
  size) and the dense block LU: the solutions against the oracle's (about a minute of host
  LAPACK work and 35 GB of host memory for its block factors), plus the true residual with the
  oracle's dense operator and, for the block LU, sampled factor blocks against the oracle's K_k
  by products with random vectors.

Solutions are compared norm-wise and entry by entry (the worst entry relative to the
solution's largest)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1305_6653_amd import BvmSolver
from paper_1305_6653_amd import _native as N

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _elem(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()


def _factor_product_error(S, p, k, rng):
    """||K_k x - L (U x)|| / ||K_k x|| for a random complex x, K_k = lambda_k I - tau mu_k J
    from the oracle's matrices and Strang eigenvalues, L and U from the GPU's factors."""
    J, F, tau, _ = O.problem_matrices(p)
    lam, mu = O.strang_eigs(F, p.s)
    x = rng.standard_normal(p.m) + 1j * rng.standard_normal(p.m)
    y = lam[k] * x - tau * mu[k] * (J @ x)
    Fk = S.factor_block(k)
    ux = np.triu(Fk) @ x
    z = np.tril(Fk, -1) @ ux + ux
    return _rel(z, y)


def test_m1023_s512_fp64_and_mixed_match_the_oracle():
    p = W.smooth_c2()
    S = BvmSolver(p)
    ref = O.solve_gmres(p, tol=1e-11, maxit=200,  # true rel-res ~4e-12
                        progress=lambda t: print(t, flush=True))
    rng = np.random.default_rng(5)
    nb = p.s // 2 + 1
    for prec, tol, ftol in (("fp64", 1e-9, 1e-12), ("mixed", 1e-8, 1e-5)):
        # the default route (the band route for FP64 at this size: s / 2 + 1 >= 257), then the
        # dense block LU, whose factor blocks are L U = K_k
        for blocks in ("auto", "lu"):
            S.factor(prec, blocks=blocks)
            u, info = S.solve(p.u0, p.f, rtol=1e-10)
            assert info["converged"] == 1 and info["true_relres"] <= 1e-10
            assert _rel(u, ref.x) <= tol, (prec, blocks, _rel(u, ref.x))
            assert _elem(u, ref.x) <= tol, (prec, blocks, _elem(u, ref.x))
            assert O.true_relres(p, u) <= 1.5e-10
        assert S.get_option(N.FDE_OPT_BLOCKS_IN_USE) == N.FDE_BLOCKS_LU
        for k in (0, 1, nb // 2, nb - 1):
            e = _factor_product_error(S, p, k, rng)
            assert e <= ftol, (prec, k, e)
    S.close()


@pytest.fixture(scope="module")
def c3_oracle():
    p = W.smooth_c3()
    print("oracle solve of the 4095 x 256 workload (about a minute)", flush=True)
    return p, O.solve_gmres(p, tol=1e-11, maxit=200, progress=lambda t: print(t, flush=True))


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("blocks", ["band", "lu"])
@pytest.mark.parametrize("prec,tol,ftol", [("fp64", 1e-9, 1e-12), ("mixed", 1e-8, 1e-4)])
def test_m4095_s256_matches_the_oracle(c3_oracle, prec, tol, ftol, blocks):
    """Both block solvers at the benchmark's largest size: the band route (the default at this m)
    and the dense block LU (whose factors are also checked against the oracle's K_k)."""
    p, ref = c3_oracle
    assert ref.converged
    S = BvmSolver(p)
    if blocks == "band":
        S.factor(prec)  # the default route choice takes the band route at m = 4095
        assert S.get_option(N.FDE_OPT_BLOCKS_IN_USE) == N.FDE_BLOCKS_BAND
    else:
        S.factor(prec, blocks="lu")
    u, info = S.solve(p.u0, p.f, rtol=1e-10)
    assert info["converged"] == 1 and info["true_relres"] <= 1e-10
    assert _rel(u, ref.x) <= tol, (prec, _rel(u, ref.x))
    assert _elem(u, ref.x) <= tol, (prec, _elem(u, ref.x))
    assert O.true_relres(p, u) <= 1.5e-10
    if blocks == "lu":
        rng = np.random.default_rng(6)
        nb = p.s // 2 + 1
        for k in (0, 1, nb // 2, nb - 1):
            e = _factor_product_error(S, p, k, rng)
            assert e <= ftol, (prec, k, e)
    S.close()
