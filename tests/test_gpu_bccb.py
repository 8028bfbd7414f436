"""The BCCB preconditioners S2 (eq. (x1)) and S2~ (eq. (xc)) on the GPU against the oracle:
the 2-D DFT solve through the C ABI, whole solves and batches."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1305_6653_amd import BvmSolver, solve_batch
from paper_1305_6653_amd import _native as N

pytestmark = pytest.mark.gpu

SIZES = [(7, 8, 1.9, 3, "gbdf3"), (63, 64, 1.5, 0, "trapezoidal"), (130, 16, 1.2, 5, "trapezoidal"),
         (200, 32, 1.7, 4, "gbdf3"), (255, 128, 1.4, 6, "gbdf3")]


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.mark.parametrize("pc", ["bccb", "bccb_shifted"])
@pytest.mark.parametrize("size", SIZES)
def test_bccb_apply_matches_oracle(size, pc):
    """S2^{-1} v through fde_apply_precond: Bluestein DFTs of any order m on the device."""
    p = W.tiny(*size)
    S = BvmSolver(p)
    S.factor("fp64", preconditioner=pc)
    v = np.random.default_rng(7).standard_normal((p.s, p.m))
    P = O.BccbPreconditioner(p, shifted=pc == "bccb_shifted")
    # forward error of a backward-stable transform-and-divide: a few eps times the condition
    # number max|eig| / min|eig| (S2's zero-frequency eigenvalues can be small)
    kappa = np.abs(P.eig).max() / np.abs(P.eig).min()
    assert _rel(S.precond(v), P.apply(v)) <= 30 * 2.0 ** -53 * max(kappa, 10.0) * np.log2(p.m + 1)


@pytest.mark.parametrize("pc", ["bccb", "bccb_shifted"])
@pytest.mark.parametrize("size", SIZES[1:4])
def test_bccb_solve_matches_oracle(size, pc):
    p = W.tiny(*size)
    S = BvmSolver(p)
    S.factor("fp64", preconditioner=pc)
    u, info = S.solve(p.u0, p.f, rtol=1e-10, maxit=3000)
    assert info["converged"] == 1 and info["true_relres"] <= 1e-10
    ref = O.solve_gmres(p, tol=1e-12, precond=pc, maxit=5000)
    assert _rel(u, ref.x) <= 1e-9
    ref10 = O.solve_gmres(p, tol=1e-10, precond=pc, maxit=5000)
    assert abs(info["iters"] - ref10.iters) <= 2, (info["iters"], ref10.iters)


def test_bccb_batch_and_switching_back():
    ps = [W.tiny(*a) for a in SIZES[:3]]
    Ss = [BvmSolver(p) for p in ps]
    for S in Ss:
        S.factor("fp64", preconditioner="bccb")
    singles = [S.solve(p.u0, p.f, maxit=3000)[0] for p, S in zip(ps, Ss)]
    outs, infos = solve_batch(Ss, [p.u0 for p in ps], [p.f for p in ps], maxit=3000)
    for a, b in zip(outs, singles):
        assert np.array_equal(a, b)
    S = Ss[2]
    S.factor("fp64", preconditioner="strang")
    assert S.get_option(N.FDE_OPT_PRECOND) == N.FDE_PC_STRANG
    u, info = S.solve(ps[2].u0, ps[2].f)
    assert info["true_relres"] <= 1e-10 and _rel(u, singles[2]) <= 1e-8
