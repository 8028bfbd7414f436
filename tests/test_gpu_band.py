"""The band route to the blocks of S (FDE_BLOCKS_BAND, not in the paper): J = Q H Q^T with H of
lower bandwidth 64 by a blocked Householder reduction, then per block an LU of
lambda_k I - tau mu_k H with partial pivoting among the 128 rows of each panel.  The reduction
is checked by the properties that define it (Q H Q^T = J, Q^T Q = I, the band); the block solves
and whole solves against the oracle's S^{-1} (LAPACK block LUs with partial pivoting) and its
GMRES solution, and the iteration counts against the block-LU route's."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1305_6653_amd import BvmSolver, factor_batch, solve_batch
from paper_1305_6653_amd import _native as N

pytestmark = pytest.mark.gpu

CASES = {
    "gbdf3_m1_s4": lambda: W.tiny(1, 4, 1.3, 2, "gbdf3"),
    "gbdf3_m63_s16": lambda: W.tiny(63, 16, 1.7, 3, "gbdf3"),         # one panel: no reduction
    "trap_m130_s16": lambda: W.tiny(130, 16, 1.2, 5, "trapezoidal"),  # three panels, ragged
    "gbdf3_m128_s16": lambda: W.tiny(128, 16, 1.4, 6, "gbdf3"),        # m = mp: H's last entry is read
    "gbdf3_m200_s32": lambda: W.tiny(200, 32, 1.7, 4, "gbdf3"),
    "gam5_m96_s64": lambda: W.example41(1.5, 96, 64),
    "gbdf3_m255_s128": lambda: W.warmstart_instance(7),
}


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _elem(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()


@pytest.mark.parametrize("name", ["gbdf3_m63_s16", "trap_m130_s16", "gbdf3_m200_s32", "gbdf3_m255_s128"])
def test_band_reduction_properties(name):
    p = CASES[name]()
    S = BvmSolver(p)
    S.factor("fp64", blocks="band")
    H, Q = S.hessenberg()
    J, _, _, _ = O.problem_matrices(p)
    m = p.m
    eps = np.finfo(float).eps
    assert np.abs(Q @ H @ Q.T - J).max() <= 50 * m * eps * np.abs(J).max()
    assert np.abs(Q.T @ Q - np.eye(m)).max() <= 50 * m * eps
    i, j = np.indices(H.shape)
    assert np.all(H[i > j + 64] == 0.0)
    S.close()


@pytest.mark.parametrize("prec,eps", [("fp64", 2.0 ** -53), ("mixed", 2.0 ** -24)])
@pytest.mark.parametrize("name", ["gbdf3_m1_s4", "gbdf3_m63_s16", "trap_m130_s16", "gbdf3_m128_s16", "gbdf3_m200_s32"])
def test_band_preconditioner_apply(name, prec, eps):
    """Forward error of S^{-1} v within 100 eps max_k cond(K_k) of the oracle's (the reduction
    adds an orthogonal similarity, the pivoting only bounded growth)."""
    p = CASES[name]()
    S = BvmSolver(p)
    S.factor(prec, blocks="band")
    J, F, tau, _ = O.problem_matrices(p)
    P = O.StrangPreconditioner(J, F, p.s, tau)
    kappa = max(np.linalg.cond(P.block(k, J, tau)) for k in range(p.s // 2 + 1))
    v = np.random.default_rng(4).standard_normal((p.s, p.m))
    assert _rel(S.precond(v), P.apply(v)) <= 100 * eps * max(kappa, 10.0)
    S.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-8)])
@pytest.mark.parametrize("name", list(CASES))
def test_band_solve_vs_oracle(name, prec, tol):
    p = CASES[name]()
    S = BvmSolver(p)
    S.factor(prec, blocks="band")
    u, info = S.solve(p.u0, p.f, rtol=1e-10)
    assert info["converged"] == 1 and info["true_relres"] <= 1e-10
    ref = O.solve_gmres(p, tol=1e-12)
    assert _rel(u, ref.x) <= tol and _elem(u, ref.x) <= tol, (_rel(u, ref.x), _elem(u, ref.x))
    assert O.true_relres(p, u) <= 1.5e-10
    S2 = BvmSolver(p)
    S2.factor(prec)
    _, i2 = S2.solve(p.u0, p.f, rtol=1e-10)
    assert abs(info["iters"] - i2["iters"]) <= 1, (info["iters"], i2["iters"])
    S2.close()
    S.close()


def test_band_batch_equals_single():
    ps = [CASES[n]() for n in ("gbdf3_m63_s16", "trap_m130_s16", "gbdf3_m200_s32")]
    batch = [BvmSolver(p) for p in ps]
    for S in batch:
        S.set_option(N.FDE_OPT_BLOCKS, N.FDE_BLOCKS_BAND)
    factor_batch(batch, "fp64")
    outs, infos = solve_batch(batch, [p.u0 for p in ps], [p.f for p in ps])
    for p, u, info in zip(ps, outs, infos):
        S = BvmSolver(p)
        S.factor("fp64", blocks="band")
        u1, i1 = S.solve(p.u0, p.f)
        assert np.array_equal(u, u1) and info["iters"] == i1["iters"], p.name
        S.close()
    for S in batch:
        S.close()


def test_band_route_switches_with_the_others_on_one_handle():
    p = CASES["gbdf3_m200_s32"]()
    S = BvmSolver(p)
    sols = {}
    for blocks in ("band", "lu", "hessenberg", "band"):
        S.factor("fp64", blocks=blocks)
        sols.setdefault(blocks, []).append(S.solve(p.u0, p.f)[0])
    assert np.array_equal(sols["band"][0], sols["band"][1])   # refactoring repeats the bits
    assert _rel(sols["band"][0], sols["lu"][0]) <= 1e-9
    assert _rel(sols["hessenberg"][0], sols["lu"][0]) <= 1e-9
    S.close()


def test_automatic_route_choice_by_size():
    """FDE_BLOCKS_AUTO (the default): the band route from m = 1152 on for FP64 blocks (from
    m = 960 when s / 2 + 1 >= 257) and from m = 1792 for FP32 blocks, block LU below; a batch
    takes the band route only if every instance qualifies."""
    small, big = W.tiny(200, 8, 1.5, 1, "gbdf3"), W.tiny(1600, 8, 1.5, 2, "gbdf3")
    Ss, Sb = BvmSolver(small), BvmSolver(big)
    assert Ss.get_option(N.FDE_OPT_BLOCKS) == N.FDE_BLOCKS_AUTO
    Ss.factor("fp64")
    Sb.factor("fp64")
    assert Ss.get_option(N.FDE_OPT_BLOCKS_IN_USE) == N.FDE_BLOCKS_LU
    assert Sb.get_option(N.FDE_OPT_BLOCKS_IN_USE) == N.FDE_BLOCKS_BAND
    u, info = Sb.solve(big.u0, big.f)
    assert info["converged"] == 1 and O.true_relres(big, u) <= 1.5e-10
    Sb.factor("mixed")
    assert Sb.get_option(N.FDE_OPT_BLOCKS_IN_USE) == N.FDE_BLOCKS_LU
    factor_batch([Ss, Sb], "fp64")
    assert Sb.get_option(N.FDE_OPT_BLOCKS_IN_USE) == N.FDE_BLOCKS_LU
    Ss.close()
    Sb.close()
    # long time axis (s / 2 + 1 >= 257): the band route from m = 960 in FP64
    mid_short, mid_long = W.tiny(1000, 256, 1.5, 3, "gbdf3"), W.tiny(1000, 512, 1.5, 3, "gbdf3")
    for p, want in ((mid_short, N.FDE_BLOCKS_LU), (mid_long, N.FDE_BLOCKS_BAND)):
        S = BvmSolver(p)
        S.factor("fp64")
        assert S.get_option(N.FDE_OPT_BLOCKS_IN_USE) == want, (p.s, want)
        S.factor("mixed")
        assert S.get_option(N.FDE_OPT_BLOCKS_IN_USE) == N.FDE_BLOCKS_LU
        S.close()
