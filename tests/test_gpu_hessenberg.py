"""The Hessenberg route to the blocks of S on the HIP path: J = Q H Q^T against the oracle's
(LAPACK) reduction, the preconditioner apply and whole solves against the oracle, batches and
switching between the two block solvers."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1305_6653_amd import BvmSolver, FdeError, factor_batch, solve_batch
from paper_1305_6653_amd import _native as N

pytestmark = pytest.mark.gpu

CASES = {
    "trap_m1_s2": lambda: W.tiny(1, 2, 1.5, 1, "trapezoidal"),
    "gbdf3_m2_s4": lambda: W.tiny(2, 4, 1.3, 2, "gbdf3"),
    "gbdf3_m7_s8": lambda: W.tiny(7, 8, 1.9, 3, "gbdf3"),
    "trap_m63_s64_manufactured": W.manufactured_c1,
    "gbdf3_m200_s32": lambda: W.tiny(200, 32, 1.7, 4, "gbdf3"),
    "trap_m130_s16": lambda: W.tiny(130, 16, 1.2, 5, "trapezoidal"),
    "gam5_m96_s64_example41": lambda: W.example41(1.5, 96, 64),
    "gbdf3_m255_s128_random": lambda: W.warmstart_instance(7),
    "gbdf3_m300_s8": lambda: W.tiny(300, 8, 1.6, 6, "gbdf3"),
}


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def _hess_solver(p, prec="fp64"):
    S = BvmSolver(p)
    S.factor(prec, "strang", blocks="hessenberg")
    return S


@pytest.mark.parametrize("name", list(CASES))
def test_reduction_matches_lapack(name):
    p = CASES[name]()
    S = _hess_solver(p)
    H, Q = S.hessenberg()
    J, _, _, _ = O.problem_matrices(p)
    Hr, Qr = __import__("scipy.linalg").linalg.hessenberg(J, calc_q=True)
    nJ = np.abs(J).max()
    assert np.array_equal(np.tril(H, -2), np.zeros_like(H))
    assert np.abs(Q @ H @ Q.T - J).max() <= 1e-13 * nJ * np.sqrt(p.m)
    assert np.abs(Q.T @ Q - np.eye(p.m)).max() <= 1e-13 * np.sqrt(p.m)
    # the same first reflection as LAPACK (same sign convention); later columns of two
    # backward-stable reductions may drift apart where subdiagonal entries get small, so the
    # rest is checked by the backward error above
    np.testing.assert_allclose(H[:, 0], Hr[:, 0], rtol=0, atol=1e-13 * nJ * np.sqrt(p.m))


@pytest.mark.parametrize("prec,eps", [("fp64", 2.0 ** -53), ("mixed", 2.0 ** -24)])
@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_the_oracle(name, prec, eps):
    p = CASES[name]()
    S = _hess_solver(p, prec)
    J, F, tau, _ = O.problem_matrices(p)
    P = O.StrangPreconditioner(J, F, p.s, tau)
    kappa = max(np.linalg.cond(P.block(k, J, tau)) for k in range(p.s // 2 + 1))
    v = np.random.default_rng(4).standard_normal((p.s, p.m))
    err = _rel(S.precond(v), P.apply(v))
    assert err <= 100 * eps * max(kappa, 10.0) * np.sqrt(p.m), (err, kappa)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-8)])
@pytest.mark.parametrize("name", list(CASES))
def test_solve_matches_the_oracle_and_the_lu_route(name, prec, tol):
    p = CASES[name]()
    S = _hess_solver(p, prec)
    u, info = S.solve(p.u0, p.f, rtol=1e-10)
    assert info["converged"] == 1 and info["true_relres"] <= 1e-10
    ref = O.solve_gmres(p, tol=1e-12)
    assert _rel(u, ref.x) <= tol, _rel(u, ref.x)
    assert O.true_relres(p, u) <= 1.5e-10
    S2 = BvmSolver(p)
    S2.factor(prec, "strang", blocks="lu")
    _, i2 = S2.solve(p.u0, p.f, rtol=1e-10)
    assert abs(info["iters"] - i2["iters"]) <= 1


def test_switching_block_solvers_and_batches():
    ps = [W.tiny(7, 8, 1.9, 3, "gbdf3"), W.tiny(130, 16, 1.2, 5, "trapezoidal"),
          W.example41(1.2, 48, 32)]
    Ss = [BvmSolver(p) for p in ps]
    for S in Ss:
        S.set_option(N.FDE_OPT_BLOCKS, N.FDE_BLOCKS_HESSENBERG)
    factor_batch(Ss, "fp64")
    ub, ib = solve_batch(Ss, [p.u0 for p in ps], [p.f for p in ps])
    for p, u, info in zip(ps, ub, ib):
        S1 = _hess_solver(p)
        u1, i1 = S1.solve(p.u0, p.f)
        assert np.array_equal(u, u1) and info["iters"] == i1["iters"]
    S = Ss[2]
    outs = []
    for blocks in ("lu", "hessenberg", "lu", "hessenberg"):
        S.factor("fp64", "strang", blocks=blocks)
        outs.append(S.solve(ps[2].u0, ps[2].f)[0])
    assert np.array_equal(outs[0], outs[2]) and np.array_equal(outs[1], outs[3])
    assert _rel(outs[0], outs[1]) <= 1e-9


def test_orders_beyond_the_register_resident_reduction_are_refused():
    p = W.tiny(1100, 4, 1.5, 1, "gbdf3")
    S = BvmSolver(p)
    S.set_option(N.FDE_OPT_BLOCKS, N.FDE_BLOCKS_HESSENBERG)
    with pytest.raises(FdeError) as e:
        S.factor("fp64")
    assert e.value.status == N.FDE_EUNSUPPORTED
    S.factor("fp64", blocks="lu")   # the handle stays usable
    u, info = S.solve(p.u0, p.f)
    assert info["converged"] == 1
