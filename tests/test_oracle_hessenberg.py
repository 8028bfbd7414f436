"""Pins of the oracle's Hessenberg route to the blocks of S: every K_k is a shift of the same
J, so J = Q H Q^T turns each block solve into a shifted Hessenberg solve."""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W


def _rand_hess(m, rng, diag_scale=1.0):
    C = np.triu(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)), -1)
    C[np.diag_indices(m)] *= diag_scale
    return C


@pytest.mark.parametrize("m", [1, 2, 5, 33, 100])
@pytest.mark.parametrize("diag_scale", [1.0, 1e-3])
def test_hessenberg_lu_solves_like_the_dense_solver(m, diag_scale):
    rng = np.random.default_rng(m)
    C = _rand_hess(m, rng, diag_scale)
    U, l, sw = O.hessenberg_lu(C)
    assert np.array_equal(U, np.triu(U))
    assert np.all(np.abs(l) <= 1.0)            # partial pivoting bounds every multiplier
    Y = rng.standard_normal((m, 3)) + 1j * rng.standard_normal((m, 3))
    for c in range(3):
        z = O.hessenberg_lu_solve(U, l, sw, Y[:, c])
        ref = np.linalg.solve(C, Y[:, c])
        assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.cond(C) * np.linalg.norm(ref) + 1e-300
    if diag_scale < 1 and m > 1:
        assert sw.any()                         # tiny diagonal: rows are exchanged


def test_pivot_exchange_is_needed_and_taken():
    C = np.array([[0.0, 1.0], [1.0, 1.0]], dtype=complex)   # zero pivot without exchange
    U, l, sw = O.hessenberg_lu(C)
    assert sw[0] and l[0] == 0.0
    np.testing.assert_allclose(O.hessenberg_lu_solve(U, l, sw, np.array([1.0, 2.0])), [1.0, 1.0])


@pytest.mark.parametrize("kind", ["trapezoidal", "gbdf3", "gam5"])
def test_hessenberg_route_equals_the_block_lu_route(kind):
    p = W.tiny(37, 16, 1.6, 2, kind)
    J, F, tau, _ = O.problem_matrices(p)
    Ph = O.HessenbergPreconditioner(J, F, p.s, tau)
    np.testing.assert_allclose(Ph.Q @ Ph.H @ Ph.Q.T, J, atol=1e-12 * np.abs(J).max())
    np.testing.assert_allclose(Ph.Q.T @ Ph.Q, np.eye(p.m), atol=1e-13)
    assert np.array_equal(Ph.H, np.triu(Ph.H, -1))
    v = np.random.default_rng(3).standard_normal((p.s, p.m))
    ref = O.StrangPreconditioner(J, F, p.s, tau).apply(v)
    assert np.linalg.norm(Ph.apply(v) - ref) <= 1e-11 * np.linalg.norm(ref)


def test_hessenberg_route_in_gmres():
    p = W.tiny(40, 32, 1.8, 1, "gbdf3")
    a = O.solve_gmres(p, tol=1e-12, precond="strang")
    b = O.solve_gmres(p, tol=1e-12, precond="strang_hessenberg")
    assert a.iters == b.iters and np.linalg.norm(a.x - b.x) <= 1e-10 * np.linalg.norm(a.x)
