"""Pins of the oracle's preconditioner and solver (Sections 3.1-3.2) and of the whole
s-form system against the manufactured solution."""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W

KINDS = ["trapezoidal", "gbdf3"]


def _paper_circulant(coef, nu, mu, s):
    """s(A) of eq. (1.11) written from its printed first row
    (alpha_nu, ..., alpha_mu, 0, ..., 0, alpha_0, ..., alpha_{nu-1}); row n is row 0 shifted by n."""
    row0 = np.zeros(s)
    row0[:mu - nu + 1] = coef[nu:]
    if nu:
        row0[s - nu:] = coef[:nu]
    return np.array([np.roll(row0, n) for n in range(s)])


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("s", [4, 8, 16])
def test_strang_circulant_and_eigenvalues(kind, s):
    F = O.formula(kind)
    cA, cB = O.strang_columns(F, s)
    np.testing.assert_array_equal(O.strang_circulant(cA), _paper_circulant(F.alpha, F.nu, F.mu, s))
    np.testing.assert_array_equal(O.strang_circulant(cB), _paper_circulant(F.beta, F.nu, F.mu, s))
    lam, mu = O.strang_eigs(F, s)
    # closed form phi_j = sum_{r=-nu}^{mu-nu} alpha_{r+nu} omega^{rj}, omega = e^{2 pi i/s}
    w = np.exp(2j * np.pi / s)
    j = np.arange(s)
    phi = sum(F.alpha[r + F.nu] * w ** (r * j) for r in range(-F.nu, F.mu - F.nu + 1))
    psi = sum(F.beta[r + F.nu] * w ** (r * j) for r in range(-F.nu, F.mu - F.nu + 1))
    np.testing.assert_allclose(lam, phi, atol=1e-14)
    np.testing.assert_allclose(mu, psi, atol=1e-14)
    assert abs(lam[0]) < 1e-15                       # phi_0 = rho(1) = 0
    # eigen-decomposition of the dense circulant
    C = O.strang_circulant(cA)
    Fm = np.exp(-2j * np.pi * np.outer(j, j) / s)
    np.testing.assert_allclose(Fm @ C @ np.linalg.inv(Fm), np.diag(lam), atol=1e-12)


@pytest.mark.parametrize("kind", KINDS)
def test_strang_fft_apply_inverts_dense_S(kind):
    p = W.tiny(7, 16, 1.4, 1, kind)
    J, F, tau, _ = O.problem_matrices(p)
    S = O.strang_dense(J, F, p.s, tau)
    P = O.StrangPreconditioner(J, F, p.s, tau)
    v = np.random.default_rng(2).standard_normal(p.s * p.m)
    np.testing.assert_allclose(S @ P.apply(v).reshape(-1), v, atol=1e-12)
    np.testing.assert_allclose(P.apply(v).reshape(-1), np.linalg.solve(S, v), atol=1e-12)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("alpha", [1.2, 1.8])
def test_blocks_invertible_and_diagonally_dominant(kind, alpha):
    """Cor. 3.2 (S invertible) and the derived fact that every K_k = lambda_k I - tau mu_k J is
    strictly row diagonally dominant (Re(lambda_k/mu_k) >= 0 for an A-stable BVM, Prop 2.2)."""
    p = W.tiny(24, 32, alpha, 5, kind)
    J, F, tau, _ = O.problem_matrices(p)
    P = O.StrangPreconditioner(J, F, p.s, tau)
    for k in range(p.s // 2 + 1):
        K = P.block(k, J, tau)
        d = np.abs(np.diag(K))
        off = np.abs(K).sum(axis=1) - d
        assert np.all(d > off)
        assert np.linalg.svd(K, compute_uv=False).min() > 0


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("m,s", [(3, 8), (5, 8), (4, 16)])
def test_rank_theorem(kind, m, s):
    """Theorem 3.3: S^{-1} M = I + L with rank L <= 2 m mu; here rank L = mu m exactly
    (M - S is supported on the nu + (mu - nu) boundary block rows)."""
    p = W.tiny(m, s, 1.5, 3, kind)
    J, F, tau, _ = O.problem_matrices(p)
    M, _ = O.problem_system(p)
    S = O.strang_dense(J, F, s, tau)
    L = np.linalg.solve(S, M) - np.eye(m * s)
    sv = np.linalg.svd(L, compute_uv=False)
    rank = int(np.sum(sv > 1e-10 * sv[0]))
    assert rank <= 2 * m * F.mu
    assert rank == F.mu * m


@pytest.mark.parametrize("kind", KINDS)
def test_gmres_iteration_bound(kind):
    """Theorem 3.3: GMRES on S^{-1} M converges in at most 2 m mu + 1 iterations (here mu m + 1)."""
    p = W.tiny(5, 16, 1.7, 4, kind)
    F = O.formula(kind)
    r = O.solve_gmres(p, tol=1e-12, restart=400)
    assert r.converged
    assert r.iters <= F.mu * p.m + 1 <= 2 * F.mu * p.m + 1


def test_gmres_is_minimal_residual():
    """Textbook property: after k steps from x0 = 0, GMRES returns argmin over the Krylov
    space K_k(A P, b) of ||b - A P y|| (checked by least squares on an explicit basis)."""
    rng = np.random.default_rng(11)
    n = 30
    A = np.eye(n) * 4 + rng.standard_normal((n, n))
    Pm = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    for k in (1, 3, 6):
        r = O.gmres(lambda x: A @ x, lambda v: Pm @ v, b, tol=0.0, restart=k, maxit=k)
        AP = A @ Pm
        K = np.column_stack([np.linalg.matrix_power(AP, i) @ b for i in range(k)])
        y, *_ = np.linalg.lstsq(AP @ K, b, rcond=None)
        np.testing.assert_allclose(r.x, Pm @ K @ y, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("kind", KINDS)
def test_gmres_matches_direct(kind):
    """O2 (preconditioned GMRES) equals O1 (dense LAPACK solve)."""
    p = W.tiny(31, 32, 1.6, 9, kind)
    U1 = O.solve_direct(p)
    r = O.solve_gmres(p, tol=1e-13)
    assert r.converged
    assert np.linalg.norm(r.x - U1) / np.linalg.norm(U1) < 1e-12
    assert O.true_relres(p, r.x) < 1e-13


def test_manufactured_c1_accuracy():
    """The manufactured workload (alpha=1.5, m=63, s=64, trapezoidal): the discrete solution
    is within the first-order spatial error of the analytic u (relative L2 ~ 1.1e-2)."""
    p = W.manufactured_c1()
    U = O.solve_gmres(p, tol=1e-13).x
    Ue = p.exact(W.grid_x(p.m), W.grid_t(p.s)[1:])
    e = np.linalg.norm(U - Ue) / np.linalg.norm(Ue)
    assert 0.005 < e < 0.02


def test_manufactured_first_order_in_space():
    errs = []
    for m in (15, 31, 63):
        p = W.manufactured(m, 128, 1.5)
        U = O.solve_gmres(p, tol=1e-12).x
        errs.append(np.abs(U - p.exact(W.grid_x(m), W.grid_t(128)[1:])).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 1.0) < 0.15), rates


@pytest.mark.slow
def test_c1_dense_direct_equals_gmres():
    p = W.manufactured_c1()
    U1 = O.solve_direct(p)
    r = O.solve_gmres(p, tol=1e-13)
    assert np.linalg.norm(r.x - U1) / np.linalg.norm(U1) < 1e-12
