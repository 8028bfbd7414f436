"""Pins of the oracle's BCCB preconditioners S2 (eq. (x1)) and S2~ (eq. (xc)) of Section 3.1
and their 2-D FFT diagonalisation (Section 3.2)."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W


def _strang_of_toeplitz(T: np.ndarray) -> np.ndarray:
    """Generic Strang circulant of a Toeplitz matrix: copy the central diagonals.  For order
    N, the first column holds t_i (i = 0 .. floor((N-1)/2)) and t_{-i} at N - i for the
    remaining i (t_k = T[k][0], t_{-k} = T[0][k])."""
    N = T.shape[0]
    c = np.zeros(N)
    for i in range(N):
        c[i] = T[i, 0] if i <= (N - 1) // 2 else T[0, N - i]
    return c


@pytest.mark.parametrize("N", [2, 3, 7, 8, 15, 16])
@pytest.mark.parametrize("alpha", [1.2, 1.7])
def test_space_column_is_the_strang_circulant_of_G(N, alpha):
    g = O.grunwald_weights(alpha, N)
    G = O.space_matrix(alpha, np.ones(N), np.zeros(N), 1.0)  # dx = 1, d+ = 1, d- = 0: J = G
    np.testing.assert_array_equal(O.strang_space_column(g, N), _strang_of_toeplitz(G))


@pytest.mark.parametrize("N", [5, 16, 31, 64, 255])
@pytest.mark.parametrize("alpha", [1.05, 1.5, 1.95])
def test_strang_space_eigenvalues_in_the_disc(N, alpha):
    """Theorem of Section 3.1: every eigenvalue of s(G) and s(G^T) lies in |z + alpha| < alpha,
    so Re lambda(s(J)) < 0 and S2 is invertible for a stable BVM."""
    g = O.grunwald_weights(alpha, N)
    c = O.strang_space_column(g, N)
    for lam in (np.fft.fft(c), np.fft.fft(c[(-np.arange(N)) % N])):
        assert np.all(np.abs(lam + alpha) < alpha)
    lamJ, _ = O.strang_space_symbol(alpha, np.full(N, 0.6), np.full(N, 0.5), 0.1)
    assert np.all(lamJ.real < 0.0)


def test_space_symbol_matches_J_on_the_central_diagonals():
    """With constant d+-, J is Toeplitz and s(J) agrees with it on the central diagonals."""
    N, alpha, dx = 15, 1.6, 2.0 / 16
    dp, dm = np.full(N, 0.6), np.full(N, 0.5)
    J = O.space_matrix(alpha, dp, dm, dx)
    _, c = O.strang_space_symbol(alpha, dp, dm, dx)
    C = O.strang_circulant(c)
    for i in range(N):
        for j in range(N):
            if abs(i - j) <= (N - 1) // 2:
                assert abs(C[i, j] - J[i, j]) <= 1e-12 * np.abs(J).max()


@pytest.mark.parametrize("shifted", [False, True])
@pytest.mark.parametrize("kind", ["trapezoidal", "gbdf3"])
def test_bccb_fft_form_inverts_the_dense_matrix(kind, shifted):
    p = W.tiny(15, 16, 1.6, 1, kind)
    D = O.bccb_dense(p, shifted)
    P = O.BccbPreconditioner(p, shifted)
    v = np.random.default_rng(0).standard_normal(p.s * p.m)
    assert np.linalg.norm(D @ P.apply(v).reshape(-1) - v) <= 1e-13 * np.linalg.norm(v)
    # eigenvalues of the dense matrix = eq. (1.13), matched one to one
    from scipy.optimize import linear_sum_assignment
    ev = np.linalg.eigvals(D)
    ref = O.bccb_eigs(p, shifted).reshape(-1)
    dist = np.abs(ev[:, None] - ref[None, :])
    r, c = linear_sum_assignment(dist)
    assert dist[r, c].max() <= 1e-9 * np.abs(ref).max()


def test_shifted_variant_moves_only_the_zero_frequency():
    p = W.tiny(7, 8, 1.5, 2, "gbdf3")
    e0, e1 = O.bccb_eigs(p, False), O.bccb_eigs(p, True)
    F = O.formula("gbdf3")
    phi, _ = O.strang_eigs(F, p.s)
    assert abs(phi[0]) < 1e-15                     # phi_0 = rho(1) = 0
    np.testing.assert_array_equal(e0[1:], e1[1:])
    np.testing.assert_allclose(e1[0] - e0[0], np.full(p.m, phi[p.s - 1].real), rtol=1e-13)


@pytest.mark.parametrize("pc", ["bccb", "bccb_shifted"])
def test_bccb_gmres_reaches_the_direct_solution(pc):
    p = W.tiny(15, 16, 1.6, 1, "gbdf3")
    U = O.solve_direct(p)
    r = O.solve_gmres(p, tol=1e-12, precond=pc)
    assert r.converged and np.linalg.norm(r.x - U) <= 1e-9 * np.linalg.norm(U)
    # more iterations than the block-circulant S on the same system (Tables 1-2 ordering)
    assert r.iters > O.solve_gmres(p, tol=1e-12).iters


@pytest.mark.parametrize("kind", ["trapezoidal", "gbdf3", "gam5"])
@pytest.mark.parametrize("s", [8, 16, 64])
def test_shift_is_the_real_part_of_the_last_time_eigenvalue(kind, s):
    """Eq. (xc): S2~ replaces the eigenvalue phi_0 = rho(1) = 0 of s(A) by the real part of its
    last eigenvalue.  Independent of the FFT: the eigenvalue closed form after eq. (1.13),
    phi_j = sum_r alpha_{r+nu} w^{rj} with w = e^{2 pi i/s} (order s), gives at j = s-1 the
    real part sum_r alpha_{r+nu} cos(2 pi r/s); and changing only the zero frequency adds
    exactly shift * (1/s) 1 1^T (x) I_m to the dense matrix (the projector on constant time
    vectors).  A shift taken at another frequency, a complex shift or one added at another
    frequency fails here."""
    p = W.tiny(5, s, 1.4, 3, kind)
    F = O.formula(kind)
    r = np.arange(F.mu + 1) - F.nu
    shift = float(np.sum(F.alpha * np.cos(2 * np.pi * r / s)))
    D0, D1 = O.bccb_dense(p, False), O.bccb_dense(p, True)
    expect = shift / s * np.kron(np.ones((s, s)), np.eye(p.m))
    np.testing.assert_allclose(D1 - D0, expect, rtol=0, atol=1e-13 * max(1.0, np.abs(D0).max()))
    e0, e1 = O.bccb_eigs(p, False), O.bccb_eigs(p, True)
    np.testing.assert_allclose(e1[0] - e0[0], shift, rtol=1e-12, atol=1e-15)
    if kind in ("trapezoidal", "gam5"):  # rho(z) = z - 1 on these: shift = 1 - cos(2 pi/s)
        assert abs(shift - (1 - np.cos(2 * np.pi / s))) <= 1e-15


def test_shifted_bccb_counts_follow_table_1():
    """Table 1 (alpha = 1.2), column S2~: with the printed shift, left preconditioning and the
    preconditioned-residual test of Section 4, every count is within 4 of the table.  (A shift
    at the middle frequency, Re phi_{s/2}, needs 31-225 more iterations here.)  Table 2
    (alpha = 1.5) is not reproduced by this reading, nor by a shift of |phi_1| or by the
    (s+1)-form system: the S2~ table counts are unpinned there."""
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "example41_its.txt"),
                      comments="#")
    for a, m, s, _, _, _, s2t in rows:
        if a != 1.2:
            continue
        p = W.example41(float(a), int(m), int(s))
        n = O.solve_gmres(p, tol=1e-8, precond="bccb_shifted", side="left", maxit=3000).iters
        assert abs(n - s2t) <= 4, (a, m, s, n, s2t)


def test_shift_readings_against_table_2():
    """Table 2 (alpha = 1.5), column S2~, under two readings of the shift of eq. (xc) (left
    preconditioning, the preconditioned-residual test of Section 4): with |phi_1| in place of
    Re phi_{s-1} every count is within 9 of the table, and like the table's they do not fall as
    s grows; with the printed Re phi_{s-1} the counts fall with s at every m and miss the table
    by up to 19.  The library keeps the printed reading (its Table 1 counts are within 4), so
    S2~ is unpinned against Table 2."""
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "example41_its.txt"),
                      comments="#")
    got = {"printed": {}, "abs_phi1": {}}
    miss = {"printed": 0, "abs_phi1": 0}
    for a, m, s, _, _, _, s2t in rows:
        if a != 1.5:
            continue
        p = W.example41(float(a), int(m), int(s))
        J, F, tau, _ = O.problem_matrices(p)
        A, B, a0, b0, Bfull = O.s_form(F, p.s)
        b = (tau * (Bfull @ p.f) - np.outer(a0, p.u0) + tau * np.outer(b0, J @ p.u0)).reshape(-1)
        mv = lambda z: O.apply_M(J, A, B, tau, z.reshape(p.s, p.m)).reshape(-1)
        phi, _ = O.strang_eigs(F, p.s)
        for name, shift in (("printed", phi[p.s - 1].real), ("abs_phi1", abs(phi[1]))):
            pc = O.BccbPreconditioner(p, False)
            pc.eig = pc.eig.copy()
            pc.eig[0, :] += shift - phi[0]  # phi_0 = rho(1) = 0 replaced by the shift
            n = O.gmres(mv, lambda v: pc.apply(v).reshape(-1), b, None, 1e-8, 20, 3000, "left").iters
            got[name][(int(m), int(s))] = n
            miss[name] = max(miss[name], abs(n - int(s2t)))
    assert miss["abs_phi1"] <= 9 and miss["printed"] >= 15, miss
    for m in (24, 48, 96):
        assert got["printed"][(m, 128)] < got["printed"][(m, 16)]
        assert got["abs_phi1"][(m, 128)] >= got["abs_phi1"][(m, 16)]
