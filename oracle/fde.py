"""Plain, slow, FP64 reference for the Strang-preconditioned all-at-once BVM method.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``): imported by tests, smoke() and the
CPU-baseline leg of the benchmark, never by the product path.

Every function states the passage of the paper it follows.  Layout convention: a
space-time vector is an array ``U[s][m]`` whose row n holds u_{n+1} (the unknowns
u_1..u_s of the s-form system, u_0 being the given initial value).

Readings taken where the paper is silent or garbled (all listed in the design notes):

* s-form.  The (s+1)-form of eq. (1.10) keeps u_0 as an unknown; here u_0 is moved to
  the right-hand side, so M is (s m) x (s m) and the Strang circulants have order s.
* Formulas.  The paper prints no BVM coefficients.  Trapezoidal (nu=mu=1) and the
  third-order generalized BDF (nu=2, mu=3) with one initial and one final formula are
  used; each GBDF3 formula is the unique four-point formula of order 3 whose beta is
  supported only on the derivative node.  The fifth-order GAM of Section 4 (nu=2, mu=4)
  takes, for its one initial and two final formulas, one-step Adams formulas on the five
  nodes nearest the boundary.
* Stopping rule.  True residual ||b - M x||_2 / ||b||_2 <= tol, right preconditioning;
  left preconditioning with the preconditioned residual (the convention under which
  Section 4 counts iterations) is available for reproducing its tables.
* Diffusion coefficients depend on x only (eq. (1.10) needs a time-independent J).
"""
from __future__ import annotations

import dataclasses
from fractions import Fraction
from typing import Callable, Optional

import numpy as np
import scipy.linalg

__all__ = [
    "grunwald_weights", "space_matrix", "space_matrix_entries", "Formula",
    "trapezoidal", "gbdf3", "gam5", "formula", "bvm_matrices", "s_form", "all_at_once",
    "problem_matrices", "problem_system", "solve_direct", "strang_columns",
    "strang_circulant", "strang_eigs", "strang_dense", "StrangPreconditioner",
    "apply_M", "gmres", "GmresResult", "solve_gmres", "true_relres", "strang_space_column",
    "strang_space_symbol", "bccb_eigs", "bccb_dense", "BccbPreconditioner",
    "hessenberg_lu", "hessenberg_lu_solve", "HessenbergPreconditioner",
]


# ======================================================================================
# Section 2.1: shifted Grunwald semi-discretization
# ======================================================================================
def grunwald_weights(alpha: float, n: int) -> np.ndarray:
    """g_0..g_n of eq. (1.2) by its recurrence g_{k+1} = (1 - (alpha+1)/(k+1)) g_k, g_0 = 1."""
    g = np.empty(n + 1, dtype=np.float64)
    g[0] = 1.0
    for k in range(n):
        g[k + 1] = (1.0 - (alpha + 1.0) / (k + 1.0)) * g[k]
    return g


def space_matrix(alpha: float, d_plus: np.ndarray, d_minus: np.ndarray, dx: float) -> np.ndarray:
    """Dense J_N = dx^{-alpha} (D_+ G_alpha + D_- G_alpha^T), eq. (1.4)-(1.5).

    G_alpha is the lower-Hessenberg Toeplitz matrix with first column (g_1..g_N) and
    first row (g_1, g_0, 0, ..., 0): G[i][j] = g_{i-j+1} for j <= i+1, else 0.
    """
    m = len(d_plus)
    g = grunwald_weights(alpha, m)
    G = np.zeros((m, m))
    for i in range(m):
        for j in range(m):
            k = i - j + 1
            if 0 <= k <= m:
                G[i, j] = g[k]
    return (np.diag(d_plus) @ G + np.diag(d_minus) @ G.T) / dx ** alpha


def space_matrix_entries(alpha: float, d_plus: np.ndarray, d_minus: np.ndarray,
                         dx: float) -> np.ndarray:
    """Dense J_N from its entry formula p_ij in the proof of Proposition 2.2, eq. (1.10t)."""
    m = len(d_plus)
    g = grunwald_weights(alpha, m + 1)
    rp = np.asarray(d_plus, dtype=np.float64) / dx ** alpha
    rm = np.asarray(d_minus, dtype=np.float64) / dx ** alpha
    P = np.zeros((m, m))
    for i in range(m):
        for j in range(m):
            if j == i:
                P[i, j] = (rp[i] + rm[i]) * g[1]
            elif j == i - 1:
                P[i, j] = rp[i] * g[2] + rm[i] * g[0]
            elif j == i + 1:
                P[i, j] = rp[i] * g[0] + rm[i] * g[2]
            elif j < i - 1:
                P[i, j] = rp[i] * g[i - j + 1]
            else:
                P[i, j] = rm[i] * g[j - i + 1]
    return P


# ======================================================================================
# Section 2.2: boundary value methods, eq. (1.7)-(1.10)
# ======================================================================================
@dataclasses.dataclass
class Formula:
    """A BVM: main formula (eq. (1.7)) plus nu-1 initial (eq. (1.8)) and mu-nu final
    (eq. (1.9)) formulas.  Coefficient index i multiplies u_{n-nu+i} in the main formula,
    u_i in an initial formula, and u_{s-mu+i} in a final formula."""
    name: str
    nu: int
    mu: int
    alpha: np.ndarray
    beta: np.ndarray
    alpha_init: np.ndarray   # [nu-1][mu+1]
    beta_init: np.ndarray
    alpha_fin: np.ndarray    # [mu-nu][mu+1]
    beta_fin: np.ndarray


def trapezoidal() -> Formula:
    """Trapezoidal rule as a BVM with (nu, mu-nu) = (1, 0): u_n - u_{n-1} = h/2 (g_{n-1} + g_n)."""
    e = np.zeros((0, 2))
    return Formula("trapezoidal", 1, 1, np.array([-1.0, 1.0]), np.array([0.5, 0.5]),
                   e, e, e, e)


def gbdf3() -> Formula:
    """Third-order generalized BDF with (nu, mu-nu) = (2, 1).

    main     (1/6) u_{n-2} - u_{n-1} + (1/2) u_n + (1/3) u_{n+1} = h g_n
    initial  -(1/3) u_0 - (1/2) u_1 + u_2 - (1/6) u_3 = h g_1
    final    -(1/3) u_{s-3} + (3/2) u_{s-2} - 3 u_{s-1} + (11/6) u_s = h g_s   (BDF3)
    """
    return Formula(
        "gbdf3", 2, 3,
        np.array([1 / 6, -1.0, 0.5, 1 / 3]), np.array([0.0, 0.0, 1.0, 0.0]),
        np.array([[-1 / 3, -0.5, 1.0, -1 / 6]]), np.array([[0.0, 1.0, 0.0, 0.0]]),
        np.array([[-1 / 3, 1.5, -3.0, 11 / 6]]), np.array([[0.0, 0.0, 0.0, 1.0]]),
    )


def _poly_mul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _adams_weights(nodes, lo, hi):
    """w_j = integral over [lo, hi] of the Lagrange basis polynomial of node j (exact
    rationals): the weights of the quadrature that integrates the interpolant of g through
    the given nodes."""
    w = []
    for j, tj in enumerate(nodes):
        poly, den = [Fraction(1)], Fraction(1)
        for i, ti in enumerate(nodes):
            if i != j:
                poly = _poly_mul(poly, [Fraction(-ti), Fraction(1)])
                den *= tj - ti
        w.append(sum(c * (Fraction(hi) ** (q + 1) - Fraction(lo) ** (q + 1)) / (q + 1)
                     for q, c in enumerate(poly)) / den)
    return w


def gam5() -> Formula:
    """Fifth-order generalized Adams method, mu = 4, nu = 2 (the BVM of Section 4).

    Every row is a one-step Adams formula u_r - u_{r-1} = h sum_i beta_i g_{c+i}: beta
    integrates, over [t_{r-1}, t_r], the quartic interpolating g at the five consecutive
    nodes t_c..t_{c+4}.  The main formula (rows 2..s-2) centres those nodes on u_r
    (c = r - 2); the initial row r = 1 uses t_0..t_4 and the final rows r = s-1, s use
    t_{s-4}..t_s."""
    nodes = range(5)
    z = [Fraction(0)] * 5

    def row(r_local):
        a = list(z)
        a[r_local - 1], a[r_local] = Fraction(-1), Fraction(1)
        return a, _adams_weights(nodes, r_local - 1, r_local)

    a_main, b_main = row(2)
    a_i1, b_i1 = row(1)
    a_f1, b_f1 = row(3)
    a_f2, b_f2 = row(4)
    f = lambda rows: np.array([[float(v) for v in r] for r in rows])
    return Formula("gam5", 2, 4, f([a_main])[0], f([b_main])[0], f([a_i1]), f([b_i1]),
                   f([a_f1, a_f2]), f([b_f1, b_f2]))


def formula(kind: str) -> Formula:
    return {"trapezoidal": trapezoidal, "gbdf3": gbdf3, "gam5": gam5}[kind]()


def bvm_matrices(F: Formula, s: int):
    """The (s+1)x(s+1) matrices A, B of eq. (1.10) (called Ahat, Bhat here).

    Row 0 is the initial condition u_0 = u_0 (first row of A = e_1^T, of B = 0);
    rows 1..nu-1 the initial formulas on u_0..u_mu; rows nu..s-mu+nu the main formula
    on u_{n-nu}..u_{n-nu+mu}; rows s-mu+nu+1..s the final formulas on u_{s-mu}..u_s.
    """
    nu, mu = F.nu, F.mu
    if s < mu + 1:
        raise ValueError("s must be at least mu+1")
    Ah = np.zeros((s + 1, s + 1))
    Bh = np.zeros((s + 1, s + 1))
    Ah[0, 0] = 1.0
    for j in range(1, nu):
        Ah[j, 0:mu + 1] = F.alpha_init[j - 1]
        Bh[j, 0:mu + 1] = F.beta_init[j - 1]
    for n in range(nu, s - mu + nu + 1):
        Ah[n, n - nu:n - nu + mu + 1] = F.alpha
        Bh[n, n - nu:n - nu + mu + 1] = F.beta
    for r, n in enumerate(range(s - mu + nu + 1, s + 1)):
        Ah[n, s - mu:s + 1] = F.alpha_fin[r]
        Bh[n, s - mu:s + 1] = F.beta_fin[r]
    return Ah, Bh


def s_form(F: Formula, s: int):
    """Eliminate u_0 from eq. (1.10): A = Ahat[1:,1:], B = Bhat[1:,1:], a0 = Ahat[1:,0],
    b0 = Bhat[1:,0], and Bfull = Bhat[1:,:] (which multiplies f_0..f_s)."""
    Ah, Bh = bvm_matrices(F, s)
    return Ah[1:, 1:], Bh[1:, 1:], Ah[1:, 0], Bh[1:, 0], Bh[1:, :]


def all_at_once(J: np.ndarray, F: Formula, s: int, tau: float, f: np.ndarray, u0: np.ndarray):
    """Dense M = A (x) I - tau B (x) J and right-hand side of eq. (1.10) in s-form:

        b = tau (Bhat[1:,:] (x) I) [f_0;..;f_s] - a0 (x) u0 + tau b0 (x) (J u0).

    f is [s+1][m]; the returned b is flattened time-major ([s][m] -> s*m).
    """
    m = J.shape[0]
    A, B, a0, b0, Bfull = s_form(F, s)
    M = np.kron(A, np.eye(m)) - tau * np.kron(B, J)
    rhs = tau * (Bfull @ f) - np.outer(a0, u0) + tau * np.outer(b0, J @ u0)
    return M, rhs.reshape(-1)


def problem_matrices(p):
    """J, formula, tau and dx of a ``workloads.Problem`` (grid of Section 2.1, mesh of eq. (1.7))."""
    dx = (p.xR - p.xL) / (p.m + 1)
    tau = (p.T - p.t0) / p.s
    J = space_matrix(p.alpha, p.d_plus, p.d_minus, dx)
    return J, formula(p.bvm), tau, dx


def problem_system(p):
    J, F, tau, _ = problem_matrices(p)
    return all_at_once(J, F, p.s, tau, p.f, p.u0)


def solve_direct(p) -> np.ndarray:
    """O1: dense LAPACK solve (dgesv) of the s-form system; returns U[s][m]."""
    M, b = problem_system(p)
    return np.linalg.solve(M, b).reshape(p.s, p.m)


# ======================================================================================
# Section 3.1: Strang block-circulant preconditioner S = s(A) (x) I - h s(B) (x) J, eq. (1.11)
# ======================================================================================
def strang_columns(F: Formula, s: int):
    """First columns of the order-s circulants s(A), s(B) of eq. (1.11).

    s(A) keeps the main band of A and wraps it around: row n carries alpha_i in column
    (n - nu + i) mod s, so the first column holds alpha_i at index (nu - i) mod s.
    """
    cA = np.zeros(s)
    cB = np.zeros(s)
    for i in range(F.mu + 1):
        cA[(F.nu - i) % s] += F.alpha[i]
        cB[(F.nu - i) % s] += F.beta[i]
    return cA, cB


def strang_circulant(c: np.ndarray) -> np.ndarray:
    """Dense circulant with first column c: C[i][j] = c[(i - j) mod s]."""
    s = len(c)
    idx = (np.arange(s)[:, None] - np.arange(s)[None, :]) % s
    return c[idx]


def strang_eigs(F: Formula, s: int):
    """Eigenvalues lambda_k, mu_k (k = 0..s-1) of s(A), s(B): the DFT (e^{-2 pi i jk/s})
    of their first columns, so that s(A) = F^{-1} diag(lambda) F for the DFT matrix F."""
    cA, cB = strang_columns(F, s)
    return np.fft.fft(cA), np.fft.fft(cB)


def strang_dense(J: np.ndarray, F: Formula, s: int, tau: float) -> np.ndarray:
    cA, cB = strang_columns(F, s)
    m = J.shape[0]
    return np.kron(strang_circulant(cA), np.eye(m)) - tau * np.kron(strang_circulant(cB), J)


class StrangPreconditioner:
    """S^{-1} v by the time-axis FFT diagonalisation of Section 3.2:

        S^{-1} = (F^{-1} (x) I) blockdiag(lambda_k I - tau mu_k J)^{-1} (F (x) I).

    The blocks K_k = lambda_k I - tau mu_k J are factored with LAPACK zgetrf (partial
    pivoting) for k = 0..floor(s/2); K_{s-k} = conj(K_k) because J, A and B are real.
    """

    def __init__(self, J: np.ndarray, F: Formula, s: int, tau: float, progress=None):
        self.s = s
        self.m = J.shape[0]
        lam, mu = strang_eigs(F, s)
        self.lam = lam[: s // 2 + 1]
        self.mu = mu[: s // 2 + 1]
        eye = np.eye(self.m)
        self.factors = []
        for k, (lk, mk) in enumerate(zip(self.lam, self.mu)):
            self.factors.append(scipy.linalg.lu_factor(lk * eye - tau * mk * J, check_finite=False))
            if progress and (k + 1) % 16 == 0:
                progress(f"oracle: {k + 1} of {len(self.lam)} blocks factored")

    def block(self, k: int, J: np.ndarray, tau: float) -> np.ndarray:
        return self.lam[k] * np.eye(self.m) - tau * self.mu[k] * J

    def apply(self, V: np.ndarray) -> np.ndarray:
        V = V.reshape(self.s, self.m)
        Vh = np.fft.rfft(V, axis=0)
        Wh = np.empty_like(Vh)
        for k, lu in enumerate(self.factors):
            Wh[k] = scipy.linalg.lu_solve(lu, Vh[k], check_finite=False)
        return np.fft.irfft(Wh, n=self.s, axis=0)


# ======================================================================================
# The blocks of S through one Hessenberg form of J (not in the paper): every block
# K_k = lambda_k I - tau mu_k J is a shift of the same matrix, so with J = Q H Q^T
# (Q orthogonal, H upper Hessenberg) K_k = Q (lambda_k I - tau mu_k H) Q^T, and each shifted
# Hessenberg matrix is factored in O(m^2).
# ======================================================================================
def hessenberg_lu(C: np.ndarray):
    """Gaussian elimination with partial pivoting on an upper Hessenberg matrix C: at step i
    only rows i and i+1 hold entries in column i, so the pivot is the larger of the two.
    Returns (U, l, swapped): U upper triangular, l[i] the multiplier of step i, swapped[i]
    whether rows i and i+1 were exchanged first; C = P_0 L_0 P_1 L_1 ... U in product form."""
    U = np.array(C, dtype=np.complex128)
    m = U.shape[0]
    l = np.zeros(max(m - 1, 0), dtype=np.complex128)
    swapped = np.zeros(max(m - 1, 0), dtype=bool)
    for i in range(m - 1):
        if abs(U[i + 1, i]) > abs(U[i, i]):
            U[[i, i + 1], i:] = U[[i + 1, i], i:]
            swapped[i] = True
        l[i] = U[i + 1, i] / U[i, i]
        U[i + 1, i:] -= l[i] * U[i, i:]
        U[i + 1, i] = 0.0
    return U, l, swapped


def hessenberg_lu_solve(U: np.ndarray, l: np.ndarray, swapped: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Solve C z = y with the factors of ``hessenberg_lu``: replay the row exchanges and
    eliminations on y, then back substitution with U."""
    z = np.array(y, dtype=np.complex128)
    for i in range(len(l)):
        if swapped[i]:
            z[[i, i + 1]] = z[[i + 1, i]]
        z[i + 1] -= l[i] * z[i]
    return scipy.linalg.solve_triangular(U, z, lower=False, check_finite=False)


class HessenbergPreconditioner:
    """S^{-1} v with the blocks solved through J = Q H Q^T (scipy's Householder reduction):
    time rfft, then for each k: Q^T v_k, the shifted Hessenberg solve, Q times the result;
    inverse rfft.  The same operator as ``StrangPreconditioner`` up to rounding."""

    def __init__(self, J: np.ndarray, F: Formula, s: int, tau: float):
        self.s, self.m = s, J.shape[0]
        H, Q = scipy.linalg.hessenberg(J, calc_q=True)
        self.H, self.Q = H, Q
        lam, mu = strang_eigs(F, s)
        self.lam, self.mu = lam[: s // 2 + 1], mu[: s // 2 + 1]
        eye = np.eye(self.m)
        self.factors = [hessenberg_lu(lk * eye - tau * mk * H) for lk, mk in zip(self.lam, self.mu)]

    def apply(self, V: np.ndarray) -> np.ndarray:
        V = V.reshape(self.s, self.m)
        Vh = np.fft.rfft(V, axis=0)
        Wh = np.empty_like(Vh)
        for k, (U, l, sw) in enumerate(self.factors):
            Wh[k] = self.Q @ hessenberg_lu_solve(U, l, sw, self.Q.T @ Vh[k])
        return np.fft.irfft(Wh, n=self.s, axis=0)


# ======================================================================================
# Section 3.1, BCCB variants: S2 = s(A) (x) I - h s(B) (x) s(J), eq. (x1), and the shifted
# S2~ = s~(A) (x) I - h s(B) (x) s(J), eq. (xc); Section 3.2 (their 2-D FFT diagonalisation)
# ======================================================================================
def strang_space_column(g: np.ndarray, N: int) -> np.ndarray:
    """First column of the order-N circulant s(G_alpha) as printed in Section 3.1:
    g_1, ..., g_{floor((N+1)/2)}, then zeros, then g_0 in the last position."""
    c = np.zeros(N)
    h = (N + 1) // 2
    c[:h] = g[1:h + 1]
    if N - 1 >= h:
        c[N - 1] = g[0]
    return c


def strang_space_symbol(alpha: float, d_plus: np.ndarray, d_minus: np.ndarray, dx: float):
    """Eigenvalues of s(J_N) = dx^{-alpha} (dbar+ s(G) + dbar- s(G^T)) with dbar the means of
    d+ and d- (Section 3.1), in the DFT convention C = F^{-1} diag(fft(c)) F.

    s(G^T) is read as s(G)^T (the printed first column of s(G^T) is garbled), whose first
    column is c[(-i) mod N] and whose eigenvalues are those of s(G) at frequency -j."""
    N = len(d_plus)
    g = grunwald_weights(alpha, N)
    cG = strang_space_column(g, N)
    cGT = cG[(-np.arange(N)) % N]
    dbp, dbm = float(np.mean(d_plus)), float(np.mean(d_minus))
    c = dx ** (-alpha) * (dbp * cG + dbm * cGT)
    return np.fft.fft(c), c


def bccb_eigs(p, shifted: bool = False):
    """Eigenvalues of S2 (or S2~) as an [s][m] array: phi_k - h psi_k lambda_j(s(J)),
    eq. (1.13) rebased to the order-s circulants of the s-form.  The shifted variant replaces
    phi_0 (= rho(1) = 0) by Re(phi_{s-1}), the last eigenvalue of s(A)."""
    J, F, tau, dx = problem_matrices(p)
    phi, psi = strang_eigs(F, p.s)
    if shifted:
        phi = phi.copy()
        phi[0] = phi[p.s - 1].real
    lam, _ = strang_space_symbol(p.alpha, p.d_plus, p.d_minus, dx)
    return phi[:, None] - tau * psi[:, None] * lam[None, :]


def bccb_dense(p, shifted: bool = False) -> np.ndarray:
    """S2 (S2~) assembled from circulants: the time circulants from their first columns (for
    S2~, s~(A) = F^{-1} diag(phi~) F) and s(J) from its first column."""
    J, F, tau, dx = problem_matrices(p)
    cA, cB = strang_columns(F, p.s)
    if shifted:
        phi = np.fft.fft(cA)
        phi[0] = phi[p.s - 1].real
        cA = np.fft.ifft(phi).real
    _, cJ = strang_space_symbol(p.alpha, p.d_plus, p.d_minus, dx)
    return np.kron(strang_circulant(cA), np.eye(p.m)) - tau * np.kron(strang_circulant(cB),
                                                                      strang_circulant(cJ))


class BccbPreconditioner:
    """S2^{-1} v (or S2~^{-1} v) by the 2-D DFT: FFT along time and space, divide by the
    eigenvalues, inverse FFTs (Section 3.2)."""

    def __init__(self, p, shifted: bool = False):
        self.s, self.m = p.s, p.m
        self.eig = bccb_eigs(p, shifted)

    def apply(self, V: np.ndarray) -> np.ndarray:
        V = np.asarray(V, dtype=np.float64).reshape(self.s, self.m)
        return np.fft.ifft2(np.fft.fft2(V) / self.eig).real


def apply_M(J: np.ndarray, A: np.ndarray, B: np.ndarray, tau: float, Z: np.ndarray) -> np.ndarray:
    """M z for z = U[s][m]: (A (x) I) z - tau (B (x) J) z = A U - tau B U J^T (dense J, no FFT)."""
    return A @ Z - tau * (B @ Z) @ J.T


# ======================================================================================
# GMRES (Section 2.2 end, Section 4): restarted, right-preconditioned, MGS + Givens
# ======================================================================================
@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    restarts: int
    converged: bool
    relres: float
    history: list


def gmres(matvec: Callable, precond: Optional[Callable], b: np.ndarray, x0: Optional[np.ndarray] = None,
          tol: float = 1e-10, restart: int = 20, maxit: int = 1000,
          side: str = "right", progress=None) -> GmresResult:
    """Restarted GMRES(restart) with right preconditioning, as flexible GMRES (the
    preconditioned directions z_j are kept), modified Gram-Schmidt Arnoldi and Givens
    rotations for the small least-squares problem.  Convergence is declared only on
    the recomputed true residual ||b - M x|| <= tol ||b||.

    side="left" runs GMRES on P^{-1} M x = P^{-1} b instead (the form in which Section 3.3
    states its convergence theorem and Section 4 counts iterations): the Arnoldi vectors
    span P^{-1} M's Krylov space, x is updated with them directly, and the stopping test
    is on the preconditioned residual, ||P^{-1}(b - M x)|| <= tol ||P^{-1} b||."""
    if side == "left":
        return _gmres_left(matvec, precond, b, x0, tol, restart, maxit)
    if side != "right":
        raise ValueError(f"side must be 'right' or 'left', got {side!r}")
    n = b.size
    bnorm = np.linalg.norm(b)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64).reshape(-1)
    P = precond if precond is not None else (lambda v: v)
    its = 0
    restarts = 0
    history = []
    if bnorm == 0.0:
        return GmresResult(np.zeros(n), 0, 0, True, 0.0, history)
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        history.append(beta / bnorm)
        if beta <= tol * bnorm:
            return GmresResult(x, its, restarts, True, beta / bnorm, history)
        if its >= maxit:
            return GmresResult(x, its, restarts, False, beta / bnorm, history)
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = P(V[j]).reshape(-1)
            w = matvec(Z[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if progress:
                progress(f"oracle: GMRES iteration {its}, estimate {history[-1]:.2e}")
            if abs(g[j + 1]) <= tol * bnorm or its >= maxit:
                break
        y = scipy.linalg.solve_triangular(H[:k, :k], g[:k])
        x = x + Z[:k].T @ y
        restarts += 1


def _gmres_left(matvec, precond, b, x0, tol, restart, maxit) -> GmresResult:
    """Left-preconditioned restarted GMRES (see ``gmres``); relres is the preconditioned one."""
    n = b.size
    P = precond if precond is not None else (lambda v: v)
    op = lambda v: np.asarray(P(matvec(v)), dtype=np.float64).reshape(-1)
    pb = np.asarray(P(b), dtype=np.float64).reshape(-1)
    pbnorm = np.linalg.norm(pb)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64).reshape(-1)
    its, restarts, history = 0, 0, []
    if pbnorm == 0.0:
        return GmresResult(np.zeros(n), 0, 0, True, 0.0, history)
    while True:
        r = np.asarray(P(b - matvec(x)), dtype=np.float64).reshape(-1)
        beta = np.linalg.norm(r)
        history.append(beta / pbnorm)
        if beta <= tol * pbnorm:
            return GmresResult(x, its, restarts, True, beta / pbnorm, history)
        if its >= maxit:
            return GmresResult(x, its, restarts, False, beta / pbnorm, history)
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs, sn, g = np.zeros(restart), np.zeros(restart), np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            w = op(V[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j], H[j + 1, j] = d, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            history.append(abs(g[j + 1]) / pbnorm)
            if abs(g[j + 1]) <= tol * pbnorm or its >= maxit:
                break
        x = x + V[:k].T @ scipy.linalg.solve_triangular(H[:k, :k], g[:k])
        restarts += 1


def true_relres(p, U: np.ndarray) -> float:
    """||b - M u||_2 / ||b||_2 in FP64 with the dense-J product (any size that fits in RAM)."""
    J, F, tau, _ = problem_matrices(p)
    A, B, a0, b0, Bfull = s_form(F, p.s)
    b = tau * (Bfull @ p.f) - np.outer(a0, p.u0) + tau * np.outer(b0, J @ p.u0)
    r = b - apply_M(J, A, B, tau, np.asarray(U, dtype=np.float64).reshape(p.s, p.m))
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def solve_gmres(p, tol: float = 1e-13, restart: int = 20, maxit: int = 2000,
                x0: Optional[np.ndarray] = None, preconditioned: bool = True,
                precond: str = "strang", side: str = "right", progress=None) -> GmresResult:
    """O2: preconditioned GMRES(restart) on the s-form system of a Problem; precond is
    "strang" (S, eq. (1.11)), "bccb" (S2, eq. (x1)), "bccb_shifted" (S2~, eq. (xc)) or
    "none" (the unpreconditioned column I of Tables 1-2).  progress, if given, is called with a
    line of text as the long steps finish (every 16 block factorizations, every iteration)."""
    J, F, tau, _ = problem_matrices(p)
    A, B, a0, b0, Bfull = s_form(F, p.s)
    b = (tau * (Bfull @ p.f) - np.outer(a0, p.u0) + tau * np.outer(b0, J @ p.u0)).reshape(-1)
    mv = lambda z: apply_M(J, A, B, tau, z.reshape(p.s, p.m)).reshape(-1)
    if not preconditioned or precond == "none":
        pc = None
    elif precond == "strang":
        pc = StrangPreconditioner(J, F, p.s, tau, progress).apply
    elif precond == "strang_hessenberg":
        pc = HessenbergPreconditioner(J, F, p.s, tau).apply
    elif precond in ("bccb", "bccb_shifted"):
        pc = BccbPreconditioner(p, shifted=precond == "bccb_shifted").apply
    else:
        raise ValueError(f"unknown preconditioner {precond!r}")
    res = gmres(mv, (lambda v: pc(v).reshape(-1)) if pc else None, b, x0, tol, restart, maxit,
                side, progress if side == "right" else None)
    res.x = res.x.reshape(p.s, p.m)
    return res
