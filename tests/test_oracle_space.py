"""Pins of the oracle's spatial part (Section 2.1) against closed forms and the paper's propositions."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.special

import oracle as O
import workloads as W


@pytest.mark.parametrize("alpha", [1.05, 1.3, 1.5, 1.8, 1.95])
def test_weights_closed_form(alpha):
    """eq. (1.2): g_k = (-1)^k C(alpha, k) = Gamma(k-alpha)/(Gamma(-alpha) Gamma(k+1))."""
    n = 60
    g = O.grunwald_weights(alpha, n)
    k = np.arange(n + 1)
    binom = (-1.0) ** k * scipy.special.binom(alpha, k)
    np.testing.assert_allclose(g, binom, rtol=1e-13, atol=1e-16)
    kk = np.arange(2, 40)
    gam = scipy.special.gamma(kk - alpha) / (scipy.special.gamma(-alpha) * scipy.special.gamma(kk + 1))
    np.testing.assert_allclose(g[2:40], gam, rtol=1e-12)


def test_weights_exact_rational():
    """alpha = 3/2 in exact rational arithmetic from the product form of eq. (1.2)."""
    a = Fraction(3, 2)
    g = O.grunwald_weights(1.5, 25)
    for k in range(26):
        prod = Fraction(1)
        for j in range(k):
            prod *= (a - j)
        exact = (-1) ** k * prod / math.factorial(k)
        assert abs(g[k] - float(exact)) <= 4e-16 * max(1.0, abs(float(exact)))


@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.9])
def test_weights_proposition_2_1(alpha):
    """Proposition 2.1: g0=1, g1=-alpha, g2>g3>...>0, partial sums negative, total sum 0."""
    n = 4000
    g = O.grunwald_weights(alpha, n)
    assert g[0] == 1.0 and g[1] == -alpha
    assert np.all(g[2:] > 0) and np.all(np.diff(g[2:]) < 0)
    ps = np.cumsum(g)
    assert np.all(ps[1:] < 0)
    # partial sums have the closed form (-1)^n C(alpha-1, n)  (reading of the garbled second sum)
    nn = np.arange(1, 200)
    np.testing.assert_allclose(ps[1:200], (-1.0) ** nn * scipy.special.binom(alpha - 1, nn), rtol=1e-11, atol=1e-15)
    # sum_k g_k = (1-1)^alpha = 0 in the limit, tail O(n^{1-alpha})
    assert abs(ps[-1]) < 5 * n ** (1 - alpha)
    # sum_k |g_k| -> 2 alpha (proof of the Wiener-class theorem)
    assert abs(np.abs(g).sum() - 2 * alpha) < 5 * n ** (1 - alpha)


def _rand_coeffs(m, seed=0, const=False):
    rng = np.random.default_rng(seed)
    if const:
        return np.full(m, 0.6), np.full(m, 0.5)
    return rng.uniform(0.0, 2.0, m), rng.uniform(0.0, 2.0, m)


@pytest.mark.parametrize("m", [1, 2, 3, 7, 20])
def test_two_assemblies_agree(m):
    """eq. (1.4)-(1.5) and the entry formula p_ij of eq. (1.10t) describe the same matrix."""
    dp, dm = _rand_coeffs(m, m)
    dx = 2.0 / (m + 1)
    J1 = O.space_matrix(1.6, dp, dm, dx)
    J2 = O.space_matrix_entries(1.6, dp, dm, dx)
    np.testing.assert_allclose(J1, J2, rtol=1e-14, atol=1e-14 * np.abs(J1).max())


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_gershgorin_proposition_2_2(alpha):
    """Proof of Prop 2.2: strict row dominance, Gershgorin discs in C^-; Remark 2.1:
    Re lambda < 0 and |lambda| <= 2 max |gamma_i|.  The proof states p_ij <= 0 off the
    diagonal; since g_0 = 1 > 0 and g_k > 0 for k >= 2 the off-diagonal entries are in fact
    >= 0 (a sign slip that does not affect the Gershgorin bound, which uses |p_ij|)."""
    m = 40
    dp, dm = _rand_coeffs(m, 3)
    J = O.space_matrix(alpha, dp, dm, 2.0 / (m + 1))
    off = J - np.diag(np.diag(J))
    assert np.all(off >= 0)
    gamma = np.diag(J)
    assert np.all(gamma < 0)
    R = np.abs(off).sum(axis=1)
    assert np.all(R < -gamma)
    lam = np.linalg.eigvals(J)
    assert np.all(lam.real < 0)
    assert np.all(np.abs(lam) <= 2 * np.abs(gamma).max() * (1 + 1e-12))


def test_constant_coefficients_toeplitz_and_wiener():
    """eq. (eqgu): constant d+- gives a Toeplitz J; the Wiener-class sum is 2 alpha (d+ + d-)/dx^alpha."""
    alpha, m = 1.5, 3000
    dp, dm = _rand_coeffs(m, const=True)
    dx = 2.0 / (m + 1)
    J = O.space_matrix(alpha, dp, dm, dx)
    assert np.allclose(J[1:, 1:], J[:-1, :-1], rtol=0, atol=1e-12 * np.abs(J).max())
    t = np.concatenate([J[::-1, 0], J[0, 1:]])        # diagonals t_{-(m-1)}..t_{m-1}
    wiener = 2 * alpha * (0.6 + 0.5) / dx ** alpha
    assert abs(np.abs(t).sum() / wiener - 1) < 5 * m ** (1 - alpha)


@pytest.mark.parametrize("alpha", [1.3, 1.5, 1.8])
def test_J_approximates_fractional_operator(alpha):
    """J applied to x^2(2-x)^2 approaches d+ D+^a u + d- D-^a u (Riemann-Liouville power rule,
    independent of the weights) at first order in dx (shifted Grunwald).  This pins the
    orientation of G versus G^T and the dx^{-alpha} scaling."""
    errs = []
    for m in (63, 127, 255, 511):
        x = W.grid_x(m)
        G3 = math.gamma(3 - alpha)
        dp, dm = G3 * x ** alpha, G3 * (2 - x) ** alpha
        u = x ** 2 * (2 - x) ** 2
        J = O.space_matrix(alpha, dp, dm, 2.0 / (m + 1))
        # at t = 0: u_t = -u, so d+D+u + d-D-u = u_t - f = -u - f
        exact = -u - W.manufactured_source(alpha, x, np.array([0.0]))[0]
        errs.append(np.abs(J @ u - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 0.85) and np.all(rates < 1.3), rates


def test_weights_golden_fixture():
    """Hand-worked exact weights for alpha = 3/2 (eq. (1.2); g_0, g_1 as printed in Prop 2.1)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "grunwald_weights_alpha_3_2.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    g = O.grunwald_weights(1.5, len(rows) - 1)
    for k, num, den in rows:
        assert abs(g[int(k)] - float(Fraction(int(num), int(den)))) <= 4e-16
