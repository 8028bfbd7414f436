"""Pins of the oracle's BVM part (Section 2.2, Definition 3.1) against exact order
conditions, the A_{nu,mu-nu}-stability root count and a scalar ODE with closed form."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _order(alpha, beta, offsets, pmax=6):
    """Largest p with sum_j alpha_j r_j^q = q sum_j beta_j r_j^{q-1} for q = 0..p (exact)."""
    a = [Fraction(x).limit_denominator(1000) for x in alpha]
    b = [Fraction(x).limit_denominator(1000) for x in beta]
    p = -1
    for q in range(pmax + 1):
        lhs = sum(aj * Fraction(r) ** q for aj, r in zip(a, offsets))
        rhs = q * sum(bj * (Fraction(r) ** (q - 1) if q > 0 else 0) for bj, r in zip(b, offsets))
        if lhs != rhs:
            break
        p = q
    return p


def _derive(offsets, deriv_index):
    """The unique 4-point formula of order 3 with beta = e_{deriv_index}, alpha normalised
    by the q=1 condition sum alpha_j r_j = 1 (solved exactly)."""
    n = len(offsets)
    rows = [[Fraction(r) ** q for r in offsets] for q in range(n)]
    rhs = [Fraction(0)] + [q * Fraction(offsets[deriv_index]) ** (q - 1) for q in range(1, n)]
    # Gauss-Jordan in exact arithmetic
    Mx = [row + [v] for row, v in zip(rows, rhs)]
    for c in range(n):
        piv = next(r for r in range(c, n) if Mx[r][c] != 0)
        Mx[c], Mx[piv] = Mx[piv], Mx[c]
        Mx[c] = [v / Mx[c][c] for v in Mx[c]]
        for r in range(n):
            if r != c and Mx[r][c] != 0:
                f = Mx[r][c]
                Mx[r] = [vr - f * vc for vr, vc in zip(Mx[r], Mx[c])]
    return [float(Mx[r][n]) for r in range(n)]


def test_trapezoidal_coefficients_and_order():
    F = O.trapezoidal()
    assert (F.nu, F.mu) == (1, 1)
    assert _order(F.alpha, F.beta, [-1, 0]) == 2


def test_gbdf3_coefficients_from_order_conditions():
    """Each GBDF3 formula equals the one derived here from the order conditions."""
    F = O.gbdf3()
    assert (F.nu, F.mu) == (2, 3)
    np.testing.assert_allclose(F.alpha, _derive([-2, -1, 0, 1], 2), rtol=0, atol=1e-15)
    np.testing.assert_allclose(F.alpha_init[0], _derive([-1, 0, 1, 2], 1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(F.alpha_fin[0], _derive([-3, -2, -1, 0], 3), rtol=0, atol=1e-15)
    assert _order(F.alpha, F.beta, [-2, -1, 0, 1]) == 3
    assert _order(F.alpha_init[0], F.beta_init[0], [-1, 0, 1, 2]) == 3
    assert _order(F.alpha_fin[0], F.beta_fin[0], [-3, -2, -1, 0]) == 3


@pytest.mark.parametrize("kind", ["trapezoidal", "gbdf3"])
def test_consistency(kind):
    """Consistency rho(1) = 0, rho'(1) = sigma(1) (Section 3.1, eq. (1.12))."""
    F = O.formula(kind)
    z = np.arange(F.mu + 1)
    assert abs(F.alpha.sum()) < 1e-15
    assert abs((F.alpha * z).sum() - F.beta.sum()) < 1e-15


@pytest.mark.parametrize("kind", ["trapezoidal", "gbdf3"])
def test_A_stability_root_count(kind):
    """Definition 3.1: for q in C^-, rho(z) - q sigma(z) has nu zeros inside |z| = 1
    and mu - nu outside."""
    F = O.formula(kind)
    rng = np.random.default_rng(7)
    qs = -rng.exponential(3.0, 4000) + 1j * rng.normal(0, 5.0, 4000)
    qs = np.concatenate([qs, [-1e-3, -1e3, -1 + 40j, -1e-6 + 1j]])
    for q in qs:
        # rho(z) = sum_i alpha_i z^i (the z^nu factor absorbs the negative powers)
        c = (F.alpha - q * F.beta)[::-1]
        r = np.roots(c)
        inside = int(np.sum(np.abs(r) < 1))
        assert inside == F.nu and len(r) - inside == F.mu - F.nu


@pytest.mark.parametrize("kind,order", [("trapezoidal", 2), ("gbdf3", 3)])
def test_scalar_ode_temporal_order(kind, order):
    """m = 1 case of eq. (1.10): y' = lam y + f(t), exact y = e^{-t} cos 3t + t^2.  The global
    error must fall at the formula's order; this pins the rows of A, B, the initial and final
    formulas and every term of the right-hand side (u0 and f_0 included)."""
    lam = -2.0
    yex = lambda t: np.exp(-t) * np.cos(3 * t) + t ** 2
    dy = lambda t: -np.exp(-t) * np.cos(3 * t) - 3 * np.exp(-t) * np.sin(3 * t) + 2 * t
    F = O.formula(kind)
    errs = []
    for s in (32, 64, 128, 256):
        t = np.linspace(0.0, 1.0, s + 1)
        f = (dy(t) - lam * yex(t))[:, None]
        M, b = O.all_at_once(np.array([[lam]]), F, s, 1.0 / s, f, np.array([yex(0.0)]))
        y = np.linalg.solve(M, b)
        errs.append(np.abs(y - yex(t[1:])).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.25), rates


def test_s_form_gbdf3_structure():
    """For GBDF3, B = I_s (beta only on the derivative node), b0 = 0, a0 = (-1/3, 1/6, 0, ...)."""
    A, B, a0, b0, _ = O.s_form(O.gbdf3(), 10)
    np.testing.assert_array_equal(B, np.eye(10))
    np.testing.assert_array_equal(b0, 0)
    np.testing.assert_allclose(a0[:3], [-1 / 3, 1 / 6, 0], atol=1e-16)
    A, B, a0, b0, _ = O.s_form(O.trapezoidal(), 6)
    np.testing.assert_array_equal(A, np.eye(6) - np.eye(6, k=-1))
    np.testing.assert_array_equal(B, 0.5 * (np.eye(6) + np.eye(6, k=-1)))
    np.testing.assert_array_equal(a0, [-1, 0, 0, 0, 0, 0])
    np.testing.assert_array_equal(b0, [0.5, 0, 0, 0, 0, 0])
