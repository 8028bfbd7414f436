"""What a warm start can and cannot do for the Strang-preconditioned solve, on the oracle.

Theorem 3.3 writes M = S - C with C supported on the nu initial and mu - nu final block rows.
Hence u = S^{-1}(b + C u): knowing c = C u on those rows is knowing u.  These tests pin that
identity and measure how GMRES's iteration count responds to an inexact c or u (the regime a
learned predictor lives in)."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _system(p):
    J, F, tau, _ = O.problem_matrices(p)
    A, B, a0, b0, Bfull = O.s_form(F, p.s)
    b = (tau * (Bfull @ p.f) - np.outer(a0, p.u0) + tau * np.outer(b0, J @ p.u0)).reshape(-1)
    cA, cB = O.strang_columns(F, p.s)
    CA, CB = O.strang_circulant(cA), O.strang_circulant(cB)
    P = O.StrangPreconditioner(J, F, p.s, tau)
    sh = (p.s, p.m)
    Mv = lambda z: O.apply_M(J, A, B, tau, z.reshape(sh)).reshape(-1)
    Sv = lambda z: (CA @ z.reshape(sh) - tau * (CB @ z.reshape(sh)) @ J.T).reshape(-1)
    Pv = lambda v: P.apply(v.reshape(sh)).reshape(-1)
    return F, b, Mv, Sv, Pv


@pytest.fixture(scope="module")
def case():
    p = W.random_instance(11, m=63, s=64, zero_u0=True)
    F, b, Mv, Sv, Pv = _system(p)
    u = O.gmres(Mv, Pv, b, tol=1e-13).x
    zero = O.gmres(Mv, Pv, b, tol=1e-10).iters
    return p, F, b, Mv, Sv, Pv, u, zero


def test_exact_lowrank_correction_gives_the_solution(case):
    p, F, b, Mv, Sv, Pv, u, zero = case
    c = (Sv(u) - Mv(u)).reshape(p.s, p.m)
    rows = list(range(F.nu)) + list(range(p.s - (F.mu - F.nu), p.s))
    interior = np.setdiff1d(np.arange(p.s), rows)
    assert np.abs(c[interior]).max() <= 1e-13 * np.abs(c).max()
    x0 = Pv(b + c.reshape(-1))
    assert np.linalg.norm(x0 - u) <= 1e-11 * np.linalg.norm(u)
    assert O.gmres(Mv, Pv, b, x0=x0, tol=1e-10).iters == 0


def test_iterations_respond_only_logarithmically_to_the_guess(case):
    """A correction with a 1 % error in a random direction leaves r0 ~ 2e-2 ||b|| but saves
    at most two of ~17 iterations; 10 % costs an iteration.  A guess of u itself with 10 %
    error has ||b - M x0|| >> ||b||, which is why the solver projects it (gamma)."""
    p, F, b, Mv, Sv, Pv, u, zero = case
    rng = np.random.default_rng(0)
    c = (Sv(u) - Mv(u)).reshape(p.s, p.m)
    rows = list(range(F.nu)) + list(range(p.s - (F.mu - F.nu), p.s))
    res = {}
    for lvl in (1e-1, 1e-2):
        E = np.zeros_like(c)
        for r in rows:
            e = rng.standard_normal(p.m)
            E[r] = e / np.linalg.norm(e) * lvl * np.linalg.norm(c[r])
        res[lvl] = O.gmres(Mv, Pv, b, x0=Pv(b + (c + E).reshape(-1)), tol=1e-10).iters
    assert 15 <= zero <= 19
    assert zero - 2 <= res[1e-2] <= zero
    assert res[1e-1] >= zero - 1
    U = u + 0.1 * np.linalg.norm(u) * (lambda e: e / np.linalg.norm(e))(rng.standard_normal(u.size))
    assert np.linalg.norm(b - Mv(U)) > 10 * np.linalg.norm(b)
