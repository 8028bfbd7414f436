"""The spectra of Fig. 1 (Section 4): M and the preconditioned matrices S^{-1} M, (S2)^{-1} M and
(S2~)^{-1} M for the example of Section 4 with n = 48, s = 64 (alpha = 1.5; the caption does not
say which of the example's two alphas).  Every matrix is formed column by column through the
library (fde_apply_matvec, then fde_apply_precond with each preconditioner factored), compared
entry by entry with the oracle's dense matrices (the parity check: eigenvalues of these far
from normal matrices move by much more than the entries' rounding, so they are not compared),
and S^{-1} M against the theorem of Section 3.3: rank(S^{-1} M - I) <= 2 m mu, by singular
values, the same for both.  With FDE_FIG1_OUT set, a summary of the four spectra (LAPACK
eigenvalues of the library-formed matrices: extremes, cluster counts, a 24 x 24 histogram over
each bounding box and the eigenvalues away from 1) is written to that path."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1305_6653_amd import BvmSolver

pytestmark = pytest.mark.gpu

FORMS = (("M", None), ("S^-1 M", "strang"), ("(S2)^-1 M", "bccb"), ("(S2~)^-1 M", "bccb_shifted"))


def _columns(S, p, pc):
    n = p.s * p.m
    A = np.empty((n, n))
    e = np.zeros((p.s, p.m))
    for i in range(n):
        e.flat[i] = 1.0
        w = S.matvec(e)
        A[:, i] = (S.precond(w) if pc else w).reshape(-1)
        e.flat[i] = 0.0
    return A


def _oracle(p, pc):
    M, _ = O.problem_system(p)
    if pc is None:
        return M
    J, F, tau, _ = O.problem_matrices(p)
    P = O.strang_dense(J, F, p.s, tau) if pc == "strang" else O.bccb_dense(p, pc == "bccb_shifted")
    return np.linalg.solve(P, M)


def _summary(name, ev, bins=24):
    lines = [f"== {name}: {ev.size} eigenvalues",
             f"Re in [{ev.real.min():.6g}, {ev.real.max():.6g}], Im in [{ev.imag.min():.6g}, {ev.imag.max():.6g}], "
             f"|lambda| in [{np.abs(ev).min():.6g}, {np.abs(ev).max():.6g}]"]
    for r in (1e-1, 1e-2, 1e-6):
        lines.append(f"|lambda - 1| < {r:g}: {int(np.sum(np.abs(ev - 1) < r))}")
    h, xe, ye = np.histogram2d(ev.real, ev.imag, bins=bins)
    lines.append(f"histogram {bins} x {bins}: Re edges {xe[0]:.6g} .. {xe[-1]:.6g}, Im edges {ye[0]:.6g} .. {ye[-1]:.6g}"
                 " (rows: Re bins, columns: Im bins)")
    lines += [" ".join(f"{int(c)}" for c in row) for row in h]
    away = ev[np.abs(ev - 1) >= 1e-2]
    if name != "M" and away.size <= 400:
        away = away[np.lexsort((away.imag, away.real))]
        lines.append(f"eigenvalues with |lambda - 1| >= 1e-2 ({away.size}):")
        lines += [f"{z.real:.8g} {z.imag:+.8g}" for z in away]
    return lines


@pytest.mark.timeout(900)
def test_fig1_spectra():
    p = W.example41(1.5, 48, 64)
    mu = 4  # GAM5
    out = []
    S = BvmSolver(p)
    for name, pc in FORMS:
        if pc:
            S.factor("fp64", pc)
        A = _columns(S, p, pc)
        R = _oracle(p, pc)
        err = np.abs(A - R).max() / np.abs(R).max()
        assert err <= 1e-10, (name, err)
        if pc == "strang":
            # theorem of Section 3.3: rank(S^{-1} M - I) <= 2 m mu (singular values, which are
            # well conditioned, unlike the eigenvalues of these far-from-normal matrices)
            ranks = []
            for X in (A, R):
                sv = np.linalg.svd(X - np.eye(X.shape[0]), compute_uv=False)
                ranks.append(int(np.sum(sv > 1e-10 * sv[0])))
            assert ranks[0] == ranks[1] <= 2 * p.m * mu, ranks
        print(f"{name}: entries within {err:.1e} of the oracle's", flush=True)
        out += _summary(name, np.linalg.eigvals(A))
    S.close()
    path = os.environ.get("FDE_FIG1_OUT")
    if path:
        with open(path, "w") as fh:
            fh.write("Fig. 1 (Section 4): spectra for the example of Section 4, alpha = 1.5, n = 48, s = 64, "
                     "fifth-order GAM; matrices formed through the library's matrix-vector product and "
                     "preconditioner applies (FP64), eigenvalues by LAPACK\n")
            fh.write("command: FDE_FIG1_OUT=profiles/fig1_spectra_n48_s64.txt python -m pytest "
                     "tests/test_gpu_spectra.py -m gpu\n")
            fh.write("\n".join(out) + "\n")
