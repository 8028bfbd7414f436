"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle, step by step and
end to end.  Sizes span several 64-wide tiles with ragged tails; the full-size cases
use the workloads' seeded generators."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1305_6653_amd import BvmSolver, FdeError, factor_batch, solve_batch
from paper_1305_6653_amd import _native as N

pytestmark = pytest.mark.gpu

CASES = {
    "trap_m1_s2": lambda: W.tiny(1, 2, 1.5, 1, "trapezoidal"),
    "gbdf3_m1_s4": lambda: W.tiny(1, 4, 1.3, 2, "gbdf3"),
    "gbdf3_m7_s8": lambda: W.tiny(7, 8, 1.9, 3, "gbdf3"),
    "trap_m63_s64_manufactured": W.manufactured_c1,
    "gbdf3_m200_s32": lambda: W.tiny(200, 32, 1.7, 4, "gbdf3"),
    "trap_m130_s16": lambda: W.tiny(130, 16, 1.2, 5, "trapezoidal"),
    "gbdf3_m255_s128_random": lambda: W.warmstart_instance(7),
}
SMALL = ["trap_m1_s2", "gbdf3_m1_s4", "gbdf3_m7_s8", "trap_m63_s64_manufactured",
         "gbdf3_m200_s32", "trap_m130_s16"]


def _setup(name):
    p = CASES[name]()
    return p, BvmSolver(p)


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _elem(a, b):
    """max_i |a_i - b_i| / max_i |b_i|: the worst single entry, relative to the solution's scale."""
    a = np.asarray(a)
    b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", SMALL)
def test_toeplitz_matvec_vs_dense(name):
    p, S = _setup(name)
    J, _, _, _ = O.problem_matrices(p)
    x = np.random.default_rng(1).standard_normal((min(3, p.s), p.m))
    y = S.toeplitz(x)
    ref = x @ J.T
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(J).max() * np.abs(x).sum(axis=1).max()


@pytest.mark.parametrize("name", SMALL)
def test_time_rfft_vs_dft(name):
    p, S = _setup(name)
    V = np.random.default_rng(2).standard_normal((p.s, p.m))
    Vh = S.time_rfft(V)
    # plain DFT definition, e^{-2 pi i n k / s}
    n = np.arange(p.s)
    k = np.arange(p.s // 2 + 1)
    ref = np.exp(-2j * np.pi * np.outer(k, n) / p.s) @ V
    assert np.abs(Vh - ref).max() <= 1e-13 * np.abs(V).sum(axis=0).max()


@pytest.mark.parametrize("name", SMALL)
def test_rhs_and_matvec_vs_oracle(name):
    p, S = _setup(name)
    J, F, tau, _ = O.problem_matrices(p)
    A, B, a0, b0, Bfull = O.s_form(F, p.s)
    b_ref = tau * (Bfull @ p.f) - np.outer(a0, p.u0) + tau * np.outer(b0, J @ p.u0)
    b = S.rhs(p.u0, p.f)
    assert _rel(b, b_ref) <= 1e-13
    Z = np.random.default_rng(3).standard_normal((p.s, p.m))
    w = S.matvec(Z)
    assert _rel(w, O.apply_M(J, A, B, tau, Z)) <= 1e-13


@pytest.mark.parametrize("name", ["gbdf3_m7_s8", "trap_m130_s16", "gbdf3_m200_s32"])
def test_strang_forward_and_lowrank_correction(name):
    """S z (eq. (1.11) applied forward) and (S - M) z, whose support is the nu + (mu - nu)
    boundary block rows of Theorem 3.3."""
    p, S = _setup(name)
    J, F, tau, _ = O.problem_matrices(p)
    Sd = O.strang_dense(J, F, p.s, tau)
    M, _ = O.problem_system(p)
    z = np.random.default_rng(6).standard_normal((p.s, p.m))
    assert _rel(S.strang_apply(z).reshape(-1), Sd @ z.reshape(-1)) <= 1e-13
    c = S.lowrank_correction(z)
    assert _rel(c.reshape(-1), (Sd - M) @ z.reshape(-1)) <= 1e-13
    rows = sorted(set(range(F.nu)) | set(range(p.s - (F.mu - F.nu), p.s)))
    mask = np.ones(p.s, bool)
    mask[rows] = False
    assert np.all(c[mask] == 0.0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 2e-6)])
@pytest.mark.parametrize("name", ["gbdf3_m7_s8", "trap_m63_s64_manufactured", "gbdf3_m200_s32",
                                  "trap_m130_s16"])
def test_block_lu_factors(name, prec, tol):
    """||L U - K_k|| / ||K_k|| for the pivot-free MFMA factorization."""
    p, S = _setup(name)
    S.factor(prec)
    J, F, tau, _ = O.problem_matrices(p)
    P = O.StrangPreconditioner(J, F, p.s, tau)
    nb = p.s // 2 + 1
    for k in sorted({0, 1, nb // 2, nb - 1}):
        Fk = S.factor_block(k)
        L = np.tril(Fk, -1) + np.eye(p.m)
        U = np.triu(Fk)
        K = P.block(k, J, tau)
        assert _rel(L @ U, K) <= tol, (k, _rel(L @ U, K))


@pytest.mark.parametrize("prec,eps", [("fp64", 2.0 ** -53), ("mixed", 2.0 ** -24)])
@pytest.mark.parametrize("name", SMALL)
def test_preconditioner_apply(name, prec, eps):
    """Forward error of S^{-1} v within 30 * eps * max_k cond(K_k) (backward-stable solves)."""
    p, S = _setup(name)
    S.factor(prec)
    J, F, tau, _ = O.problem_matrices(p)
    P = O.StrangPreconditioner(J, F, p.s, tau)
    kappa = max(np.linalg.cond(P.block(k, J, tau)) for k in range(p.s // 2 + 1))
    v = np.random.default_rng(4).standard_normal((p.s, p.m))
    assert _rel(S.precond(v), P.apply(v)) <= 30 * eps * max(kappa, 10.0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-8)])
@pytest.mark.parametrize("name", SMALL + ["gbdf3_m255_s128_random"])
def test_solve_vs_oracle(name, prec, tol):
    p, S = _setup(name)
    S.factor(prec)
    u, info = S.solve(p.u0, p.f, rtol=1e-10)
    assert info["converged"] == 1 and info["true_relres"] <= 1e-10
    ref = O.solve_gmres(p, tol=1e-12)   # 1e-13 is below the FP64 floor of some cases
    assert ref.converged
    assert _rel(u, ref.x) <= tol, _rel(u, ref.x)
    assert _elem(u, ref.x) <= tol, _elem(u, ref.x)
    assert O.true_relres(p, u) <= 1.5e-10
    if prec == "fp64":
        ref10 = O.solve_gmres(p, tol=1e-10)
        assert abs(info["iters"] - ref10.iters) <= 1, (info["iters"], ref10.iters)


def test_manufactured_solution_accuracy():
    p, S = _setup("trap_m63_s64_manufactured")
    S.factor("fp64")
    u, info = S.solve(p.u0, p.f)
    Ue = p.exact(W.grid_x(p.m), W.grid_t(p.s)[1:])
    assert 0.005 < _rel(u, Ue) < 0.02


def test_deterministic_and_warm_start():
    p, S = _setup("gbdf3_m200_s32")
    S.factor("fp64")
    u1, i1 = S.solve(p.u0, p.f)
    u2, i2 = S.solve(p.u0, p.f)
    assert np.array_equal(u1, u2) and i1["iters"] == i2["iters"]
    u3, i3 = S.solve(p.u0, p.f, x0=u1)    # the guess is projected (gamma ~ 1), no iteration
    assert i3["iters"] == 0 and _rel(u3, u1) <= 1e-12 and i3["true_relres"] <= 1e-10


def test_initial_guess_gate():
    """FDE_OPT_X0_GATE: a guess whose gamma-scaled residual exceeds the gate (default 1e-2 of
    ||b||) is dropped, and the solve is then the zero-start solve bit for bit; with the gate off
    (0) the same guess is used; a close guess passes the default gate and saves iterations."""
    p, S = _setup("gbdf3_m200_s32")
    S.factor("fp64")
    assert S.get_option(N.FDE_OPT_X0_GATE) == 10000
    u0, i0 = S.solve(p.u0, p.f)
    assert S.get_option(N.FDE_OPT_X0_KEPT) == 0
    xs = np.arange(1, p.m + 1) / (p.m + 1)
    smooth = np.outer(np.ones(p.s), np.sin(np.pi * xs) + 0.3 * np.sin(3 * np.pi * xs))
    rough = u0 + 0.05 * np.linalg.norm(u0) / np.linalg.norm(smooth) * smooth
    u1, i1 = S.solve(p.u0, p.f, x0=rough)
    assert S.get_option(N.FDE_OPT_X0_KEPT) == 0
    assert np.array_equal(u1, u0) and i1["iters"] == i0["iters"]
    S.set_option(N.FDE_OPT_X0_GATE, 0)
    u2, i2 = S.solve(p.u0, p.f, x0=rough)
    assert S.get_option(N.FDE_OPT_X0_KEPT) == 1 and i2["true_relres"] <= 1e-10
    assert _rel(u2, u0) <= 1e-9
    S.set_option(N.FDE_OPT_X0_GATE, 10000)
    close = u0 + 1e-9 * np.linalg.norm(u0) / np.linalg.norm(smooth) * smooth
    u3, i3 = S.solve(p.u0, p.f, x0=close)
    assert S.get_option(N.FDE_OPT_X0_KEPT) == 1 and i3["iters"] < i0["iters"]
    assert i3["true_relres"] <= 1e-10 and _rel(u3, u0) <= 1e-9
    with pytest.raises(FdeError):
        S.set_option(N.FDE_OPT_X0_GATE, -1)


def test_lowrank_start_with_exact_correction_needs_no_iteration():
    """x0_kind = LOWRANK: with the exact c = (S - M) u the start S^{-1}(b + c) is u itself."""
    p, S = _setup("gbdf3_m200_s32")
    S.factor("fp64")
    u, _ = S.solve(p.u0, p.f, rtol=1e-12)
    c = S.lowrank_correction(u)
    u2, info = S.solve(p.u0, p.f, x0=c, x0_kind=N.FDE_X0_LOWRANK)
    assert info["iters"] == 0 and _rel(u2, u) <= 1e-10


def test_errors_and_noconv():
    p, S = _setup("gbdf3_m7_s8")
    with pytest.raises(FdeError) as e:
        S.solve(p.u0, p.f)
    assert e.value.status == N.FDE_EINVAL
    S.factor("fp64")
    u, info = S.solve(p.u0, p.f, maxit=1, rtol=1e-14, raise_on_noconv=False)
    assert info["converged"] == 0 and info["iters"] == 1
    with pytest.raises(FdeError) as e:
        S.solve(p.u0, p.f, maxit=1, rtol=1e-14)
    assert e.value.status == N.FDE_ENOCONV


def test_device_pointers_match_host():
    import torch
    p, S = _setup("gbdf3_m200_s32")
    S.factor("fp64")
    uh, _ = S.solve(p.u0, p.f)
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(p.u0).to(dev)
    f = torch.from_numpy(np.ascontiguousarray(p.f)).to(dev)
    ud, info = S.solve(u0, f)
    torch.cuda.synchronize()
    assert np.array_equal(ud.cpu().numpy(), uh)


def test_device_inputs_produced_just_before_the_call():
    """Device inputs written by torch work still queued on torch's current stream (a long
    product first, then the copies that fill f and u0) are read only after that work: the
    binding orders the library's stream after torch's producers."""
    import torch
    p, S = _setup("gbdf3_m200_s32")
    S.factor("fp64")
    uh, _ = S.solve(p.u0, p.f)
    dev = torch.device("cuda:0")
    a = torch.randn(4096, 4096, device=dev)
    f = torch.zeros((p.s + 1, p.m), dtype=torch.float64, device=dev)
    u0 = torch.zeros(p.m, dtype=torch.float64, device=dev)
    fh = torch.from_numpy(np.ascontiguousarray(p.f)).pin_memory()
    u0h = torch.from_numpy(np.ascontiguousarray(p.u0)).pin_memory()
    torch.cuda.synchronize()
    for _ in range(8):
        a = a @ a / 64.0          # queued ahead of the copies
    f.copy_(fh, non_blocking=True)
    u0.copy_(u0h, non_blocking=True)
    ud, info = S.solve(u0, f)
    torch.cuda.synchronize()
    assert np.array_equal(ud.cpu().numpy(), uh)
    w = S.matvec(ud)
    torch.cuda.synchronize()
    assert np.array_equal(w.cpu().numpy(), S.matvec(uh))


def test_device_array_inputs_match_host():
    """Device buffers from the library's own allocator (no torch) give the host result."""
    from paper_1305_6653_amd.devmem import DeviceArray
    p, S = _setup("trap_m130_s16")
    S.factor("fp64")
    uh, _ = S.solve(p.u0, p.f)
    u0, f = DeviceArray.from_numpy(p.u0), DeviceArray.from_numpy(p.f)
    ud, _ = S.solve(u0, f)
    assert isinstance(ud, DeviceArray) and np.array_equal(ud.numpy(), uh)
    for a in (u0, f, ud):
        a.free()


@pytest.mark.parametrize("where", ["f", "u0"])
def test_non_finite_input_is_rejected(where):
    """A NaN in f or u0 makes the right-hand side non-finite: FDE_EINVAL, nothing solved."""
    p, S = _setup("gbdf3_m7_s8")
    S.factor("fp64")
    f, u0 = p.f.copy(), p.u0.copy()
    if where == "f":
        f[1, 3] = np.nan
    else:
        u0[3] = np.nan
    with pytest.raises(FdeError) as e:
        S.solve(u0, f)
    assert e.value.status == N.FDE_EINVAL
    # the handle is still good: a finite right-hand side solves as on a fresh handle
    u, info = S.solve(p.u0, p.f)
    S2 = BvmSolver(p)
    S2.factor("fp64")
    u2, info2 = S2.solve(p.u0, p.f)
    assert info["converged"] == 1 and np.array_equal(u, u2) and info["iters"] == info2["iters"]
    S2.close()


def test_non_finite_instance_in_a_batch_is_rejected():
    """One instance of a batch with a NaN in f: the batch call returns FDE_EINVAL; the other
    instances then solve as before."""
    ps = [CASES["gbdf3_m7_s8"](), CASES["gbdf3_m200_s32"]()]
    Ss = [BvmSolver(q) for q in ps]
    factor_batch(Ss, "fp64")
    f_bad = ps[1].f.copy()
    f_bad[2, 5] = np.nan
    with pytest.raises(FdeError) as e:
        solve_batch(Ss, [q.u0 for q in ps], [ps[0].f, f_bad])
    assert e.value.status == N.FDE_EINVAL
    outs, infos = solve_batch(Ss, [q.u0 for q in ps], [q.f for q in ps])
    for q, u, info in zip(ps, outs, infos):
        assert info["converged"] == 1 and O.true_relres(q, u) <= 1.5e-10
    for S in Ss:
        S.close()


def test_custom_formula_equals_the_built_in_one():
    """FDE_BVM_CUSTOM carrying the third-order GBDF's coefficients (eq. (1.7)-(1.9)) gives the
    built-in GBDF3 solve bit for bit: same tables, same kernels."""
    p = CASES["gbdf3_m200_s32"]()
    S1, S2 = BvmSolver(p), BvmSolver(p, formula=O.gbdf3())
    for prec in ("fp64", "mixed"):
        S1.factor(prec)
        S2.factor(prec)
        u1, i1 = S1.solve(p.u0, p.f)
        u2, i2 = S2.solve(p.u0, p.f)
        assert np.array_equal(u1, u2) and i1["iters"] == i2["iters"], prec
    S1.close()
    S2.close()


def test_zero_pivot_returns_esingular():
    """A consistent custom formula with sigma = 0 and a double root of rho at 1
    (u_{n+1} - 2 u_n + u_{n-1} = 0) makes the zero-frequency block K_0 = rho(1) I = 0: the
    factorization reports FDE_ESINGULAR and leaves the handle unfactored."""
    import types
    p = W.tiny(20, 8, 1.5, 9, "gbdf3")
    F = types.SimpleNamespace(nu=1, mu=2, alpha=[1.0, -2.0, 1.0], beta=[0.0, 0.0, 0.0],
                              alpha_init=[], beta_init=[], alpha_fin=[1.0, -2.0, 1.0],
                              beta_fin=[0.0, 0.0, 0.0])
    S = BvmSolver(p, formula=F)
    with pytest.raises(FdeError) as e:
        S.factor("fp64")
    assert e.value.status == N.FDE_ESINGULAR
    with pytest.raises(FdeError) as e:
        S.solve(p.u0, p.f)
    assert e.value.status == N.FDE_EINVAL
    S.close()


def test_batch_equals_single():
    from paper_1305_6653_amd import solve_batch
    names = ["gbdf3_m7_s8", "trap_m130_s16", "gbdf3_m200_s32"]
    ps, Ss = zip(*[_setup(n) for n in names])
    for S in Ss:
        S.factor("fp64")
    singles = [S.solve(p.u0, p.f)[0] for p, S in zip(ps, Ss)]
    outs, infos = solve_batch(list(Ss), [p.u0 for p in ps], [p.f for p in ps])
    for a, b, i in zip(outs, singles, infos):
        assert i["converged"] == 1
        assert _rel(a, b) <= 1e-12


def test_options_validate_and_read_back():
    p, S = _setup("gbdf3_m7_s8")
    defaults = {N.FDE_OPT_GRAPHS: 1, N.FDE_OPT_AUTOTUNE: 1, N.FDE_OPT_TRSV_W: 0,
                N.FDE_OPT_PRECOND: N.FDE_PC_STRANG, N.FDE_OPT_SIDE: N.FDE_SIDE_RIGHT,
                N.FDE_OPT_BLOCKS: N.FDE_BLOCKS_AUTO, N.FDE_OPT_ORTHO: N.FDE_ORTHO_MGS}
    for opt, v in defaults.items():
        assert S.get_option(opt) == v, opt
    for opt, bad in [(N.FDE_OPT_PRECOND, 7), (N.FDE_OPT_SIDE, 2), (N.FDE_OPT_BLOCKS, -1),
                     (N.FDE_OPT_ORTHO, 5), (N.FDE_OPT_TRSV_W, -3), (N.FDE_OPT_TRSV_W_IN_USE, 1),
                     (99, 0)]:
        with pytest.raises(FdeError) as e:
            S.set_option(opt, bad)
        assert e.value.status == N.FDE_EINVAL, opt
    for opt, v in [(N.FDE_OPT_PRECOND, N.FDE_PC_NONE), (N.FDE_OPT_SIDE, N.FDE_SIDE_LEFT),
                   (N.FDE_OPT_BLOCKS, N.FDE_BLOCKS_HESSENBERG), (N.FDE_OPT_ORTHO, N.FDE_ORTHO_CGS2)]:
        S.set_option(opt, v)
        assert S.get_option(opt) == v
    # a changed preconditioner or block solver discards the factorization
    with pytest.raises(FdeError) as e:
        S.solve(p.u0, p.f)
    assert e.value.status == N.FDE_EINVAL
    S.factor("fp64")
    u, info = S.solve(p.u0, p.f, rtol=1e-10, maxit=2000)
    assert info["converged"] == 1


@pytest.mark.parametrize("bvm", ["trapezoidal", "gbdf3"])
def test_largest_step_count(bvm):
    """s = 1024, the largest step count the library takes (the time FFT's LDS buffers and the
    widest frequency range), with a ragged m: solution and true residual against the oracle."""
    p = W.tiny(33, 1024, 1.6, 8, bvm)
    S = BvmSolver(p)
    S.factor("fp64")
    u, info = S.solve(p.u0, p.f, rtol=1e-10)
    assert info["converged"] == 1 and info["true_relres"] <= 1e-10
    ref = O.solve_gmres(p, tol=1e-12, maxit=400)
    assert _rel(u, ref.x) <= 1e-9, _rel(u, ref.x)
    assert O.true_relres(p, u) <= 1.5e-10
    S.close()
