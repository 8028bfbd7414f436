"""Seeded synthetic inputs for the two-sided space-fractional diffusion problem.

This module only *samples* problem data (alpha, d+(x), d-(x), f(x,t), u0(x)) on the
uniform grid of the problem statement (Section 2, eq. (1.1) and the grid definition
x_i = x_L + i*dx, dx = (x_R - x_L)/(m+1); t_n = t_0 + n*tau, tau = (T - t_0)/s).  It holds
none of the method's arithmetic (no Grunwald weights, no BVM, no preconditioner), so
both the CPU oracle and the GPU path may use it.

All random draws use numpy.random.default_rng(seed) (PCG64) in a fixed, documented order.

Workloads (all on x in (0, 2), t in [0, 1], homogeneous Dirichlet boundary):

* ``manufactured_c1``   alpha=1.5, m=63, s=64, trapezoidal, d+ = Gamma(3-a) x^a,
  d- = Gamma(3-a)(2-x)^a, exact u = e^{-t} x^2 (2-x)^2 with its analytic source.
* ``smooth_random``     alpha=1.8, m=1023, s=512, GBDF3, seed 2 (and, with alpha=1.3,
  m=4095, s=256, seed 3): d+- = 1 + 0.5 sin(pi x/2) + U(-0.1, 0.1) per node,
  f = sum_{p<=8, q<=4} a_pq sin(p pi x/2) cos(q pi t), a_pq ~ N(0,1)/(p^2 (1+q^2)),
  u0 = sum_{p<=8} c_p sin(p pi x/2), c_p ~ N(0,1)/p^2.
* ``batch_instance``    seed 4000+i: m from {127,...,2047}, s from {64,...,512},
  alpha ~ U(1.1, 1.9), d+- = 1 + 0.5 tanh(sum_{p<=6} e_p sin(p pi x/2)/p), f and u0 as
  above, GBDF3.
* ``warmstart_instance`` m=255, s=128, GBDF3, the batch generators for alpha/d+-/f, u0=0.
* ``example41``         the analytic example of Section 4 (no random draws): f = 0,
  d+ = 0.6, d- = 0.5, u(x,0) a Gaussian pulse centred at 1.2 of width 0.08, fifth-order
  GAM; alpha in {1.2, 1.5}, m in {24, 48, 96}, s in {16, 32, 64, 128} in its tables.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

TRAPEZOIDAL = "trapezoidal"
GBDF3 = "gbdf3"
GAM5 = "gam5"


@dataclasses.dataclass
class Problem:
    """Discrete data of one instance of eq. (1.1), sampled on the grid.

    d_plus, d_minus: [m] at interior nodes x_1..x_m.
    f: [s+1][m] at (t_n, x_i), n = 0..s (time-major).
    u0: [m] initial values at interior nodes.
    """
    alpha: float
    m: int
    s: int
    d_plus: np.ndarray
    d_minus: np.ndarray
    f: np.ndarray
    u0: np.ndarray
    bvm: str = GBDF3
    xL: float = 0.0
    xR: float = 2.0
    t0: float = 0.0
    T: float = 1.0
    name: str = ""
    exact: Optional[Callable[[np.ndarray, np.ndarray], np.ndarray]] = None

    @property
    def n_unknowns(self) -> int:
        return self.m * self.s


def grid_x(m: int, xL: float = 0.0, xR: float = 2.0) -> np.ndarray:
    """Interior nodes x_1..x_m of the uniform spatial partition."""
    dx = (xR - xL) / (m + 1)
    return xL + dx * np.arange(1, m + 1, dtype=np.float64)


def grid_t(s: int, t0: float = 0.0, T: float = 1.0) -> np.ndarray:
    """Time levels t_0..t_s of the uniform temporal mesh."""
    tau = (T - t0) / s
    return t0 + tau * np.arange(0, s + 1, dtype=np.float64)


# --------------------------------------------------------------------------------------
# Manufactured workload: exact solution u = e^{-t} x^2 (2-x)^2 on (0,2).
# --------------------------------------------------------------------------------------
def manufactured_exact(x: np.ndarray, t: np.ndarray) -> np.ndarray:
    """u(x,t) = e^{-t} x^2 (2-x)^2, returned as [len(t)][len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return np.exp(-t)[:, None] * (x ** 2 * (2.0 - x) ** 2)[None, :]


def manufactured_source(alpha: float, x: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Analytic source for u = e^{-t} x^2 y^2 (y = 2-x) with d+ = G x^a, d- = G y^a,
    G = Gamma(3-a).  Riemann-Liouville power rule D^a x^p = Gamma(p+1)/Gamma(p+1-a) x^{p-a}
    applied to 4x^2 - 4x^3 + x^4 (and the mirror image in y) gives

      f = -e^{-t} [ x^2 y^2 + 8(x^2+y^2) - 24(x^3+y^3)/(3-a) + 24(x^4+y^4)/((3-a)(4-a)) ].
    """
    a = float(alpha)
    x = np.asarray(x, dtype=np.float64)
    y = 2.0 - x
    spatial = (x ** 2 * y ** 2 + 8.0 * (x ** 2 + y ** 2)
               - 24.0 * (x ** 3 + y ** 3) / (3.0 - a)
               + 24.0 * (x ** 4 + y ** 4) / ((3.0 - a) * (4.0 - a)))
    return -np.exp(-np.asarray(t, dtype=np.float64))[:, None] * spatial[None, :]


def manufactured(m: int = 63, s: int = 64, alpha: float = 1.5, bvm: str = TRAPEZOIDAL) -> Problem:
    x = grid_x(m)
    t = grid_t(s)
    G = math.gamma(3.0 - alpha)
    return Problem(alpha=alpha, m=m, s=s,
                   d_plus=G * x ** alpha, d_minus=G * (2.0 - x) ** alpha,
                   f=manufactured_source(alpha, x, t),
                   u0=manufactured_exact(x, np.array([0.0]))[0],
                   bvm=bvm, name=f"manufactured_m{m}_s{s}",
                   exact=manufactured_exact)


def manufactured_c1() -> Problem:
    """alpha=1.5, m=63, s=64, trapezoidal BVM (4032 unknowns)."""
    p = manufactured(63, 64, 1.5, TRAPEZOIDAL)
    p.name = "c1_manufactured_m63_s64_trap"
    return p


# --------------------------------------------------------------------------------------
# Smooth random workloads
# --------------------------------------------------------------------------------------
def _sine_modes(x: np.ndarray, P: int) -> np.ndarray:
    """[P][m] table of sin(p pi (x - xL)/(xR - xL)) for p = 1..P on x in (0,2)."""
    p = np.arange(1, P + 1, dtype=np.float64)
    return np.sin(np.outer(p, np.pi * x / 2.0))


def _fourier_source(rng: np.random.Generator, x: np.ndarray, t: np.ndarray) -> np.ndarray:
    """f = sum_{p=1..8} sum_{q=0..4} a_pq sin(p pi x/2) cos(q pi t), a_pq ~ N(0,1)/(p^2(1+q^2))."""
    P, Q = 8, 5
    p = np.arange(1, P + 1, dtype=np.float64)[:, None]
    q = np.arange(0, Q, dtype=np.float64)[None, :]
    a = rng.standard_normal((P, Q)) / (p ** 2 * (1.0 + q ** 2))
    sx = _sine_modes(x, P)                                  # [P][m]
    ct = np.cos(np.outer(np.arange(Q, dtype=np.float64), np.pi * t))  # [Q][s+1]
    return ct.T @ (a.T @ sx)                                # [s+1][m]


def _fourier_u0(rng: np.random.Generator, x: np.ndarray) -> np.ndarray:
    P = 8
    c = rng.standard_normal(P) / np.arange(1, P + 1, dtype=np.float64) ** 2
    return c @ _sine_modes(x, P)


def smooth_random(m: int, s: int, alpha: float, seed: int, bvm: str = GBDF3) -> Problem:
    """Draw order: noise(d+)[m], noise(d-)[m], a[8][5], c[8]."""
    rng = np.random.default_rng(seed)
    x = grid_x(m)
    t = grid_t(s)
    base = 1.0 + 0.5 * np.sin(np.pi * x / 2.0)
    d_plus = base + rng.uniform(-0.1, 0.1, m)
    d_minus = base + rng.uniform(-0.1, 0.1, m)
    f = _fourier_source(rng, x, t)
    u0 = _fourier_u0(rng, x)
    return Problem(alpha=alpha, m=m, s=s, d_plus=d_plus, d_minus=d_minus, f=f, u0=u0,
                   bvm=bvm, name=f"smooth_m{m}_s{s}_a{alpha}_seed{seed}")


def smooth_c2() -> Problem:
    """alpha=1.8, m=1023, s=512, GBDF3, seed 2 (523,776 unknowns)."""
    return smooth_random(1023, 512, 1.8, 2)


def smooth_c3() -> Problem:
    """alpha=1.3, m=4095, s=256, GBDF3, seed 3 (1,048,320 unknowns)."""
    return smooth_random(4095, 256, 1.3, 3)


BATCH_M = (127, 255, 511, 1023, 2047)
BATCH_S = (64, 128, 256, 512)


def _tanh_field(rng: np.random.Generator, x: np.ndarray) -> np.ndarray:
    """1 + 0.5 tanh(sum_{p=1..6} e_p sin(p pi x/2)/p), e_p ~ N(0,1); values in (0.5, 1.5)."""
    P = 6
    e = rng.standard_normal(P) / np.arange(1, P + 1, dtype=np.float64)
    return 1.0 + 0.5 * np.tanh(e @ _sine_modes(x, P))


def random_instance(seed: int, m: Optional[int] = None, s: Optional[int] = None,
                    zero_u0: bool = False) -> Problem:
    """Draw order: m index, s index, alpha, e(d+)[6], e(d-)[6], a[8][5], c[8].

    m and s, if given, override the drawn values (the draws still happen so the
    remaining fields do not depend on the override)."""
    rng = np.random.default_rng(seed)
    mi = int(rng.integers(0, len(BATCH_M)))
    si = int(rng.integers(0, len(BATCH_S)))
    m = BATCH_M[mi] if m is None else int(m)
    s = BATCH_S[si] if s is None else int(s)
    alpha = float(rng.uniform(1.1, 1.9))
    x = grid_x(m)
    t = grid_t(s)
    d_plus = _tanh_field(rng, x)
    d_minus = _tanh_field(rng, x)
    f = _fourier_source(rng, x, t)
    u0 = _fourier_u0(rng, x)
    if zero_u0:
        u0 = np.zeros(m)
    return Problem(alpha=alpha, m=m, s=s, d_plus=d_plus, d_minus=d_minus, f=f, u0=u0,
                   bvm=GBDF3, name=f"random_seed{seed}_m{m}_s{s}")


def batch_instance(i: int) -> Problem:
    """Instance i (0 <= i < 64) of the uneven 64-instance batch, seed 4000+i."""
    return random_instance(4000 + i)


def batch_c4(count: int = 64):
    return [batch_instance(i) for i in range(count)]


def warmstart_instance(seed: int) -> Problem:
    """m=255, s=128, GBDF3, u0 = 0; training seeds 0..19999, held-out 1_000_000..1_000_999."""
    p = random_instance(seed, m=255, s=128, zero_u0=True)
    p.name = f"warmstart_seed{seed}"
    return p


def tiny(m: int, s: int, alpha: float = 1.5, seed: int = 0, bvm: str = GBDF3) -> Problem:
    """Small smooth-random instance for tests (any m, s)."""
    p = smooth_random(m, s, alpha, seed, bvm)
    p.name = f"tiny_m{m}_s{s}_a{alpha}_{bvm}_seed{seed}"
    return p


def example41(alpha: float, m: int, s: int, bvm: str = GAM5) -> Problem:
    """Example 4.1: f = 0, constant d+ = 0.6 and d- = 0.5, Gaussian initial pulse
    exp(-(x - 1.2)^2 / (2 * 0.08^2)) on (0, 2), t in [0, 1]."""
    x = grid_x(m)
    u0 = np.exp(-((x - 1.2) ** 2) / (2.0 * 0.08 ** 2))
    return Problem(alpha=float(alpha), m=m, s=s, d_plus=np.full(m, 0.6), d_minus=np.full(m, 0.5),
                   f=np.zeros((s + 1, m)), u0=u0, bvm=bvm, name=f"example41_a{alpha}_m{m}_s{s}")


# (alpha, m, s) of the rows of Tables 1 and 2
EXAMPLE41_GRID = [(a, m, s) for a in (1.2, 1.5) for m in (24, 48, 96) for s in (16, 32, 64, 128)]
