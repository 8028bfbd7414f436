"""MI355X-native Strang-preconditioned all-at-once BVM solver for the two-sided
space-fractional diffusion equation (HIP kernels for gfx950 behind a C ABI)."""
from ._native import FdeError, NativeLibraryMissing, lib  # noqa: F401
from .solver import BvmSolver, autotune_report, factor_batch, solve_batch  # noqa: F401

__all__ = ["BvmSolver", "autotune_report", "factor_batch", "solve_batch", "FdeError", "NativeLibraryMissing", "lib"]
