"""MI355X-native batched trace(E X(p)) for parametrized Lyapunov equations.

The compute path lives in liblyapsmw.so (HIP, gfx950); ``lyapsmw`` is its
thin ctypes binding.  Importing the package does not touch the GPU.
"""
from .lyapsmw import (Seed, Engine, LyapError, solve_opts, load, EXPORTS,  # noqa: F401
                      RESULT_DTYPE, PREC, BASIS, profile_enable, profile_read, calib_copy,
                      real_schur, last_error, EKSpace, seed_x0v, EK_RESULT_DTYPE)
