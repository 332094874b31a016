"""MI355X-native direct solver for compact 4th/6th-order 27-point discretisations.

Gonzales, Gryazin & Lee, "Scalable Algorithms for High-Order Approximations on
Three-Dimensional Compact Stencils" (arXiv 1912.03565), Section 3.6: 2-D DST-I in
x and y, N_x N_y tridiagonal LU solves along z, inverse DST - as hand-written HIP
kernels for gfx950 behind the C ABI of include/cs3d.h.
"""
from .native import CS3DError, lib  # noqa: F401  (raises ImportError if not built)
from .solver import Batch, Plan, batch_member, plan_for_problem  # noqa: F401
from .tuning import tuned_batch, tuned_plan  # noqa: F401
