"""CPU FP64 oracle for the compact-stencil FFT direct solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never calls it and shares
no code with it.
"""
from .cs3d_oracle import *  # noqa: F401,F403
