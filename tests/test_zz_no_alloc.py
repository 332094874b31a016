"""cs3d_solve_static: the solve variant that allocates nothing (its workspace is a static
device array of the library), through the C ABI, against cs3d_solve on the same plan.

Two calls in a row on one device share the scratch; the second is smaller than the first,
so stale contents of the first call sit where the second one works.  Each result must match
cs3d_solve with the plan's own workspace to the FP64 parity bar (in fact bitwise: the same
kernels run on the same data).  Sizes beyond the scratch are refused with E_TOO_LARGE.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def cs3d():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_03565_amd as m
    return m


def _check(label, u, ref, tol):
    """Element-wise and 2-norm relative difference, both below tol."""
    d = u - ref
    l2 = float(np.linalg.norm(d) / np.linalg.norm(ref))
    mx = float(np.abs(d).max() / np.abs(ref).max())
    print(f"  {label}: rel L2 {l2:.3e}, rel max {mx:.3e} (bar {tol:.0e})", flush=True)
    assert l2 < tol and mx < tol, (label, l2, mx)


def _static_solve(cs3d, plan, f, gl, gh, nrhs):
    N = cs3d.native
    u = torch.full((nrhs, plan.nz, plan.ny, plan.nx), float("nan"), dtype=torch.float64, device=DEV)
    st = N.lib.cs3d_solve_static(plan._plan, nrhs, f.data_ptr(), gl.data_ptr(), gh.data_ptr(),
                                 u.data_ptr(), ctypes.c_void_p(0))
    N.check("cs3d_solve_static", st)
    torch.cuda.synchronize()
    return u


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_scratch_matches_solve_twice(cs3d, precision):
    cases = [("helm6", 127, 63, 40, 2), ("helm4", 63, 31, 17, 1)]  # second call smaller
    for scheme, nx, ny, nz, nrhs in cases:
        p = WL.noise_problem(nx, ny, nz, scheme, seed=7100 + nx + nz, nrhs=nrhs)
        plan = cs3d.plan_for_problem(p, precision=precision, refine_steps=2, device=DEV)
        need = cs3d.native.lib.cs3d_workspace_bytes(plan._plan, nrhs)
        assert 0 < need <= (64 << 20)
        f, gl, gh = p.f.to(DEV), p.g_lo.to(DEV), p.g_hi.to(DEV)
        ref = plan.solve(f, gl, gh).cpu().numpy()
        us = _static_solve(cs3d, plan, f, gl, gh, nrhs).cpu().numpy()
        st = plan.stats()
        assert st["bad_pivots"] == 0 and st["status"] == 0
        for r in range(nrhs):
            _check(f"static {precision} {scheme} {nx}x{ny}x{nz} rhs {r}", us[r], ref[r],
                   1e-12 if precision == "fp64" else 1e-10)
        print(f"  bitwise equal to cs3d_solve: {np.array_equal(us, ref)}", flush=True)
        plan.close()


def test_static_scratch_refuses_large_problems(cs3d):
    p = WL.noise_problem(255, 255, 255, "helm4", seed=3, boundary=False)
    plan = cs3d.plan_for_problem(p, device=DEV)
    N = cs3d.native
    assert N.lib.cs3d_workspace_bytes(plan._plan, 1) > (64 << 20)
    u = torch.empty((1, 255, 255, 255), dtype=torch.float64, device=DEV)
    f = p.f.to(DEV)
    st = N.lib.cs3d_solve_static(plan._plan, 1, f.data_ptr(), None, None, u.data_ptr(), ctypes.c_void_p(0))
    assert st == N.E_TOO_LARGE
    assert "static" in N.status_str(st)
    plan.close()
