"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Sizes span several workgroup tiles and ragged tails, both line-transform paths
(FFT for N+1 a power of two in 64..1024, direct sine sums otherwise), every scheme,
non-cubic grids, variable k(z) and non-zero z-face data.  The oracle forms weights
and right-hand side in FP64 and solves that discrete system with extended-precision
transforms and Thomas sweeps, so its own rounding is far below the FP64 level; the
bar for the FP64 GPU path is a relative L2 error of 1e-12, or four times the error of
the plain FP64 oracle on the same system where small pivots of the LU without
pivoting (Section 3.6) push that FP64 floor above 1e-12.  Every comparison is element
by element (max |u - U_o| / max |U_o|) and in the 2-norm, against a bar fixed before the
comparison (``parity.py``).
"""
import numpy as np
import pytest
import torch

import oracle as O
import parity as PT
import workloads as WL

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12


@pytest.fixture(scope="module")
def cs3d():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_03565_amd as m
    return m


def _oracle(p, r=0, F=None, W=None):
    gl = None if p.g_lo is None else p.g_lo[r].numpy()
    gh = None if p.g_hi is None else p.g_hi[r].numpy()
    return O.solve(p.scheme, None if F is not None else p.f[r].numpy(), p.hx, p.hy, p.hz,
                   p.k2, p.k2_z, p.k2_zz, p.gamma, gl, gh, W=W, F=F, dtype=np.longdouble)


def _bar(p, ref, r=0, tol=TOL_FP64):
    """Parity bar: tol, or 4x the FP64 noise floor of this discrete system where that is
    larger (ill-conditioned modal systems), per norm (parity.oracle_bar)."""
    return PT.oracle_bar(PT.problem_kw(p, r), ref.U, tol)


def _gpu_solve(cs3d, p):
    dev = torch.device("cuda:0")
    plan = cs3d.plan_for_problem(p, device=dev)
    u = plan.solve(p.f.to(dev), None if p.g_lo is None else p.g_lo.to(dev),
                   None if p.g_hi is None else p.g_hi.to(dev))
    st = plan.stats()
    out = u.cpu().numpy()
    plan.close()
    return out, st


CASES = [
    # (scheme, nx, ny, nz)   x/y transform path noted
    ("helm4", 63, 63, 63),      # fft64 / fft64
    ("helm6", 63, 127, 33),     # fft64 / fft128
    ("cd4", 255, 63, 17),       # fft256 / fft64
    ("helm2", 127, 255, 9),     # fft128 / fft256
    ("helm6", 511, 63, 6),      # fft512 / fft64
    ("helm4", 1023, 63, 5),     # fft1024 / fft64
    ("helm4", 63, 1023, 4),     # fft64 / fft1024
    ("helm6", 30, 17, 9),       # dense / dense, ragged tiles
    ("helm6", 65, 66, 7),       # dense / dense: last RHS tile of 1 column (x-face pass)
    ("helm6", 67, 70, 8),       # dense / dense: last RHS tile of 3 columns (x faces in the RHS pass)
    ("helm6", 5, 9, 6),         # dense tiny, x faces through the face pass
    ("cd4", 100, 63, 12),       # dense / fft64
    ("helm4", 63, 50, 7),       # fft64 / dense
    ("helm2", 5, 7, 6),         # dense tiny
    ("helm4", 1, 1, 1),         # degenerate single unknown
    ("cd4", 3, 2, 1),           # one plane
]


@pytest.mark.parametrize("scheme,nx,ny,nz", CASES)
def test_solve_matches_oracle(cs3d, scheme, nx, ny, nz):
    p = WL.noise_problem(nx, ny, nz, scheme, seed=1000 + nx + 7 * ny + 13 * nz)
    print(f"case {scheme} {nx}x{ny}x{nz}", flush=True)
    ref = _oracle(p)
    bar = _bar(p, ref)
    u, st = _gpu_solve(cs3d, p)
    PT.check(f"{scheme} {nx}x{ny}x{nz}", u[0], ref.U, bar)
    print(f"  minpiv gpu {st['min_abs_pivot']:.3e} oracle {ref.minpiv:.3e}", flush=True)
    assert st["bad_pivots"] == 0
    assert abs(st["min_abs_pivot"] - ref.minpiv) <= 1e-9 * max(1.0, ref.minpiv)


def test_multiple_rhs_share_one_plan(cs3d):
    p = WL.noise_problem(63, 63, 40, "helm6", seed=77, nrhs=3)
    refs = [_oracle(p, r) for r in range(3)]
    bars = [_bar(p, refs[r], r) for r in range(3)]
    u, _ = _gpu_solve(cs3d, p)
    for r in range(3):
        PT.check(f"rhs {r}", u[r], refs[r].U, bars[r])


def test_solve_assembled_with_generic_weights(cs3d):
    nx, ny, nz = 63, 30, 11
    rng = np.random.default_rng(3)
    W = rng.uniform(-1, 1, size=(nz, 3, 4))
    W[:, 1, 3] += 8.0  # keep the modal systems comfortably non-singular
    F = rng.standard_normal((1, nz, ny, nx))
    dev = torch.device("cuda:0")
    plan = cs3d.Plan(nx, ny, nz, 1.0, 1.0, 1.0, "weights", weights=W, device=dev)
    u = plan.solve_assembled(torch.from_numpy(F).to(dev)).cpu().numpy()
    ref = O.solve(None, None, 1.0, 1.0, 1.0, W=W, F=F[0], dtype=np.longdouble)
    PT.check("assembled, generic weights", u[0], ref.U, PT.Bar.fixed(TOL_FP64))


def test_residual_kernel_matches_oracle_operator(cs3d):
    p = WL.noise_problem(63, 40, 12, "helm6", seed=9)
    dev = torch.device("cuda:0")
    plan = cs3d.plan_for_problem(p, device=dev)
    rng = np.random.default_rng(4)
    U = rng.standard_normal((1, p.nz, p.ny, p.nx))
    W = O.stencil_weights("helm6", p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz)
    F = O.rhs("helm6", p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z)
    ref = F - O.apply_operator(W, O.closed(U[0], p.g_lo[0].numpy(), p.g_hi[0].numpy()))
    r = plan.residual(p.f.to(dev), torch.from_numpy(U).to(dev), p.g_lo.to(dev), p.g_hi.to(dev))
    PT.check("residual pass vs oracle operator", r[0].cpu().numpy(), ref, PT.Bar.fixed(TOL_FP64))


def test_config1_helm4_63_manufactured(cs3d):
    p = WL.config1()
    ref = _oracle(p)
    u, st = _gpu_solve(cs3d, p)
    PT.check("config 1 helm4 63^3", u[0], ref.U, PT.Bar.fixed(TOL_FP64))
    ue = p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1]
    # 4th-order discretisation error of the oracle's own solution is reproduced
    assert abs(np.abs(u[0] - ue).max() - np.abs(ref.U - ue).max()) < 1e-12


def test_paper_table5_on_gpu(cs3d):
    """Section 5.2.2, Table 5 (4th order, N = 125): printed max-err 3.4493268e-05."""
    p = WL.paper_variable_k(125, "helm4")
    ref = _oracle(p)
    u, _ = _gpu_solve(cs3d, p)
    PT.check("table 5 problem 125^3", u[0], ref.U, PT.Bar.fixed(TOL_FP64))
    ue = p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1]
    assert abs(np.abs(u[0] - ue).max() - 3.4493268e-05) < 0.75e-12


# ---------------------------------------------------------------------------
# Mixed precision: FP32 line transforms, FP64 tridiagonal LU, FP64 residual refinement
# ---------------------------------------------------------------------------
TOL_MIXED = 1e-10

MIXED_CASES = [
    ("helm6", 63, 127, 33),   # fft64 / fft128
    ("helm4", 255, 63, 17),   # fft256 / fft64
    ("cd4", 511, 63, 9),      # fft512 / fft64
    ("helm6", 63, 1023, 5),   # fft64 / fft1024 (two-wave lines)
    ("helm6", 30, 17, 9),     # dense / dense
]


@pytest.mark.parametrize("scheme,nx,ny,nz", MIXED_CASES)
def test_mixed_refined_matches_oracle(cs3d, scheme, nx, ny, nz):
    p = WL.noise_problem(nx, ny, nz, scheme, seed=2000 + nx + 7 * ny + 13 * nz)
    print(f"case mixed {scheme} {nx}x{ny}x{nz}", flush=True)
    ref = _oracle(p)
    bar = _bar(p, ref, tol=TOL_MIXED)
    dev = torch.device("cuda:0")
    plan = cs3d.plan_for_problem(p, precision="mixed", refine_steps=2, device=dev)
    u = plan.solve(p.f.to(dev), p.g_lo.to(dev), p.g_hi.to(dev)).cpu().numpy()
    st = plan.stats()
    plan.close()
    hist = st["residual_history"][:3]
    PT.check(f"mixed {scheme} {nx}x{ny}x{nz}", u[0], ref.U, bar)
    print(f"  residual history {hist}", flush=True)
    assert st["refine_done"] == 2
    assert hist[1] < hist[0] and hist[2] <= hist[1] * 1.01
    assert hist[2] < 1e-12
    assert st["status"] == 0


def test_mixed_without_refinement_is_fp32_accurate(cs3d):
    p = WL.noise_problem(127, 63, 20, "helm4", seed=31)
    dev = torch.device("cuda:0")
    plan = cs3d.plan_for_problem(p, precision="mixed", refine_steps=0, device=dev)
    u = plan.solve(p.f.to(dev), p.g_lo.to(dev), p.g_hi.to(dev)).cpu().numpy()
    st = plan.stats()
    ref = _oracle(p)
    l2, mx = PT.errors(u[0], ref.U)
    print(f"  mixed without refinement: rel L2 {l2:.3e}, rel max {mx:.3e}", flush=True)
    # single-precision transforms: error well above FP64, well below 1e-4
    assert 1e-9 < l2 < 1e-4 and 1e-9 < mx < 1e-4, (l2, mx)
    assert st["refine_done"] == 0 and st["residual_history"][0] > 1e-9


def test_mixed_multi_rhs(cs3d):
    p = WL.noise_problem(63, 63, 24, "helm6", seed=41, nrhs=2)
    refs = [_oracle(p, r) for r in range(2)]
    bars = [_bar(p, refs[r], r, tol=TOL_MIXED) for r in range(2)]
    dev = torch.device("cuda:0")
    plan = cs3d.plan_for_problem(p, precision="mixed", refine_steps=2, device=dev)
    u = plan.solve(p.f.to(dev), p.g_lo.to(dev), p.g_hi.to(dev)).cpu().numpy()
    for r in range(2):
        PT.check(f"mixed rhs {r}", u[r], refs[r].U, bars[r])
