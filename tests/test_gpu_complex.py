"""GPU parity of complex k(z) (absorbing media) against the CPU oracle, through the C ABI.

A complex plan (desc.k2_im set) takes planar fields: every complex array is its real part
followed by its imaginary part.  The cases span both transform paths (FFT lengths 64 to
1024 with one- and two-wave lines, dense sine sums), every Helmholtz scheme, non-cubic
grids, complex z-face data, a single plane and several right-hand sides.  The oracle
solves the same complex discrete system with extended-precision transforms and Thomas
sweeps; the bar is that of the real FP64 path, element by element and in the 2-norm
(``parity.py``).
"""
import numpy as np
import pytest
import torch

import oracle as O
import parity as PT
import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL_FP64 = 1e-12


@pytest.fixture(scope="module")
def cs3d():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_03565_amd as m
    return m


def planar(t):
    """(nrhs, ...) complex -> (nrhs, 2, ...) float64: real part, then imaginary part."""
    return torch.stack([t.real, t.imag], dim=1).contiguous().to(DEV)


def unplanar(t):
    a = t.cpu().numpy()
    return a[:, 0] + 1j * a[:, 1]


def _oracle(p, r=0, dtype=np.longdouble, k2=None, k2z=None, k2zz=None, f=None):
    gl = None if p.g_lo is None else p.g_lo[r].numpy()
    gh = None if p.g_hi is None else p.g_hi[r].numpy()
    return O.solve(p.scheme, p.f[r].numpy() if f is None else f, p.hx, p.hy, p.hz,
                   p.k2 if k2 is None else k2, p.k2_z if k2z is None else k2z,
                   p.k2_zz if k2zz is None else k2zz, 0.0, gl, gh, dtype=dtype)


def _gpu(cs3d, p, nrhs=1):
    plan = cs3d.plan_for_problem(p, device=DEV, max_rhs=nrhs)
    assert plan.complex
    u = plan.solve(planar(p.f), None if p.g_lo is None else planar(p.g_lo),
                   None if p.g_hi is None else planar(p.g_hi))
    st = plan.stats()
    plan.close()
    return unplanar(u), st


CASES = [
    ("helm4", 63, 63, 31),      # fft64 / fft64
    ("helm6", 63, 127, 33),     # fft64 / fft128
    ("helm2", 127, 255, 9),     # fft128 / fft256
    ("helm4", 511, 63, 6),      # fft512 / fft64
    ("helm6", 63, 1023, 5),     # fft64 / fft1024 (two-wave lines)
    ("helm6", 30, 17, 9),       # dense / dense, ragged tiles
    ("helm4", 3, 2, 1),         # one plane: both z faces lift into it
]


@pytest.mark.parametrize("scheme,nx,ny,nz", CASES)
def test_complex_k_matches_oracle(cs3d, scheme, nx, ny, nz):
    p = WL.complex_noise_problem(nx, ny, nz, scheme, seed=3000 + nx + 7 * ny + 13 * nz)
    print(f"case complex {scheme} {nx}x{ny}x{nz}", flush=True)
    ref = _oracle(p)
    bar = PT.oracle_bar(PT.problem_kw(p), ref.U)
    u, st = _gpu(cs3d, p)
    PT.check(f"complex {scheme} {nx}x{ny}x{nz}", u[0], ref.U, bar)
    print(f"  |Im U|/|U| {np.linalg.norm(ref.U.imag) / np.linalg.norm(ref.U):.2f}, "
          f"min pivot {st['min_abs_pivot']:.3e} (oracle {ref.minpiv:.3e})", flush=True)
    assert st["bad_pivots"] == 0
    assert abs(st["min_abs_pivot"] - ref.minpiv) <= 1e-9 * max(1.0, ref.minpiv)


def test_complex_several_rhs_and_assembled(cs3d):
    p = WL.complex_noise_problem(127, 63, 12, "helm6", seed=77, nrhs=3)
    refs = [_oracle(p, r).U for r in range(3)]
    bars = [PT.oracle_bar(PT.problem_kw(p, r), refs[r]) for r in range(3)]
    u, _ = _gpu(cs3d, p, nrhs=3)
    for r in range(3):
        PT.check(f"complex rhs {r}", u[r], refs[r], bars[r])
    # the assembled path: the oracle's lifted F of right-hand side 1
    W = O.stencil_weights(p.scheme, p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz)
    F = O.lift(W, O.rhs(p.scheme, p.f[1].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z),
               p.g_lo[1].numpy(), p.g_hi[1].numpy())
    plan = cs3d.plan_for_problem(p, device=DEV, max_rhs=1)
    ua = unplanar(plan.solve_assembled(planar(torch.from_numpy(F)[None])))
    plan.close()
    PT.check("assembled vs closed-grid path", ua[0], u[1], PT.Bar.fixed(1e-13))


def test_complex_conjugate_medium(cs3d):
    """k -> conj(k) with real data gives the conjugate solution."""
    p = WL.complex_noise_problem(63, 63, 20, "helm6", seed=5, boundary=False)
    p.f = torch.complex(p.f.real, torch.zeros_like(p.f.real))
    u1, _ = _gpu(cs3d, p)
    pc = WL.complex_noise_problem(63, 63, 20, "helm6", seed=5, boundary=False)
    pc.f = p.f
    pc.k2, pc.k2_z, pc.k2_zz = np.conj(p.k2), np.conj(p.k2_z), np.conj(p.k2_zz)
    u2, _ = _gpu(cs3d, pc)
    PT.check("conjugate medium", u2[0], np.conj(u1[0]), PT.Bar.fixed(1e-13))
    assert np.linalg.norm(u1[0].imag) > 1e-3 * np.linalg.norm(u1[0])


def test_complex_plan_with_real_k_equals_real_solves(cs3d):
    p = WL.noise_problem(63, 31, 17, "helm4", seed=8, boundary=False)
    fi = WL.uniform_pm1(123, tuple(p.f.shape))
    pr = WL.noise_problem(63, 31, 17, "helm4", seed=8, boundary=False)
    plan_r = cs3d.plan_for_problem(pr, device=DEV)
    ure = plan_r.solve(p.f.to(DEV)).cpu().numpy()[0]
    uim = plan_r.solve(fi.to(DEV)).cpu().numpy()[0]
    plan_r.close()
    pc = WL.noise_problem(63, 31, 17, "helm4", seed=8, boundary=False)
    pc.k2 = p.k2.astype(np.complex128)
    pc.f = torch.complex(p.f, fi)
    uc, _ = _gpu(cs3d, pc)
    PT.check("complex plan, real k", uc[0], ure + 1j * uim, PT.Bar.fixed(1e-13))
