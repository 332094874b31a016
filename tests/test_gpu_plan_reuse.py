"""Plans opened one after another on the same shape, each closed before the next opens.

The device allocator hands a new plan the addresses its predecessor freed, so every table
read by a kernel (the k^2 samples of the right-hand side pass, the stencil weights of the
residual, the modal coefficients of the y passes) then holds new values at an address
that held the previous plan's.  Each solve must follow its own k(z): the FP64, mixed,
complex and Neumann paths are checked against the oracle for three different media in
turn, twice over.
"""
import numpy as np
import pytest
import torch

import oracle as O
import parity as PT
import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SHAPE = (63, 31, 17)

PROFILES = [
    WL.problems.KProfile(lambda z: 6.0 + 2.0 * np.sin(3.0 * z), lambda z: 6.0 * np.cos(3.0 * z),
                         lambda z: -18.0 * np.sin(3.0 * z)),
    WL.problems.KProfile(lambda z: 20.0 + 5.0 * np.sin(z), lambda z: 5.0 * np.cos(z),
                         lambda z: -5.0 * np.sin(z)),
    WL.problems.KProfile(lambda z: 3.0 + np.cos(2.0 * z), lambda z: -2.0 * np.sin(2.0 * z),
                         lambda z: -4.0 * np.cos(2.0 * z)),
]
CPROFILES = [
    WL.problems.K_ABSORB,
    WL.problems.KProfile(lambda z: (15.0 + z) + 2j * (1.0 + z), lambda z: 1.0 + 2j,
                         lambda z: 0.0 * z),
]


@pytest.fixture(scope="module")
def cs3d():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_03565_amd as m
    return m


def _oracle(p, sides="dirichlet", dtype=np.longdouble):
    gl = None if p.g_lo is None else p.g_lo[0].numpy()
    gh = None if p.g_hi is None else p.g_hi[0].numpy()
    return O.solve(p.scheme, p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma,
                   gl, gh, dtype=dtype, sides=sides).U


def _bar(p, ref, tol, sides="dirichlet"):
    """tol, or four times the FP64 noise floor where the medium makes that larger (the
    parity suite's bar, parity.oracle_bar), per norm."""
    return PT.oracle_bar(PT.problem_kw(p), ref, tol)


def _dev(t, cplx):
    """To the device; complex data as planes of real, then imaginary parts."""
    if t is None:
        return None
    return (torch.stack([t.real, t.imag], dim=1).contiguous() if cplx else t).to(DEV)


def _solve(cs3d, p, **kw):
    plan = cs3d.plan_for_problem(p, device=DEV, **kw)
    c = plan.complex
    u = plan.solve(_dev(p.f, c), _dev(p.g_lo, c), _dev(p.g_hi, c)).cpu().numpy()
    plan.close()
    return u[0, 0] + 1j * u[0, 1] if c else u[0]


@pytest.mark.parametrize("path", ["fp64", "mixed", "neumann"])
def test_real_plans_in_turn_follow_their_own_medium(cs3d, path):
    nx, ny, nz = SHAPE
    for rep in range(2):
        for i, prof in enumerate(PROFILES):
            if path == "neumann":
                p = WL.neumann_noise_problem(nx, ny, nz, "helm6", seed=300 + i)
                p.k2, p.k2_z, p.k2_zz = WL.problems._zsamples(nz, p.hz, prof)
                kw, sides = {}, "neumann"
            else:
                p = WL.noise_problem(nx, ny, nz, "helm6", seed=300 + i, prof=prof)
                kw = {"precision": "mixed", "refine_steps": 2} if path == "mixed" else {}
                sides = "dirichlet"
            print(f"case {path} medium {i} pass {rep}", flush=True)
            ref = _oracle(p, sides)
            bar = _bar(p, ref, 1e-10 if path == "mixed" else 1e-12, sides)
            PT.check(f"{path} medium {i} pass {rep}", _solve(cs3d, p, **kw), ref, bar)


def test_complex_plans_in_turn_follow_their_own_medium(cs3d):
    nx, ny, nz = SHAPE
    for rep in range(2):
        for i, prof in enumerate(CPROFILES):
            p = WL.complex_noise_problem(nx, ny, nz, "helm6", seed=310 + i, prof=prof)
            print(f"case complex medium {i} pass {rep}", flush=True)
            ref = _oracle(p)
            PT.check(f"complex medium {i} pass {rep}", _solve(cs3d, p), ref, _bar(p, ref, 1e-12))


def test_batches_in_turn_follow_their_own_members(cs3d):
    """Batches of one layout (member sizes and schemes) but different media, each closed
    before the next opens: the work lists and member descriptors of each sit where its
    predecessor's were.  Every member matches a single plan of its own."""
    layout = [("helm6", 63, 31, 17), ("cd4", 127, 63, 9), ("helm4", 63, 63, 12)]
    for rep in range(2):
        for i, prof in enumerate(PROFILES):
            probs = [WL.noise_problem(nx, ny, nz, s, seed=320 + 10 * i + m, prof=prof, boundary=False)
                     for m, (s, nx, ny, nz) in enumerate(layout)]
            print(f"case batch medium {i} pass {rep}", flush=True)
            b = cs3d.Batch([cs3d.batch_member(p) for p in probs], device=DEV)
            us = [u.cpu().numpy() for u in b.solve([p.f[0].to(DEV) for p in probs])]
            b.close()
            for m, p in enumerate(probs):
                PT.check(f"batch member {m} vs own plan", us[m], _solve(cs3d, p), PT.Bar.fixed(1e-13))
