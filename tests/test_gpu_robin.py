"""GPU parity of Robin z faces (alpha u_z + beta u = g on the z faces, Section 1, eq. bc;
reading R22) against the CPU oracle, through the C ABI.

The z-face nodes are unknowns, so a solution holds nz + 2 planes (z_0 .. z_{nz+1}).  The
cases span the FFT transform (N+1 = 64 .. 1024, one and two waves per y line) and the dense
sine sums, HELM2/HELM4/HELM6, non-cubic grids, several right-hand sides and the assembled
path.  The bar is that of the Dirichlet FP64 path (``parity.py``): 1e-12 against the
extended-precision oracle, or four times the FP64 noise floor of the system (the FP64
oracle's error and the one-ulp weight and eigenvalue sensitivities), element by element and
in the 2-norm.
The manufactured solution's errors on the GPU equal the oracle's, at observed orders 2, 4, 4.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import parity as PT
import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def cs3d():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_03565_amd as m
    return m


def _kw(p, r=0):
    return dict(scheme=p.scheme, f=p.f[r].numpy(), hx=p.hx, hy=p.hy, hz=p.hz, k2=p.k2, k2_z=p.k2_z,
                k2_zz=p.k2_zz, alpha=p.robin[0], beta=p.robin[1], g_lo=p.g_lo[r].numpy(),
                g_hi=p.g_hi[r].numpy())


def _reference(p, r=0, tol=PT.TOL_FP64):
    """Extended-precision oracle solution and the bar from the oracle alone."""
    kw = _kw(p, r)
    ref = O.solve_robin(**kw, dtype=np.longdouble)
    return ref, PT.oracle_bar(dict(kw, solver="robin"), ref.U, tol)


def _gpu(cs3d, p, nrhs=1):
    plan = cs3d.plan_for_problem(p, device=DEV, max_rhs=nrhs)
    u = plan.solve(p.f.to(DEV), p.g_lo.to(DEV), p.g_hi.to(DEV)).cpu().numpy()
    st = plan.stats()
    plan.close()
    return u, st


CASES = [
    ("helm4", 63, 63, 31),      # fft64 / fft64
    ("helm6", 63, 127, 20),     # fft64 / fft128
    ("helm2", 255, 127, 9),     # fft256 / fft128
    ("helm4", 511, 63, 6),      # fft512 / fft64
    ("helm6", 63, 1023, 5),     # fft64 / fft1024 (two-wave lines)
    ("helm6", 30, 17, 9),       # dense / dense, ragged tiles
    ("helm4", 100, 63, 4),      # dense / fft64, the fewest interior planes
]


@pytest.mark.parametrize("scheme,nx,ny,nz", CASES)
def test_robin_matches_oracle(cs3d, scheme, nx, ny, nz):
    p = WL.robin_noise_problem(nx, ny, nz, scheme, seed=6000 + nx + 7 * ny + 13 * nz)
    print(f"case robin {scheme} {nx}x{ny}x{nz}", flush=True)
    ref, bar = _reference(p)
    u, st = _gpu(cs3d, p)
    assert u.shape == (1, nz + 2, ny, nx)
    PT.check(f"robin {scheme} {nx}x{ny}x{nz}", u[0], ref.U, bar)
    print(f"  min pivot {st['min_abs_pivot']:.3e} (oracle {ref.minpiv:.3e})", flush=True)
    assert st["bad_pivots"] == 0
    assert abs(st["min_abs_pivot"] - ref.minpiv) <= 1e-9 * max(1.0, ref.minpiv)


def test_robin_several_rhs_and_assembled(cs3d):
    p = WL.robin_noise_problem(127, 63, 12, "helm6", seed=93, nrhs=3)
    refs = [_reference(p, r) for r in range(3)]
    u, _ = _gpu(cs3d, p, nrhs=3)
    for r in range(3):
        PT.check(f"robin rhs {r}", u[r], refs[r][0].U, refs[r][1])
    # the assembled path: the oracle's lifted F (face rows included) of right-hand side 1
    plan = cs3d.plan_for_problem(p, device=DEV, max_rhs=1)
    ua = plan.solve_assembled(torch.from_numpy(refs[1][0].F)[None].to(DEV)).cpu().numpy()
    plan.close()
    PT.check("assembled vs closed-grid path", ua[0], u[1], PT.Bar.fixed(1e-13))


def test_robin_manufactured_orders(cs3d):
    """The HIP path's errors against the exact solution equal the oracle's, and fall at the
    closure's orders: 2 (HELM2), 4 (HELM4), 4 (HELM6) between N = 31 and 63."""
    for scheme, lo, hi in (("helm2", 1.9, 2.1), ("helm4", 3.7, 4.3), ("helm6", 3.7, 4.3)):
        errs = []
        for n in (31, 63):
            p = WL.manufactured_robin(n, scheme)
            u, _ = _gpu(cs3d, p)
            ue = p.u_exact[0].numpy()[:, 1:-1, 1:-1]
            e = np.abs(u[0] - ue).max()
            eo = np.abs(O.solve_robin(**_kw(p)).U - ue).max()
            assert abs(e - eo) <= 1e-12 + 1e-6 * eo, (scheme, n, e, eo)
            errs.append(e)
        order = math.log2(errs[0] / errs[1])
        print(f"{scheme}: max errors {errs[0]:.3e}, {errs[1]:.3e}, order {order:.2f}", flush=True)
        assert lo < order < hi


def test_robin_refused_combinations(cs3d):
    N = cs3d.native
    p = WL.robin_noise_problem(63, 31, 8, "helm4", seed=1)
    for kw in ({"precision": "mixed"},):
        with pytest.raises(cs3d.CS3DError) as ei:
            cs3d.plan_for_problem(p, device=DEV, **kw)
        assert ei.value.status == N.E_UNSUPPORTED
    q = WL.robin_noise_problem(63, 31, 8, "cd4", seed=1)
    with pytest.raises(cs3d.CS3DError) as ei:
        cs3d.plan_for_problem(q, device=DEV)
    assert ei.value.status == N.E_UNSUPPORTED
    bad = WL.robin_noise_problem(63, 31, 8, "helm4", seed=1, robin=((0.0, 1.0), (1.0, 1.0)))
    with pytest.raises(cs3d.CS3DError) as ei:
        cs3d.plan_for_problem(bad, device=DEV)
    assert ei.value.status == N.E_INVAL
    plan = cs3d.plan_for_problem(p, device=DEV)
    f = p.f.to(DEV)
    u = torch.zeros(plan.interior_shape(1), dtype=torch.float64, device=DEV)
    with pytest.raises(cs3d.CS3DError) as ei:
        plan.residual(f, u)
    assert ei.value.status == N.E_UNSUPPORTED
    plan.close()
