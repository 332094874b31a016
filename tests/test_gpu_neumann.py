"""GPU parity of Neumann sides (du/dn = 0 on the x and y faces, DCT-I transforms) against
the CPU oracle, through the C ABI.

The side nodes are unknowns, so a solution plane holds (ny+2) x (nx+2) values.  The cases
span the cosine FFT of every supported length (M = 64..512, with one or two waves per
y-line), direct cosine sums for other lengths (up to the longest line of 1023 nodes),
every scheme, non-cubic grids, z-face data on every node, a single plane and several
right-hand sides.  The bar is that of the Dirichlet FP64 path: 1e-12 relative to the
extended-precision oracle, or four times the FP64 oracle's own error where that is larger,
element by element and in the 2-norm (``parity.py``).  At 255^3 the extended-precision
oracle solves the whole system; at 511^3 (the FFT path at its largest
cosine length) the oracle's residual is checked at sampled points, faces, edges and
corners, with the mirror images taken from the full field.
"""
import numpy as np
import pytest
import torch

import oracle as O
import oracle_pool
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


def _oracle(p, r=0, dtype=np.longdouble, F=None):
    gl = None if p.g_lo is None else p.g_lo[r].numpy()
    gh = None if p.g_hi is None else p.g_hi[r].numpy()
    if F is not None:
        W = O.stencil_weights(p.scheme, p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma)
        return O.solve(None, None, p.hx, p.hy, p.hz, W=W, F=F, dtype=dtype, sides="neumann")
    return O.solve(p.scheme, p.f[r].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma, gl, gh,
                   dtype=dtype, sides="neumann")


def _gpu(cs3d, p, nrhs=1, tuning=None):
    plan = cs3d.plan_for_problem(p, device=DEV, max_rhs=nrhs)
    if tuning:
        t = plan.tuning()
        t.update(tuning)
        plan.set_tuning(t)
    gl = None if p.g_lo is None else p.g_lo.to(DEV)
    gh = None if p.g_hi is None else p.g_hi.to(DEV)
    u = plan.solve(p.f.to(DEV), gl, gh).cpu().numpy()
    st = plan.stats()
    plan.close()
    return u, st


CASES = [
    ("helm4", 63, 63, 17),      # cosine FFT 64 / 64
    ("helm6", 127, 63, 9),      # 128 / 64
    ("helm2", 255, 127, 5),     # 256 / 128
    ("cd4", 63, 511, 4),        # 64 / 512 (one wave per y-line)
    ("helm6", 511, 63, 6),      # 512 / 64
    ("helm4", 30, 17, 9),       # direct sums / direct sums, ragged tiles
    ("helm6", 600, 5, 4),       # a 602-node direct-sum line
    ("helm2", 1021, 3, 2),      # the longest line: 1023 nodes
    ("helm4", 1, 2, 1),         # 3 x 4 nodes, one plane: both z faces lift into it
]


@pytest.mark.parametrize("scheme,nx,ny,nz", CASES)
def test_neumann_matches_oracle(cs3d, scheme, nx, ny, nz):
    p = WL.neumann_noise_problem(nx, ny, nz, scheme, seed=4000 + nx + 7 * ny + 13 * nz)
    print(f"case neumann {scheme} {nx}x{ny}x{nz}", flush=True)
    ref = _oracle(p)
    bar = PT.oracle_bar(PT.problem_kw(p), ref.U)
    u, st = _gpu(cs3d, p)
    assert u.shape == (1, nz, ny + 2, nx + 2)
    PT.check(f"neumann {scheme} {nx}x{ny}x{nz}", u[0], ref.U, bar)
    print(f"  min pivot {st['min_abs_pivot']:.3e} (oracle {ref.minpiv:.3e})", flush=True)
    assert st["bad_pivots"] == 0
    assert abs(st["min_abs_pivot"] - ref.minpiv) <= 1e-9 * max(1.0, ref.minpiv)


def test_neumann_several_rhs_and_assembled(cs3d):
    p = WL.neumann_noise_problem(127, 65, 12, "helm6", seed=91, nrhs=3)
    refs = [_oracle(p, r).U for r in range(3)]
    bars = [PT.oracle_bar(PT.problem_kw(p, r), refs[r]) for r in range(3)]
    u, _ = _gpu(cs3d, p, nrhs=3)
    for r in range(3):
        PT.check(f"neumann rhs {r}", u[r], refs[r], bars[r])
    # the assembled path: the oracle's lifted F of right-hand side 2
    W = O.stencil_weights(p.scheme, p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz)
    F = O.lift(W, O.rhs(p.scheme, p.f[2].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, sides="neumann"),
               p.g_lo[2].numpy(), p.g_hi[2].numpy(), sides="neumann")
    plan = cs3d.plan_for_problem(p, device=DEV, max_rhs=1)
    ua = plan.solve_assembled(torch.from_numpy(F)[None].to(DEV)).cpu().numpy()
    plan.close()
    PT.check("assembled vs closed-grid path", ua[0], u[2], PT.Bar.fixed(1e-13))


def test_neumann_launch_shapes(cs3d):
    """xpersist leaves the result bitwise unchanged; two waves per 512-point y-line (another
    radix split) changes the rounding only."""
    p = WL.neumann_noise_problem(63, 511, 5, "helm4", seed=17)
    u0, _ = _gpu(cs3d, p)
    u1, _ = _gpu(cs3d, p, tuning={"xpersist": 0})
    u2, _ = _gpu(cs3d, p, tuning={"ywpl": 2})
    assert np.array_equal(u0, u1)
    PT.check("two waves per y-line vs one", u2, u0, PT.Bar.fixed(1e-13))


def test_neumann_manufactured_solution_orders(cs3d):
    """u = cos(pi x) cos(2 pi y) (sin 3 pi z + cos(pi z)/2): the HIP path's errors equal the
    oracle's and fall at orders 4 and 6 between N = 31 and 63."""
    prof = WL.problems.KProfile(lambda z: 4.0 + np.sin(2 * np.pi * z),
                                lambda z: 2 * np.pi * np.cos(2 * np.pi * z),
                                lambda z: -4 * np.pi ** 2 * np.sin(2 * np.pi * z))
    for scheme, lo, hi in (("helm4", 3.7, 4.4), ("helm6", 5.5, 6.8)):
        errs = []
        for n in (31, 63):
            p = WL.manufactured_cos2(n, n, n, scheme, prof)
            u, _ = _gpu(cs3d, p)
            ue = p.u_exact[0].numpy()[1:-1]
            e = np.abs(u[0] - ue).max()
            eo = np.abs(_oracle(p, dtype=np.float64).U - ue).max()
            assert abs(e - eo) <= 1e-12 + 1e-6 * eo
            errs.append(e)
        order = np.log2(errs[0] / errs[1])
        print(f"{scheme}: max errors {errs[0]:.3e}, {errs[1]:.3e}, order {order:.2f}", flush=True)
        assert lo < order < hi


def test_neumann_255_against_oracle(cs3d):
    """255^3 HELM6 with Neumann sides and z-face data against the extended-precision oracle
    (about a minute on the host, in worker processes), the bar fixed from the oracle alone."""
    p = WL.neumann_noise_problem(255, 255, 255, "helm6", seed=255, boundary=True)
    ref, minpiv, u64, ups = oracle_pool.oracle_set(PT.problem_kw(p))  # host worker processes
    bar = PT.Bar.from_oracle(ref, u64, ups)
    u, st = _gpu(cs3d, p)
    PT.check("neumann helm6 255^3", u[0], ref, bar)
    print(f"  min pivot {st['min_abs_pivot']:.3e} (oracle {minpiv:.3e})", flush=True)
    assert abs(st["min_abs_pivot"] - minpiv) <= 1e-9 * max(1.0, minpiv)


def _point_residuals(p, W, fpad, U, points):
    """|F - A U| / (|F| + sum |w| |U|) of the oracle at nodes (l, j, i) (l 1-based, j, i
    0-based), with f and U mirrored about the sides (fpad: f padded by 3 in x and y) and
    the z-face data in the boundary planes of U."""
    Upad = O.mirror_pad(O.closed(U, p.g_lo[0].numpy(), p.g_hi[0].numpy(), sides="neumann"), 1)
    out = []
    for (l, j, i) in points:
        az = min(max(l - 3, 0), p.nz - 5)  # the block's z faces are the box's near them
        blk = fpad[az:az + 7, j:j + 7, i:i + 7]  # node (j, i) at block interior (2, 2)
        Fb = O.rhs(p.scheme, blk, p.hx, p.hy, p.hz, p.k2[az:az + 7], p.k2_z[az:az + 7], p.gamma)
        F = Fb[l - 1 - az, 2, 2]
        U3 = Upad[l - 1:l + 2, j:j + 3, i:i + 3]
        Wl = W[l - 1:l]
        AU = O.apply_operator(Wl, U3)[0, 0, 0]
        scale = abs(F) + float(O.apply_operator(np.abs(Wl), np.abs(U3))[0, 0, 0])
        out.append(abs(F - AU) / scale)
    return np.array(out)


def test_neumann_511_point_residuals(cs3d):
    n = 511
    p = WL.neumann_noise_problem(n, n, n, "helm6", seed=511)
    u, st = _gpu(cs3d, p)
    assert st["bad_pivots"] == 0
    W = O.stencil_weights(p.scheme, p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz)
    fpad = O.mirror_pad(p.f[0].numpy(), 3)
    rng = np.random.default_rng(7)
    pts = {(int(rng.integers(1, n + 1)), int(rng.integers(0, n + 2)), int(rng.integers(0, n + 2)))
           for _ in range(120)}
    ends = (0, 1, n, n + 1)
    for l in (1, 2, n - 1, n):
        for j in ends:
            for i in (0, 1, n // 2, n, n + 1):
                pts.add((l, j, i))
    for j in ends:
        pts.add((n // 2, j, n // 3))
    res = _point_residuals(p, W, fpad, u[0], sorted(pts))
    print(f"511^3 neumann: {len(pts)} points, max oracle point residual {res.max():.2e}", flush=True)
    assert res.max() < 1e-11
