"""Full-size checks in the configurations the benchmark and the workload list use.

At 511^3 and 1023^3 the oracle cannot solve the whole system in seconds, but it can
evaluate its own RHS operator (eq. scheme6, readings R6-R10) and 27-point operator
(eq. stencil27) at any single point from a few neighbours.  So the solution the HIP path
returns is checked point by point: at sampled interior points, on every face, edge and
corner of the box, the oracle's residual F - A U must be at the FP64 rounding level of
the point's terms (|F| + sum |w| |U| over the 27 neighbours).  A wrong transform, a wrong
eigenvalue or a dropped face term leaves residuals of the order of those terms.

* 1023^3, 6th order, k = 80 exp(-z), 4 right-hand sides, FP64 and mixed paths with the
  plan defaults bench.py times; the mixed result must also agree with the FP64 one to
  1e-10 (relative 2-norm, the benchmark's criterion).  At this size the whole solution is
  also checked element by element against a known exact answer: a discrete manufactured
  solution U* (random), F = A U* formed by the oracle's operator, solved by both paths;
* 511^3 (k = 50(1 + 0.3z), Gaussian RHS), FP64 and mixed, against a full FP64 oracle solve,
  element by element and in the 2-norm, and against the extended-precision oracle at stored
  sample points;
* 255^3 (k = 20(1 + 0.5 sin 2 pi z), smooth + noise RHS) against the extended-precision
  oracle.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import oracle_pool
import parity as PT
import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
# point residual bar: about 100 eps log2(N) of the point's terms; a wrong solve gives O(1)
TOL_POINT = 1e-11


@pytest.fixture(scope="module")
def cs3d():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_03565_amd as m
    return m


def _block_start(n, idx):
    """Closed-grid start of the 7-point block (5 interior points) holding interior point
    idx (1-based): the block's own faces are the box's faces wherever idx is within two
    points of them, so the oracle's one-sided differences fall where the box's do."""
    return min(max(idx - 3, 0), n - 5)


def sample_points(p, count, seed):
    rng = np.random.default_rng(seed)
    pts = {tuple(int(v) for v in (rng.integers(1, p.nz + 1), rng.integers(1, p.ny + 1), rng.integers(1, p.nx + 1)))
           for _ in range(count)}
    ends = lambda n: (1, 2, n - 1, n)  # noqa: E731
    for l in ends(p.nz):
        for j in ends(p.ny):
            for i in (1, p.nx // 2, p.nx):
                pts.add((l, j, i))
        pts.add((l, p.ny // 3, p.nx // 5))
    for j in ends(p.ny):
        pts.add((p.nz // 2, j, p.nx // 7))
    for i in ends(p.nx):
        pts.add((p.nz // 3, p.ny // 2, i))
    return sorted(pts)


def point_residuals(p, W, f_dev, u_dev, r, points):
    """Relative oracle residual at each point: |F - A U| / (|F| + sum |w| |U|)."""
    out = []
    for (l, j, i) in points:
        az, ay, ax = _block_start(p.nz, l), _block_start(p.ny, j), _block_start(p.nx, i)
        fb = f_dev[r, az:az + 7, ay:ay + 7, ax:ax + 7].cpu().numpy()
        Fb = O.rhs(p.scheme, fb, p.hx, p.hy, p.hz, p.k2[az:az + 7], p.k2_z[az:az + 7], p.gamma)
        F = Fb[l - 1 - az, j - 1 - ay, i - 1 - ax]
        # U on the 3 x 3 x 3 neighbourhood; zero outside the interior (homogeneous faces)
        U3 = np.zeros((3, 3, 3))
        z0, y0, x0 = max(l - 1, 1), max(j - 1, 1), max(i - 1, 1)
        z1, y1, x1 = min(l + 1, p.nz), min(j + 1, p.ny), min(i + 1, p.nx)
        blk = u_dev[r, z0 - 1:z1, y0 - 1:y1, x0 - 1:x1].cpu().numpy()
        U3[z0 - l + 1:z1 - l + 2, y0 - j + 1:y1 - j + 2, x0 - i + 1:x1 - i + 1 + 1] = blk
        Wl = W[l - 1:l]
        AU = O.apply_operator(Wl, U3)[0, 0, 0]
        scale = abs(F) + float(O.apply_operator(np.abs(Wl), np.abs(U3))[0, 0, 0])
        out.append(abs(F - AU) / scale)
    return np.array(out)


def _solve(cs3d, p, precision, nrhs, f=None):
    plan = cs3d.plan_for_problem(p, precision=precision, refine_steps=2, max_rhs=nrhs, device=DEV)
    u = plan.solve(p.f if f is None else f)
    st = plan.stats()
    plan.close()
    del plan
    torch.cuda.empty_cache()
    return u, st


def test_bench_configuration_1023(cs3d):
    p = WL.config5(n=1023, nrhs=4, device=DEV)
    W = O.stencil_weights(p.scheme, p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz)
    pts = sample_points(p, 160, seed=11)
    print(f"1023^3 x 4: {len(pts)} points per right-hand side", flush=True)
    u64, st = _solve(cs3d, p, "fp64", 4)
    assert st["bad_pivots"] == 0 and st["min_abs_pivot"] > 0
    for r in range(4):
        res = point_residuals(p, W, p.f, u64, r, pts)
        print(f"  fp64 rhs {r}: max point residual {res.max():.2e}", flush=True)
        assert res.max() < TOL_POINT
    umx, stm = _solve(cs3d, p, "mixed", 4)
    assert stm["status"] == 0 and stm["refine_done"] == 2
    print(f"  mixed residual history {stm['residual_history'][:3]}", flush=True)
    for r in range(4):
        res = point_residuals(p, W, p.f, umx, r, pts)
        d = float(torch.linalg.vector_norm(umx[r] - u64[r]) / torch.linalg.vector_norm(u64[r]))
        print(f"  mixed rhs {r}: max point residual {res.max():.2e}, vs fp64 {d:.2e}", flush=True)
        assert res.max() < TOL_POINT
        assert d <= 1e-10


def test_bench_configuration_1023_manufactured(cs3d):
    """A discrete manufactured solution of the 1023^3 bench operator (P7): U* uniform in
    [-1, 1] (seeded), F = A U* by the oracle's 27-point operator (eq. stencil27), and the
    FP64 and mixed plans of the bench solve A U = F (solve_assembled).  An FP64 direct solve
    is accurate to about cond * eps; the bar is 16 eps max|lambda^0| / min|pivot| (the
    pivot-based condition estimate of the modal systems)."""
    p = WL.config5(n=1023, nrhs=1, device="cpu", planes=1)  # the operator only; f is not used
    W = O.stencil_weights(p.scheme, p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz)
    Us = np.random.default_rng(1023).uniform(-1.0, 1.0, (p.nz, p.ny, p.nx))
    F = O.apply_operator(W, O.closed(Us))
    Fd = torch.from_numpy(F)[None].to(DEV)
    del F
    # max |lambda^0| <= |d| + 2|b| + 2|c| + 4|a| over the rows (Section 3.6)
    lam0 = (np.abs(W[:, 1, 3]) + 2 * np.abs(W[:, 1, 1]) + 2 * np.abs(W[:, 1, 2]) + 4 * np.abs(W[:, 1, 0])).max()
    for precision in ("fp64", "mixed"):
        plan = cs3d.plan_for_problem(p, precision=precision, refine_steps=2, max_rhs=1, device=DEV)
        u = plan.solve_assembled(Fd).cpu().numpy()[0]
        st = plan.stats()
        plan.close()
        del plan
        torch.cuda.empty_cache()
        cond = lam0 / st["min_abs_pivot"]
        bar = PT.Bar.fixed(16 * np.finfo(np.float64).eps * cond,
                           f"; 16 eps cond, cond = max|lambda0| / min|pivot| = {cond:.2e}")
        PT.check(f"1023^3 manufactured, {precision}", u, Us, bar)


def _fp64_floor(golden_dir, key):
    """The FP64 oracle's own error at this workload, and the extended-precision solution at
    sampled points (stored by make_fp64_floor.py --full from the oracle alone)."""
    with open(os.path.join(golden_dir, "fp64_floor.json")) as fh:
        return json.load(fh)[key]


@pytest.mark.timeout(900)  # host oracle work in worker processes
def test_config3_511(cs3d, golden_dir):
    """511^3, FP64 and mixed: (1) against a full FP64 oracle solve (about a minute on the
    host), element by element and in the 2-norm, and (2) against the extended-precision
    oracle at 4027 stored points (corners, edge midpoints, face centres, seeded random
    points).  On this workload the FP64 oracle itself is 9e-11 away from the extended
    solution (near-singular modal systems, min pivot 3e-4), so each bar is 1e-12 (1e-10
    mixed) or four times that stored FP64-oracle error, per norm."""
    p = WL.config3(n=511, device="cpu")
    fl = _fp64_floor(golden_dir, "config3_511")["workload"]
    ref = O.solve(p.scheme, p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma, None, None)
    why = (f"; FP64 oracle vs extended on this workload L2 {fl['rel_l2']:.2e}, max {fl['rel_max']:.2e} "
           f"-> bar 4x")
    f_dev = p.f.to(DEV)
    u64, st = _solve(cs3d, p, "fp64", 1, f=f_dev)
    umx, stm = _solve(cs3d, p, "mixed", 1, f=f_dev)
    assert st["bad_pivots"] == 0 and stm["status"] == 0
    pts = tuple(np.array(fl["points"]).T)
    ext = np.array(fl["ext_values"])
    for name, u, tol in (("fp64", u64, PT.TOL_FP64), ("mixed", umx, PT.TOL_MIXED)):
        un = u[0].cpu().numpy()
        bar = PT.Bar(max(tol, 4 * fl["rel_l2"]), max(tol, 4 * fl["rel_max"]), why)
        PT.check(f"511^3 {name} vs FP64 oracle", un, ref.U, bar)
        e = float(np.max(np.abs(un[pts] - ext)) / fl["ext_absmax"])
        print(f"  511^3 {name} vs extended oracle at {len(ext)} points: rel max {e:.3e} "
              f"(bar {bar.mx:.1e})", flush=True)
        assert e < bar.mx
    d = float(torch.linalg.vector_norm(umx[0] - u64[0]) / torch.linalg.vector_norm(u64[0]))
    print(f"  mixed vs fp64 GPU {d:.2e}, min pivot {st['min_abs_pivot']:.3e} (oracle {ref.minpiv:.3e})",
          flush=True)
    assert abs(st["min_abs_pivot"] - ref.minpiv) <= 1e-9 * max(1.0, ref.minpiv)
    W = O.stencil_weights(p.scheme, p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz)
    pts = sample_points(p, 120, seed=13)
    r64 = point_residuals(p, W, p.f, u64, 0, pts)
    print(f"  oracle point residuals at {len(pts)} points: max {r64.max():.2e}", flush=True)
    assert r64.max() < TOL_POINT


@pytest.mark.timeout(900)  # host oracle work in worker processes
def test_config2_255_against_oracle(cs3d):
    """255^3 against the extended-precision oracle solved in full (about a minute on the
    host, in worker processes); bar 1e-12, or four times the FP64 noise floor of this system
    (parity.Bar.from_oracle), per norm."""
    p = WL.config2(n=255, device="cpu")
    ref, minpiv, u64, ups = oracle_pool.oracle_set(PT.problem_kw(p))  # host worker processes
    bar = PT.Bar.from_oracle(ref, u64, ups)
    u, st = _solve(cs3d, p, "fp64", 1, f=p.f.to(DEV))
    PT.check("255^3 fp64 vs extended oracle", u[0].cpu().numpy(), ref, bar)
    print(f"  min pivot {st['min_abs_pivot']:.3e} (oracle {minpiv:.3e})", flush=True)
    assert abs(st["min_abs_pivot"] - minpiv) <= 1e-9 * max(1.0, minpiv)
