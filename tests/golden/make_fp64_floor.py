"""Write fp64_floor.json: the FP64 oracle's own error at the full-size workloads.

    python tests/golden/make_fp64_floor.py

For the 511^3 workload (6th order, k = 50(1 + 0.3 z)) the extended-precision oracle is too
slow to run beside a GPU test (about 20 core-minutes per solve), so the GPU result is compared
with the FP64 oracle there, and the bar needs the FP64 oracle's own error.  This script
measures it two ways:
  * on the workload itself (--full): the FP64 oracle against the extended-precision oracle
    on the same discrete system (relative L2 and max);
  * on a discrete manufactured solution of the same operator: random U* in [-1, 1],
    F = A U* formed in extended precision (eq. stencil27) and rounded to FP64, solved by
    the FP64 oracle (relative L2 and max errors against U*).
With --full it also stores the extended-precision solution of the workload at sampled
points (every corner, edge midpoint and face centre, plus seeded random points), rounded to
FP64, with its 2-norm and largest magnitude, so that a GPU result can be compared with the
extended-precision oracle point by point at full size.
Calls only the oracle (``oracle/``) and the problem definitions (``workloads/``).  About 1.5
minutes and 25 GB; with --full about 35 minutes more.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as WL  # noqa: E402


def manufactured_error(p, seed):
    W = O.stencil_weights(p.scheme, p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma)
    Us = np.random.default_rng(seed).uniform(-1.0, 1.0, (p.nz, p.ny, p.nx))
    F = np.asarray(O.apply_operator(W, O.closed(Us.astype(np.longdouble))), dtype=np.float64)
    r = O.solve(None, None, p.hx, p.hy, p.hz, W=W, F=F)
    d = r.U - Us
    return {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(Us)),
            "rel_max": float(np.max(np.abs(d)) / np.max(np.abs(Us))),
            "min_abs_pivot": float(r.minpiv), "seed": seed}


def sample_indices(nz, ny, nx, count, seed):
    """0-based (z, y, x) indices of the interior array: corners, edge midpoints, face centres
    and `count` seeded random points."""
    pts = set()
    for z in (0, nz // 2, nz - 1):
        for y in (0, ny // 2, ny - 1):
            for x in (0, nx // 2, nx - 1):
                pts.add((z, y, x))
    rng = np.random.default_rng(seed)
    while len(pts) < 27 + count:
        pts.add((int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))))
    return sorted(pts)


def workload_error(p, samples=4000):
    """The FP64 oracle against the extended-precision oracle on the workload's own system,
    and the extended-precision solution at sampled points."""
    kw = dict(scheme=p.scheme, f=p.f[0].numpy(), hx=p.hx, hy=p.hy, hz=p.hz, k2=p.k2, k2_z=p.k2_z,
              k2_zz=p.k2_zz, gamma=p.gamma)
    u64 = O.solve(**kw).U
    ref = O.solve(**kw, dtype=np.longdouble).U
    d = u64 - ref
    pts = sample_indices(p.nz, p.ny, p.nx, samples, seed=p.nx)
    return {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "rel_max": float(np.max(np.abs(d)) / np.max(np.abs(ref))),
            "ext_norm2": float(np.linalg.norm(ref)), "ext_absmax": float(np.max(np.abs(ref))),
            "points": pts, "ext_values": [float(ref[z, y, x]) for (z, y, x) in pts]}


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--full", action="store_true", help="also the workload itself against the extended oracle")
    args = ap.parse_args()
    out = {"_source": "written by tests/golden/make_fp64_floor.py: the FP64 oracle's error on a "
                      "discrete manufactured solution (F = A U* in extended precision) of each "
                      "workload's operator, and (workload) on the workload's own system against the "
                      "extended-precision oracle"}
    for key, mk in (("config2_255", lambda: WL.config2(n=255)), ("config3_511", lambda: WL.config3(n=511))):
        t = time.time()
        out[key] = manufactured_error(mk(), seed=5)
        if args.full:
            out[key]["workload"] = workload_error(mk())
        print(key, out[key], f"{time.time() - t:.1f} s", flush=True)
    with open(os.path.join(HERE, "fp64_floor.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
