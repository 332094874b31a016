"""Oracle solves for GPU tests in CPU worker processes.

A batch of 64 members up to 255^3 needs about 800 core-seconds of extended-precision oracle
work per solve (numpy's long double products run without BLAS); spread over the host's cores
it takes about a minute.  Workers are spawned (they never touch the GPU) and run numpy with
one thread each.

For every problem the workers compute what the bar of the comparison needs, from the oracle
alone: the extended-precision solution, the plain FP64 oracle's error against it, and two
sensitivities of the extended-precision solution, which bound how far any FP64
implementation of the method can land from it:
  * weights: every stencil weight moved by one FP64 unit in the last place (random signs);
  * modal eigenvalues: every lambda^o(n, m) of Section 3.6 moved by one unit in the last
    place, with a random sign per (offset, n, m) that is the same in every row l.  Any FP64
    evaluation rounds these eigenvalues, and on rows of equal weights the rounding repeats
    down the whole z column, which near-singular modes amplify the most (two sign draws).

Test infrastructure: numpy and the oracle only.
"""
import multiprocessing as mp
import os

import numpy as np


def _errors(u, ref):
    d = u - ref
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)),
            float(np.max(np.abs(d)) / np.max(np.abs(ref))))


def perturbed_weights(W, seed=1):
    """W with every entry moved by one unit in the last place (random signs; real and
    imaginary parts alike)."""
    rng = np.random.default_rng(seed)
    eps = np.finfo(np.float64).eps
    if np.iscomplexobj(W):
        re = W.real * (1.0 + eps * rng.choice([-1.0, 1.0], size=W.shape))
        im = W.imag * (1.0 + eps * rng.choice([-1.0, 1.0], size=W.shape))
        return re + 1j * im
    return W * (1.0 + eps * rng.choice([-1.0, 1.0], size=W.shape))


def _lam_perturbation(seed):
    """A modal_eigenvalues that moves every eigenvalue by one FP64 ulp (relative), the sign
    drawn per (offset, n, m) and the same in every row."""
    import oracle.cs3d_oracle as OC
    orig = OC.modal_eigenvalues

    def perturbed(W, nx, ny, dtype=np.float64, sides="dirichlet"):
        lam = orig(W, nx, ny, dtype, sides)
        sg = np.random.default_rng(seed).choice([-1.0, 1.0], size=(1,) + lam.shape[1:])
        return lam * (1 + np.finfo(np.float64).eps * sg)
    return orig, perturbed


def _job(args):
    """kind: 'ext' (extended precision), 'fp64', 'pert' (extended precision, perturbed
    weights), 'lam1' / 'lam2' (extended precision, eigenvalues perturbed with sign draw 1 /
    2).  kw may name 'solver': 'robin' (oracle.solve_robin) instead of oracle.solve.
    Returns (U, min |pivot|)."""
    kind, kw = args
    import oracle as O
    import oracle.cs3d_oracle as OC
    kw = dict(kw)
    robin = kw.pop("solver", None) == "robin"
    solve = O.solve_robin if robin else O.solve
    sides = kw.get("sides", "dirichlet")
    if kind in ("lam1", "lam2"):
        orig, perturbed = _lam_perturbation(1 if kind == "lam1" else 2)
        OC.modal_eigenvalues = perturbed
        try:
            r = solve(**kw, dtype=np.longdouble)
        finally:
            OC.modal_eigenvalues = orig
        return r.U, r.minpiv
    if kind == "pert" and robin:
        nz = np.asarray(kw["f"]).shape[0] - 2
        W = O.robin_weights(kw["scheme"], nz, kw["hx"], kw["hy"], kw["hz"], kw["k2"], kw.get("k2_z"), kw.get("k2_zz"))
        r = O.solve_robin(**kw, dtype=np.longdouble, W=perturbed_weights(W))
        return r.U, r.minpiv
    if kind == "pert":
        W = O.stencil_weights(kw["scheme"], np.asarray(kw["f"]).shape[0] - 2, kw["hx"], kw["hy"], kw["hz"],
                              kw.get("k2"), kw.get("k2_z"), kw.get("k2_zz"), kw.get("gamma", 0.0))
        F = O.rhs(kw["scheme"], kw["f"], kw["hx"], kw["hy"], kw["hz"], kw.get("k2"), kw.get("k2_z"),
                  kw.get("gamma", 0.0), sides)
        r = O.solve(None, None, kw["hx"], kw["hy"], kw["hz"], W=perturbed_weights(W), F=F,
                    g_lo=kw.get("g_lo"), g_hi=kw.get("g_hi"), dtype=np.longdouble, sides=sides)
    else:
        r = solve(**kw, dtype=np.longdouble if kind == "ext" else np.float64)
    return r.U, r.minpiv


PERTURBATIONS = ("pert", "lam1", "lam2")


def _task(args):
    """One problem in one worker: the extended, FP64 and perturbed solves, then scalars only."""
    name, kw, u_hip = args
    ref, minpiv = _job(("ext", kw))
    u64, _ = _job(("fp64", kw))
    sens = {k: _errors(_job((k, kw))[0], ref) for k in PERTURBATIONS}
    return {"name": name, "fp64_oracle": _errors(u64, ref), "sensitivity": sens,
            "hip": _errors(u_hip, ref), "minpiv": minpiv}


def workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _indexed(args):
    fn, i, item = args
    return i, fn(item)


def _run(fn, items, nproc):
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        out = [None] * len(items)
        with mp.get_context("spawn").Pool(nproc) as pool:
            # one line per finished item, so a long pool run keeps printing
            for k, (i, r) in enumerate(pool.imap_unordered(_indexed, [(fn, i, it) for i, it in enumerate(items)])):
                out[i] = r
                print(f"    oracle jobs: {k + 1} of {len(items)} done", flush=True)
        return out
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def extended_comparisons(tasks):
    """tasks: (name, oracle.solve keyword arguments without dtype, HIP result) in any order.
    Returns per-task dicts (errors of the FP64 oracle, of the perturbed-weights solution and
    of the HIP result, each against the extended-precision oracle, as (rel L2, rel max)) in
    the order given; the most expensive tasks start first (cost ~ unknowns * (nx + ny), the
    dense transform sums)."""
    def cost(t):
        nz, ny, nx = np.asarray(t[1]["f"]).shape
        return nx * ny * nz * (nx + ny)
    order = sorted(range(len(tasks)), key=lambda i: -cost(tasks[i]))
    res = _run(_task, [tasks[i] for i in order], workers())
    out = [None] * len(tasks)
    for i, r in zip(order, res):
        out[i] = r
    return out


def oracle_set(kw):
    """One large problem: the extended-precision, FP64 and perturbed oracle solves in worker
    processes at once.  Returns (extended U, min |pivot|, FP64 U, [perturbed U ...])."""
    kinds = ("ext", "fp64") + PERTURBATIONS
    res = _run(_job, [(k, kw) for k in kinds], len(kinds))
    return res[0][0], res[0][1], res[1][0], [r[0] for r in res[2:]]
