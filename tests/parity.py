"""Comparison of HIP results with oracle results, shared by the GPU tests.

Every comparison is element by element and in the 2-norm:

    rel_max = max |u - U_o| / max |U_o|,     rel_l2 = ||u - U_o||_2 / ||U_o||_2,

each against a bar fixed before the HIP result is looked at.  The FP64 bar is 1e-12.  Where
the modal tridiagonal systems are near-singular (LU without pivoting, Section 3.6), no FP64
implementation reaches that: the bar is then four times the FP64 noise floor of this
discrete system, where that is larger, per norm.  The floor is the largest of these
oracle-only measures against the extended-precision solution: the error of the plain FP64
oracle; the change of the extended-precision solution when every stencil weight moves by
one unit in the last place (random signs); and when every modal eigenvalue moves by one unit
in the last place with a random sign per (offset, n, m) that repeats in every row (two
draws), which models the rounding any FP64 evaluation of the eigenvalues of Section 3.6
makes (``oracle_pool.py``).  The line printed for the case gives the numbers.  The
mixed-precision bar is 1e-10 (after two refinement steps), raised the same way.

Test infrastructure: numpy and the oracle only.
"""
import numpy as np

import oracle as O

TOL_FP64 = 1e-12
TOL_MIXED = 1e-10


def errors(u, ref):
    """(rel_l2, rel_max) of u against ref (any shape, real or complex)."""
    u = np.asarray(u)
    ref = np.asarray(ref)
    d = u - ref
    l2 = float(np.linalg.norm(d) / np.linalg.norm(ref))
    mx = float(np.max(np.abs(d)) / np.max(np.abs(ref)))
    return l2, mx


class Bar:
    """Per-norm bar and the reason it has its value (printed with the comparison)."""

    def __init__(self, l2, mx, why=""):
        self.l2, self.mx, self.why = float(l2), float(mx), why

    @staticmethod
    def fixed(tol, why=""):
        return Bar(tol, tol, why)

    @staticmethod
    def from_errors(e64, sens, tol=TOL_FP64):
        """tol, or four times the FP64 noise floor, per norm: e64 the FP64 oracle's (L2, max)
        error and sens the (L2, max) changes under the perturbations (weights, eigenvalues),
        all against the extended-precision solution."""
        l2 = max([tol, 4 * e64[0]] + [4 * w[0] for w in sens])
        mx = max([tol, 4 * e64[1]] + [4 * w[1] for w in sens])
        why = ""
        if l2 > tol or mx > tol:
            why = (f"; FP64 oracle vs extended L2 {e64[0]:.2e} / max {e64[1]:.2e}, one-ulp "
                   f"sensitivities (weights, eigenvalues x2) L2 "
                   + ", ".join(f"{w[0]:.2e}" for w in sens) + " -> bar 4x")
        return Bar(l2, mx, why)

    @staticmethod
    def from_oracle(ref, u64, ups, tol=TOL_FP64):
        """Bar.from_errors from the solutions: u64 (FP64 oracle) and ups (the perturbed
        extended-precision solutions), against the extended-precision solution ref."""
        return Bar.from_errors(errors(u64, ref), [errors(up, ref) for up in ups], tol)


def check(label, u, ref, bar):
    """Assert u matches ref under ``bar`` in both norms; print both errors first."""
    l2, mx = errors(u, ref)
    print(f"  {label}: rel L2 {l2:.3e} (bar {bar.l2:.1e}), rel max {mx:.3e} (bar {bar.mx:.1e})"
          f"{bar.why}", flush=True)
    assert l2 < bar.l2, (label, "L2", l2, bar.l2)
    assert mx < bar.mx, (label, "max", mx, bar.mx)
    return l2, mx


def problem_kw(p, r=0):
    """oracle.solve keyword arguments of right-hand side r of a workloads.Problem."""
    return dict(scheme=p.scheme, f=p.f[r].numpy(), hx=p.hx, hy=p.hy, hz=p.hz, k2=p.k2, k2_z=p.k2_z,
                k2_zz=p.k2_zz, gamma=p.gamma,
                g_lo=None if p.g_lo is None else p.g_lo[r].numpy(),
                g_hi=None if p.g_hi is None else p.g_hi[r].numpy(),
                sides=getattr(p, "sides", "dirichlet"))


def oracle_bar(kw, ref, tol=TOL_FP64):
    """Bar.from_oracle for a problem given as oracle.solve keyword arguments (or those of
    oracle.solve_robin with solver="robin"), whose extended-precision solution is ref
    (computed here: the FP64 oracle and the perturbed solves)."""
    import oracle_pool
    u64, _ = oracle_pool._job(("fp64", kw))
    ups = [oracle_pool._job((k, kw))[0] for k in oracle_pool.PERTURBATIONS]
    return Bar.from_oracle(ref, u64, ups, tol)


def oracle_pair(solve_kwargs):
    """Extended-precision and FP64 oracle solutions of one problem: (ref result, U64)."""
    ref = O.solve(**solve_kwargs, dtype=np.longdouble)
    u64 = O.solve(**solve_kwargs).U
    return ref, u64
