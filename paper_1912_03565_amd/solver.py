"""Python front end of the HIP solver: shape checks and pointer marshalling.

All arithmetic happens in libcs3d.so.  Tensors must be float64, contiguous and on
the HIP device; the shape of every operand is checked here before any launch so a
wrong-sized buffer is rejected instead of being read out of bounds.
"""
import ctypes

import numpy as np
import torch

from . import native as N


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _host_array(a, n, name):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if arr.size != n:
        raise ValueError(f"{name} must have {n} entries, got {arr.size}")
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_dev(t, shape, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the HIP device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _aligned_workspace(nbytes, device):
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


SIDES = {"dirichlet": 0, "neumann": 1}


def _make_desc(nx, ny, nz, hx, hy, hz, scheme, k2=None, k2_z=None, k2_zz=None, gamma=0.0,
               weights=None, precision="fp64", refine_steps=2, max_rhs=1, sides="dirichlet",
               robin=None):
    """cs3d_desc and the host arrays it points to (keep them alive during the call).

    robin: None (Dirichlet z faces) or ((alpha_lo, alpha_hi), (beta_lo, beta_hi)); the k^2
    samples then cover z_{-1}..z_{nz+2} (nz + 4 values)."""
    keep = []
    d = N.Desc()
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.hx, d.hy, d.hz = float(hx), float(hy), float(hz)
    d.scheme = N.SCHEMES[scheme]
    # complex k (absorbing media): real parts in k2..., imaginary parts in k2..._im
    cplx = k2 is not None and np.iscomplexobj(np.asarray(k2))
    nks = nz + (4 if robin is not None else 2)
    fields = [("k2", k2, nks), ("k2_z", k2_z, nks), ("k2_zz", k2_zz, nks), ("weights", weights, nz * 12)]
    if cplx:
        fields = [(nm, None if arr is None else np.real(np.asarray(arr)), n) for nm, arr, n in fields[:3]]
        fields += [(nm + "_im", None if arr is None else np.imag(np.asarray(arr)), nz + 2)
                   for nm, arr in (("k2", k2), ("k2_z", k2_z), ("k2_zz", k2_zz))]
        fields.append(("weights", weights, nz * 12))
    for field, arr, n in fields:
        a, ptr = _host_array(arr, n, field)
        keep.append(a)
        if ptr is not None:
            setattr(d, field, ptr)
    d.gamma = float(gamma)
    d.precision = N.PRECISIONS[precision]
    d.refine_steps = int(refine_steps)
    d.max_rhs = int(max_rhs)
    d.sides = SIDES[sides]
    if robin is not None:
        (a0, a1), (b0, b1) = robin
        d.zfaces = 1
        d.robin_alpha[0], d.robin_alpha[1] = float(a0), float(a1)
        d.robin_beta[0], d.robin_beta[1] = float(b0), float(b1)
    return d, keep


class Plan:
    """A solver plan for one grid, scheme and coefficient set (cs3d_plan_create)."""

    def __init__(self, nx, ny, nz, hx, hy, hz, scheme, k2=None, k2_z=None, k2_zz=None,
                 gamma=0.0, weights=None, precision="fp64", refine_steps=2, max_rhs=1,
                 device="cuda", stream=None, sides="dirichlet", robin=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        # Robin z faces: the z-face nodes are unknowns, a solution holds nz + 2 planes
        self.robin = robin
        # Neumann sides: the side nodes are unknowns, a solution plane has (ny+2) x (nx+2) nodes
        self.sides = sides
        self.scheme = scheme
        self.precision = precision
        # complex k: every field is planar, (nrhs, 2, ...) = real and imaginary parts
        self.complex = k2 is not None and bool(np.iscomplexobj(np.asarray(k2)))
        self.max_rhs = int(max_rhs)
        self.device = torch.device(device)
        d, keep = _make_desc(nx, ny, nz, hx, hy, hz, scheme, k2, k2_z, k2_zz, gamma, weights,
                             precision, refine_steps, max_rhs, sides, robin)
        self._plan = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.check("cs3d_plan_create",
                    N.lib.cs3d_plan_create(ctypes.byref(d), _stream_handle(stream), ctypes.byref(self._plan)))
            self.ws_bytes = N.lib.cs3d_workspace_bytes(self._plan, self.max_rhs)
            self._ws, ptr = _aligned_workspace(self.ws_bytes, self.device)
            N.check("cs3d_set_workspace", N.lib.cs3d_set_workspace(self._plan, ptr, self.ws_bytes))

    # shapes --------------------------------------------------------------
    def _lead(self, nrhs):
        return (nrhs, 2) if self.complex else (nrhs,)

    def closed_shape(self, nrhs):
        return self._lead(nrhs) + (self.nz + 2, self.ny + 2, self.nx + 2)

    def interior_shape(self, nrhs):
        if self.sides == "neumann":
            return self._lead(nrhs) + (self.nz, self.ny + 2, self.nx + 2)
        if self.robin is not None:
            return self._lead(nrhs) + (self.nz + 2, self.ny, self.nx)
        return self._lead(nrhs) + (self.nz, self.ny, self.nx)

    def plane_shape(self, nrhs):
        return self._lead(nrhs) + (self.ny + 2, self.nx + 2)

    def _nrhs(self, t):
        if t.dim() != (5 if self.complex else 4):
            raise ValueError("expected a tensor [nrhs, 2, z, y, x] (complex k: real and imaginary parts)"
                             if self.complex else "expected a 4-D tensor [nrhs, z, y, x]")
        nrhs = t.shape[0]
        if not 1 <= nrhs <= self.max_rhs:
            raise ValueError(f"nrhs must be in [1, {self.max_rhs}], got {nrhs}")
        return nrhs

    # solves --------------------------------------------------------------
    def solve(self, f, g_lo=None, g_hi=None, out=None, stream=None):
        """u = A^{-1}(R_h f - lift(g)) for f on the closed grid; returns the interior u."""
        nrhs = self._nrhs(f)
        _check_dev(f, self.closed_shape(nrhs), "f")
        for g, name in ((g_lo, "g_lo"), (g_hi, "g_hi")):
            if g is not None:
                _check_dev(g, self.plane_shape(nrhs), name)
        if out is None:
            out = torch.empty(self.interior_shape(nrhs), dtype=torch.float64, device=f.device)
        _check_dev(out, self.interior_shape(nrhs), "out")
        st = N.lib.cs3d_solve(self._plan, nrhs, f.data_ptr(),
                              None if g_lo is None else g_lo.data_ptr(),
                              None if g_hi is None else g_hi.data_ptr(),
                              out.data_ptr(), _stream_handle(stream))
        N.check("cs3d_solve", st)
        return out

    def solve_assembled(self, F, out=None, stream=None):
        nrhs = self._nrhs(F)
        _check_dev(F, self.interior_shape(nrhs), "F")
        if out is None:
            out = torch.empty_like(F)
        _check_dev(out, self.interior_shape(nrhs), "out")
        N.check("cs3d_solve_assembled",
                N.lib.cs3d_solve_assembled(self._plan, nrhs, F.data_ptr(), out.data_ptr(),
                                           _stream_handle(stream)))
        return out

    def residual(self, f, u, g_lo=None, g_hi=None, assembled=False, out=None, stream=None):
        """FP64 r = F - A U (F = R_h f, or f itself when assembled)."""
        nrhs = self._nrhs(u)
        _check_dev(u, self.interior_shape(nrhs), "u")
        _check_dev(f, self.interior_shape(nrhs) if assembled else self.closed_shape(nrhs), "f")
        for g, name in ((g_lo, "g_lo"), (g_hi, "g_hi")):
            if g is not None:
                _check_dev(g, self.plane_shape(nrhs), name)
        if out is None:
            out = torch.empty_like(u)
        _check_dev(out, self.interior_shape(nrhs), "out")
        N.check("cs3d_residual",
                N.lib.cs3d_residual(self._plan, nrhs, f.data_ptr(), int(bool(assembled)),
                                    None if g_lo is None else g_lo.data_ptr(),
                                    None if g_hi is None else g_hi.data_ptr(),
                                    u.data_ptr(), out.data_ptr(), _stream_handle(stream)))
        return out

    def stats(self, raise_singular=False):
        s = N.Stats()
        st = N.lib.cs3d_get_stats(self._plan, ctypes.byref(s))
        N.check("cs3d_get_stats", st, allow=() if raise_singular else (N.E_SINGULAR, N.E_NOTCONVERGED))
        return {
            "status": st,
            "min_abs_pivot": s.min_abs_pivot,
            "bad_pivots": int(s.bad_pivots),
            "refine_done": int(s.refine_done),
            "residual_history": [v for v in s.residual_history],
            "last_solve_ms": s.last_solve_ms,
            "stage_ms": [s.stage_ms[k] for k in range(s.stage_count)],
            "timed_solves": int(s.timed_solves),
        }

    def reset_timers(self):
        N.check("cs3d_reset_timers", N.lib.cs3d_reset_timers(self._plan))

    # launch shapes -------------------------------------------------------
    def tuning(self):
        t = N.Tuning()
        N.check("cs3d_get_tuning", N.lib.cs3d_get_tuning(self._plan, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, tuning):
        t = N.Tuning.from_dict({**self.tuning(), **tuning})
        N.check("cs3d_set_tuning", N.lib.cs3d_set_tuning(self._plan, ctypes.byref(t)))

    def autotune(self, f, out=None, reps=2, stream=None):
        """Time the launch-shape candidates on solves of f (cs3d_autotune) and keep the best;
        returns (tuning dict, ms per solve)."""
        nrhs = self._nrhs(f)
        _check_dev(f, self.closed_shape(nrhs), "f")
        if out is None:
            out = torch.empty(self.interior_shape(nrhs), dtype=torch.float64, device=f.device)
        _check_dev(out, self.interior_shape(nrhs), "out")
        t, ms = N.Tuning(), ctypes.c_double()
        N.check("cs3d_autotune",
                N.lib.cs3d_autotune(self._plan, nrhs, f.data_ptr(), None, None, out.data_ptr(),
                                    _stream_handle(stream), int(reps), ctypes.byref(t), ctypes.byref(ms)),
                allow=(N.E_SINGULAR, N.E_NOTCONVERGED))
        return t.as_dict(), ms.value

    def close(self):
        if getattr(self, "_plan", None) and self._plan.value:
            N.lib.cs3d_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_for_problem(p, precision="fp64", refine_steps=2, max_rhs=None, device="cuda", weights=None):
    """Plan matching a workloads.Problem description."""
    robin = getattr(p, "robin", None)
    return Plan(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, p.scheme if weights is None else "weights",
                k2=p.k2, k2_z=p.k2_z if (p.scheme == "helm6" or robin is not None) else None,
                k2_zz=p.k2_zz if p.scheme == "helm6" else None, gamma=p.gamma, weights=weights,
                precision=precision, refine_steps=refine_steps,
                max_rhs=max_rhs or p.nrhs, device=device, sides=getattr(p, "sides", "dirichlet"),
                robin=robin)


class Batch:
    """Many independent problems solved together (cs3d_batch_create): one launch per pass
    over the work items of all members, replayed from a captured HIP graph.

    members: list of dicts with the keyword arguments of Plan (nx, ny, nz, hx, hy, hz,
    scheme, k2, k2_z, k2_zz, gamma); every member takes one right-hand side, FP64."""

    def __init__(self, members, device="cuda", stream=None):
        self.device = torch.device(device)
        self.shapes = [(int(m["nx"]), int(m["ny"]), int(m["nz"])) for m in members]
        n = len(members)
        descs = (N.Desc * n)()
        keep = []
        for i, m in enumerate(members):
            d, k = _make_desc(m["nx"], m["ny"], m["nz"], m["hx"], m["hy"], m["hz"], m["scheme"],
                              m.get("k2"), m.get("k2_z"), m.get("k2_zz"), m.get("gamma", 0.0),
                              None, "fp64", 0, 1)
            descs[i] = d
            keep.append(k)
        self._b = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.check("cs3d_batch_create",
                    N.lib.cs3d_batch_create(n, descs, _stream_handle(stream), ctypes.byref(self._b)))
            self.ws_bytes = N.lib.cs3d_batch_workspace_bytes(self._b)
            self._ws, ptr = _aligned_workspace(self.ws_bytes, self.device)
            N.check("cs3d_batch_set_workspace", N.lib.cs3d_batch_set_workspace(self._b, ptr, self.ws_bytes))

    def __len__(self):
        return len(self.shapes)

    def _ptrs(self, fs, us):
        n = len(self.shapes)
        if len(fs) != n or len(us) != n:
            raise ValueError(f"expected {n} right-hand sides and {n} outputs")
        for i, ((nx, ny, nz), f, u) in enumerate(zip(self.shapes, fs, us)):
            _check_dev(f, (nz + 2, ny + 2, nx + 2), f"f[{i}]")
            _check_dev(u, (nz, ny, nx), f"u[{i}]")
        fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        up = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
        return fp, up

    def outputs(self):
        return [torch.empty((nz, ny, nx), dtype=torch.float64, device=self.device) for nx, ny, nz in self.shapes]

    def solve(self, fs, us=None, stream=None):
        """fs[i]: closed-grid f of member i, shape (nz+2, ny+2, nx+2); returns the interior solutions."""
        if us is None:
            us = self.outputs()
        fp, up = self._ptrs(fs, us)
        N.check("cs3d_batch_solve", N.lib.cs3d_batch_solve(self._b, fp, up, _stream_handle(stream)))
        return us

    def _stats_dict(self, s, st):
        return {"status": st, "min_abs_pivot": s.min_abs_pivot, "bad_pivots": int(s.bad_pivots),
                "last_solve_ms": s.last_solve_ms, "stage_ms": [s.stage_ms[k] for k in range(s.stage_count)]}

    def stats(self):
        s = N.Stats()
        st = N.check("cs3d_batch_get_stats", N.lib.cs3d_batch_get_stats(self._b, ctypes.byref(s)),
                     allow=(N.E_SINGULAR,))
        return self._stats_dict(s, st)

    def member_stats(self, i):
        s = N.Stats()
        st = N.check("cs3d_batch_member_stats", N.lib.cs3d_batch_member_stats(self._b, int(i), ctypes.byref(s)),
                     allow=(N.E_SINGULAR,))
        return self._stats_dict(s, st)

    def tuning(self):
        t = N.Tuning()
        N.check("cs3d_batch_get_tuning", N.lib.cs3d_batch_get_tuning(self._b, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, tuning):
        t = N.Tuning.from_dict({**self.tuning(), **tuning})
        N.check("cs3d_batch_set_tuning", N.lib.cs3d_batch_set_tuning(self._b, ctypes.byref(t)))

    def autotune(self, fs, us=None, reps=2, stream=None):
        if us is None:
            us = self.outputs()
        fp, up = self._ptrs(fs, us)
        t, ms = N.Tuning(), ctypes.c_double()
        N.check("cs3d_batch_autotune",
                N.lib.cs3d_batch_autotune(self._b, fp, up, _stream_handle(stream), int(reps), ctypes.byref(t),
                                          ctypes.byref(ms)),
                allow=(N.E_SINGULAR,))
        return t.as_dict(), ms.value

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            N.lib.cs3d_batch_destroy(self._b)
            self._b = ctypes.c_void_p()
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_member(p):
    """Batch member keywords of a one-right-hand-side workloads.Problem."""
    return dict(nx=p.nx, ny=p.ny, nz=p.nz, hx=p.hx, hy=p.hy, hz=p.hz, scheme=p.scheme, k2=p.k2,
                k2_z=p.k2_z if p.scheme == "helm6" else None, k2_zz=p.k2_zz if p.scheme == "helm6" else None,
                gamma=p.gamma)
