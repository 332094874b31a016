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


class Plan:
    """A solver plan for one grid, scheme and coefficient set (cs3d_plan_create)."""

    def __init__(self, nx, ny, nz, hx, hy, hz, scheme, k2=None, k2_z=None, k2_zz=None,
                 gamma=0.0, weights=None, precision="fp64", refine_steps=2, max_rhs=1,
                 device="cuda", stream=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.scheme = scheme
        self.max_rhs = int(max_rhs)
        self.device = torch.device(device)
        keep = []
        d = N.Desc()
        d.nx, d.ny, d.nz = self.nx, self.ny, self.nz
        d.hx, d.hy, d.hz = float(hx), float(hy), float(hz)
        d.scheme = N.SCHEMES[scheme]
        for field, arr, n in (("k2", k2, nz + 2), ("k2_z", k2_z, nz + 2), ("k2_zz", k2_zz, nz + 2),
                              ("weights", weights, nz * 12)):
            a, p = _host_array(arr, n, field)
            keep.append(a)
            if p is not None:
                setattr(d, field, p)
        d.gamma = float(gamma)
        d.precision = N.PRECISIONS[precision]
        d.refine_steps = int(refine_steps)
        d.max_rhs = self.max_rhs
        self._plan = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.check("cs3d_plan_create",
                    N.lib.cs3d_plan_create(ctypes.byref(d), _stream_handle(stream), ctypes.byref(self._plan)))
            self.ws_bytes = N.lib.cs3d_workspace_bytes(self._plan, self.max_rhs)
            self._ws, ptr = _aligned_workspace(self.ws_bytes, self.device)
            N.check("cs3d_set_workspace", N.lib.cs3d_set_workspace(self._plan, ptr, self.ws_bytes))

    # shapes --------------------------------------------------------------
    def closed_shape(self, nrhs):
        return (nrhs, self.nz + 2, self.ny + 2, self.nx + 2)

    def interior_shape(self, nrhs):
        return (nrhs, self.nz, self.ny, self.nx)

    def plane_shape(self, nrhs):
        return (nrhs, self.ny + 2, self.nx + 2)

    def _nrhs(self, t):
        if t.dim() != 4:
            raise ValueError("expected a 4-D tensor [nrhs, z, y, x]")
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
    return Plan(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz, p.scheme if weights is None else "weights",
                k2=p.k2, k2_z=p.k2_z if p.scheme == "helm6" else None,
                k2_zz=p.k2_zz if p.scheme == "helm6" else None, gamma=p.gamma, weights=weights,
                precision=precision, refine_steps=refine_steps,
                max_rhs=max_rhs or p.nrhs, device=device)
