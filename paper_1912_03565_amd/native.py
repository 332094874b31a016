"""ctypes binding of include/cs3d.h: argument marshalling only.

Every step of the solve runs in libcs3d.so (HIP kernels for gfx950).  PyTorch
supplies device memory and the HIP stream; it never touches the arithmetic.
If the library has not been built this module raises on import: there is no
fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# CS3D_LIBRARY selects another build of the same library (e.g. an autotuned or
# instrumented one); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("CS3D_LIBRARY") or os.path.join(HERE, "libcs3d.so")

OK = 0
E_INVAL = 1
E_NOMEM = 2
E_DEVICE = 3
E_SINGULAR = 4
E_NOTCONVERGED = 5
E_UNSUPPORTED = 6
E_WORKSPACE = 7
E_TOO_LARGE = 8

SCHEMES = {"helm2": 2, "helm4": 4, "helm6": 6, "cd4": 14, "weights": 99}
PRECISIONS = {"fp64": 0, "mixed": 1, "mixed_fp32": 1}


class Desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
        ("scheme", ctypes.c_int),
        ("k2", ctypes.POINTER(ctypes.c_double)),
        ("k2_z", ctypes.POINTER(ctypes.c_double)),
        ("k2_zz", ctypes.POINTER(ctypes.c_double)),
        ("gamma", ctypes.c_double),
        ("weights", ctypes.POINTER(ctypes.c_double)),
        ("precision", ctypes.c_int),
        ("refine_steps", ctypes.c_int),
        ("max_rhs", ctypes.c_int),
        ("k2_im", ctypes.POINTER(ctypes.c_double)),
        ("k2_z_im", ctypes.POINTER(ctypes.c_double)),
        ("k2_zz_im", ctypes.POINTER(ctypes.c_double)),
        ("sides", ctypes.c_int),
        ("zfaces", ctypes.c_int),
        ("robin_alpha", ctypes.c_double * 2),
        ("robin_beta", ctypes.c_double * 2),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("min_abs_pivot", ctypes.c_double),
        ("bad_pivots", ctypes.c_int64),
        ("refine_done", ctypes.c_int),
        ("residual_history", ctypes.c_double * 8),
        ("last_solve_ms", ctypes.c_double),
        ("stage_ms", ctypes.c_double * 8),
        ("stage_count", ctypes.c_int),
        ("timed_solves", ctypes.c_int),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("zchunk", ctypes.c_int), ("xpersist", ctypes.c_int), ("ywpl", ctypes.c_int),
        ("order", ctypes.c_int), ("graph", ctypes.c_int), ("yrhs", ctypes.c_int),
        ("xwpl", ctypes.c_int), ("pack", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        for k, _ in cls._fields_:
            setattr(t, k, int(d[k]))
        return t


EXPORTS = [
    "cs3d_plan_create", "cs3d_plan_destroy", "cs3d_workspace_bytes", "cs3d_set_workspace",
    "cs3d_solve", "cs3d_solve_static", "cs3d_solve_assembled", "cs3d_residual", "cs3d_get_stats",
    "cs3d_batch_create", "cs3d_batch_workspace_bytes", "cs3d_batch_set_workspace",
    "cs3d_batch_solve", "cs3d_batch_get_stats", "cs3d_batch_destroy", "cs3d_status_str",
    "cs3d_version", "cs3d_reset_timers", "cs3d_get_tuning", "cs3d_set_tuning", "cs3d_autotune",
    "cs3d_batch_member_stats", "cs3d_batch_get_tuning", "cs3d_batch_set_tuning", "cs3d_batch_autotune",
]


class CS3DError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed: {msg} (status {status})")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python paper_1912_03565_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, sz, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p
    sig = {
        "cs3d_plan_create": (i, [ctypes.POINTER(Desc), vp, ctypes.POINTER(vp)]),
        "cs3d_plan_destroy": (i, [vp]),
        "cs3d_workspace_bytes": (sz, [vp, i]),
        "cs3d_set_workspace": (i, [vp, vp, sz]),
        "cs3d_solve": (i, [vp, i, dp, dp, dp, dp, vp]),
        "cs3d_solve_static": (i, [vp, i, dp, dp, dp, dp, vp]),
        "cs3d_solve_assembled": (i, [vp, i, dp, dp, vp]),
        "cs3d_residual": (i, [vp, i, dp, i, dp, dp, dp, dp, vp]),
        "cs3d_get_stats": (i, [vp, ctypes.POINTER(Stats)]),
        "cs3d_reset_timers": (i, [vp]),
        "cs3d_batch_create": (i, [i, ctypes.POINTER(Desc), vp, ctypes.POINTER(vp)]),
        "cs3d_batch_workspace_bytes": (sz, [vp]),
        "cs3d_batch_set_workspace": (i, [vp, vp, sz]),
        "cs3d_batch_solve": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]),
        "cs3d_batch_get_stats": (i, [vp, ctypes.POINTER(Stats)]),
        "cs3d_batch_destroy": (i, [vp]),
        "cs3d_batch_member_stats": (i, [vp, i, ctypes.POINTER(Stats)]),
        "cs3d_batch_get_tuning": (i, [vp, ctypes.POINTER(Tuning)]),
        "cs3d_batch_set_tuning": (i, [vp, ctypes.POINTER(Tuning)]),
        "cs3d_batch_autotune": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, i,
                                    ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double)]),
        "cs3d_get_tuning": (i, [vp, ctypes.POINTER(Tuning)]),
        "cs3d_set_tuning": (i, [vp, ctypes.POINTER(Tuning)]),
        "cs3d_autotune": (i, [vp, i, dp, dp, dp, dp, vp, i, ctypes.POINTER(Tuning),
                              ctypes.POINTER(ctypes.c_double)]),
        "cs3d_status_str": (ctypes.c_char_p, [i]),
        "cs3d_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def status_str(st):
    return lib.cs3d_status_str(st).decode()


def check(fn, st, allow=()):
    if st != OK and st not in allow:
        raise CS3DError(fn, st, status_str(st))
    return st
