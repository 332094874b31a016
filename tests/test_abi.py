"""Host-side checks of the C ABI (no GPU needed: nothing here launches a kernel).

* the library loads and exports every entry point declared in include/cs3d.h,
* argument validation rejects bad descriptions before touching the device,
* the ctypes mirrors of the ABI structs match the header (names, offsets, sizes).
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def N():
    from paper_1912_03565_amd import native
    return native


def test_every_declared_symbol_is_exported(N):
    with open(os.path.join(ROOT, "include", "cs3d.h")) as fh:
        hdr = fh.read()
    declared = set(re.findall(r"\b(cs3d_[a-z_]+)\s*\(", hdr))
    assert len(declared) >= 16
    for name in declared:
        assert hasattr(N.lib, name), name
    assert set(N.EXPORTS) <= declared


def test_status_strings(N):
    for st in range(8):
        assert len(N.status_str(st)) > 0
    assert N.lib.cs3d_version().decode().startswith("cs3d")


def _desc(N, **kw):
    d = N.Desc()
    d.nx, d.ny, d.nz = kw.get("n", (63, 63, 63))
    d.hx, d.hy, d.hz = kw.get("h", (1 / 64, 1 / 64, 1 / 64))
    d.scheme = N.SCHEMES[kw.get("scheme", "helm6")]
    d.max_rhs = kw.get("max_rhs", 1)
    d.precision = 0
    d.refine_steps = kw.get("refine", 0)
    arr = np.ones(d.nz + 2)
    keep = [arr]
    if kw.get("k", True):
        p = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.k2 = d.k2_z = d.k2_zz = p
    d._keep = keep
    return d


@pytest.mark.parametrize("case", ["nx0", "nx_big", "h_neg", "h6_unequal", "h6_small", "no_k",
                                  "bad_scheme", "max_rhs0", "refine_neg", "weights_missing"])
def test_plan_create_rejects_bad_descriptions(N, case):
    kw = {}
    if case == "nx0":
        kw["n"] = (0, 5, 5)
    elif case == "nx_big":
        kw["n"] = (1025, 5, 5)
    elif case == "h_neg":
        kw["h"] = (-0.1, 0.1, 0.1)
    elif case == "h6_unequal":
        kw["h"] = (0.1, 0.1, 0.2)
    elif case == "h6_small":
        kw["n"] = (3, 8, 8)
    elif case == "no_k":
        kw["k"] = False
    elif case == "max_rhs0":
        kw["max_rhs"] = 0
    elif case == "refine_neg":
        kw["refine"] = -1
    d = _desc(N, **kw)
    if case == "bad_scheme":
        d.scheme = 7
    if case == "weights_missing":
        d.scheme = N.SCHEMES["weights"]
    plan = ctypes.c_void_p()
    st = N.lib.cs3d_plan_create(ctypes.byref(d), None, ctypes.byref(plan))
    assert st == N.E_INVAL
    assert not plan.value


def test_null_arguments_are_rejected(N):
    assert N.lib.cs3d_plan_create(None, None, None) == N.E_INVAL
    assert N.lib.cs3d_solve(None, 1, None, None, None, None, None) == N.E_INVAL
    assert N.lib.cs3d_solve_assembled(None, 1, None, None, None) == N.E_INVAL
    assert N.lib.cs3d_set_workspace(None, None, 0) == N.E_INVAL
    assert N.lib.cs3d_workspace_bytes(None, 1) == 0
    assert N.lib.cs3d_plan_destroy(None) == N.OK
    assert N.lib.cs3d_batch_destroy(None) == N.OK
    assert N.lib.cs3d_get_stats(None, None) == N.E_INVAL
    assert N.lib.cs3d_get_tuning(None, None) == N.E_INVAL
    assert N.lib.cs3d_set_tuning(None, None) == N.E_INVAL
    assert N.lib.cs3d_autotune(None, 1, None, None, None, None, None, 1, None, None) == N.E_INVAL
    assert N.lib.cs3d_batch_create(0, None, None, None) == N.E_INVAL
    assert N.lib.cs3d_batch_solve(None, None, None, None) == N.E_INVAL
    assert N.lib.cs3d_batch_get_stats(None, None) == N.E_INVAL
    assert N.lib.cs3d_batch_member_stats(None, 0, None) == N.E_INVAL
    assert N.lib.cs3d_batch_get_tuning(None, None) == N.E_INVAL
    assert N.lib.cs3d_batch_set_tuning(None, None) == N.E_INVAL
    assert N.lib.cs3d_batch_autotune(None, None, None, None, 1, None, None) == N.E_INVAL
    assert N.lib.cs3d_batch_workspace_bytes(None) == 0


@pytest.mark.parametrize("case", ["weights", "mixed", "bad_member"])
def test_batch_create_rejects_members(N, case):
    descs = (N.Desc * 2)()
    keep = []
    for i in range(2):
        d = _desc(N, n=(63, 63, 63))
        keep.append(d._keep)
        descs[i] = d
    if case == "weights":
        descs[1].scheme = N.SCHEMES["weights"]
        want = N.E_INVAL
    elif case == "mixed":
        descs[0].precision = N.PRECISIONS["mixed"]
        want = N.E_UNSUPPORTED
    else:
        descs[1].nx = 0
        want = N.E_INVAL
    b = ctypes.c_void_p()
    assert N.lib.cs3d_batch_create(2, descs, None, ctypes.byref(b)) == want
    assert not b.value


def test_tuning_cache_store_and_load(tmp_path, monkeypatch):
    from paper_1912_03565_amd import tuning
    path = str(tmp_path / "sub" / "tune.json")
    monkeypatch.setenv("CS3D_TUNE_CACHE", path)
    assert tuning.cache_path() == path
    assert tuning.load() == {}
    tuning.store("dev|plan|63x63x63|helm6|fp64|rhs1", {"tuning": {"zchunk": 16}, "ms": 1.5})
    tuning.store("dev|batch|n64|abc", {"tuning": {"zchunk": 64}, "ms": 9.0})
    data = tuning.load()
    assert data["dev|plan|63x63x63|helm6|fp64|rhs1"]["tuning"]["zchunk"] == 16
    assert len(data) == 2
    with open(path, "w") as fh:
        fh.write("{not json")
    assert tuning.load() == {}  # a damaged cache is ignored, not fatal
    monkeypatch.setenv("CS3D_AUTOTUNE", "0")
    assert not tuning.enabled()


@pytest.mark.parametrize("case", ["cd4", "mixed", "helm6_missing_im", "batch"])
def test_complex_k_validation(N, case):
    d = _desc(N, n=(63, 63, 63))
    im = np.full(d.nz + 2, 0.5)
    d._keep.append(im)
    ptr = im.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.k2_im = ptr
    if case != "helm6_missing_im":
        d.k2_z_im = d.k2_zz_im = ptr
    want = N.E_UNSUPPORTED
    if case == "cd4":
        d.scheme = N.SCHEMES["cd4"]
    elif case == "mixed":
        d.precision = N.PRECISIONS["mixed"]
    elif case == "helm6_missing_im":
        want = N.E_INVAL
    if case == "batch":
        descs = (N.Desc * 1)(d)
        b = ctypes.c_void_p()
        assert N.lib.cs3d_batch_create(1, descs, None, ctypes.byref(b)) == want
        return
    plan = ctypes.c_void_p()
    assert N.lib.cs3d_plan_create(ctypes.byref(d), None, ctypes.byref(plan)) == want
    assert not plan.value


@pytest.mark.parametrize("case", ["mixed", "complex", "too_long_x", "too_long_y", "bad_value", "batch"])
def test_neumann_sides_validation(N, case):
    """Neumann sides: FP64 plans with real k and lines of at most 1023 nodes."""
    d = _desc(N, n=(63, 63, 63))
    d.sides = 1
    want = N.E_UNSUPPORTED
    if case == "mixed":
        d.precision = N.PRECISIONS["mixed"]
    elif case == "complex":
        im = np.full(d.nz + 2, 0.5)
        d._keep.append(im)
        d.k2_im = d.k2_z_im = d.k2_zz_im = im.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    elif case == "too_long_x":
        d.nx = 1022
        want = N.E_INVAL
    elif case == "too_long_y":
        d.ny = 1022
        want = N.E_INVAL
    elif case == "bad_value":
        d.sides = 2
        want = N.E_INVAL
    if case == "batch":
        descs = (N.Desc * 1)()
        descs[0] = d
        b = ctypes.c_void_p()
        assert N.lib.cs3d_batch_create(1, descs, None, ctypes.byref(b)) == want
        assert not b.value
        return
    plan = ctypes.c_void_p()
    assert N.lib.cs3d_plan_create(ctypes.byref(d), None, ctypes.byref(plan)) == want
    assert not plan.value


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of cs3d_desc, cs3d_stats and cs3d_tuning (native.py) have the
    field names, offsets and sizes the C compiler gives the structs of include/cs3d.h
    (a host program built with gcc prints them)."""
    import ctypes
    import shutil
    import subprocess

    from paper_1912_03565_amd import native as NM

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    structs = {"cs3d_desc": NM.Desc, "cs3d_stats": NM.Stats, "cs3d_tuning": NM.Tuning}
    lines = ['#include <stdio.h>', '#include "cs3d.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu %zu\\n", offsetof({cname}, {fname}), '
                         f"sizeof((({cname}*)0)->{fname}));")
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run([gcc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        parts = ln.split()
        got[(parts[0], parts[1])] = tuple(int(v) for v in parts[2:])
    for cname, cls in structs.items():
        assert got[(cname, "size")] == (ctypes.sizeof(cls),), cname
        for fname, _ in cls._fields_:
            f = getattr(cls, fname)
            assert got[(cname, fname)] == (f.offset, f.size), (cname, fname, got[(cname, fname)], f.offset, f.size)
    # every member the header declares is mirrored, in order
    hdr = open(os.path.join(inc, "cs3d.h")).read()
    hdr = re.sub(r"/\*.*?\*/", " ", hdr, flags=re.S)
    hdr = re.sub(r"//[^\n]*", " ", hdr)
    for cname, cls in structs.items():
        body = re.search(r"typedef\s+struct\s*\{([^}]*)\}\s*" + cname + r"\s*;", hdr).group(1)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            first, *rest = decl.split(",")
            names.append(re.sub(r"\[.*?\]", "", first).replace("*", " ").split()[-1])
            names += [re.sub(r"\[.*?\]", "", r).replace("*", " ").split()[-1] for r in rest]
        assert names == [f for f, _ in cls._fields_], (cname, names)
