"""The oracle and the HIP path share nothing, and the product has no CPU fallback.

* no file of the package (Python binding, HIP sources) or of `workloads/` names the
  oracle, and no oracle file names the package or its kernels;
* `bench.py` imports the oracle only inside its CPU-baseline leg;
* importing the package with the library missing raises.
"""
import ast
import os
import pathlib
import subprocess
import sys

ROOT = pathlib.Path(__file__).resolve().parent.parent
PKG = ROOT / "paper_1912_03565_amd"


def _sources(folder, exts):
    return [p for p in folder.rglob("*") if p.suffix in exts and "__pycache__" not in p.parts]


def _imports(path):
    """Top-level module names imported anywhere in a Python file, with the enclosing
    function of each import (None at module level)."""
    tree = ast.parse(path.read_text())
    out = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            f = child.name if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) else func
            if isinstance(child, ast.Import):
                out.extend((a.name.split(".")[0], func) for a in child.names)
            elif isinstance(child, ast.ImportFrom) and child.module and child.level == 0:
                out.append((child.module.split(".")[0], func))
            visit(child, f)

    visit(tree, None)
    return out


def test_package_and_workloads_never_name_the_oracle():
    files = _sources(PKG, {".py", ".hip", ".hpp", ".h", ".cpp"}) + _sources(ROOT / "workloads", {".py"})
    files += list((ROOT / "include").glob("*.h"))
    assert files
    for p in files:
        if p.suffix == ".py":
            assert "oracle" not in {m for m, _ in _imports(p)}, p
        else:
            assert "oracle" not in p.read_text(), p


def test_oracle_never_names_the_package_or_its_kernels():
    files = _sources(ROOT / "oracle", {".py", ".c", ".h"})
    assert files
    for p in files:
        text = p.read_text()
        assert "paper_1912_03565_amd" not in text and "libcs3d" not in text, p
        if p.suffix == ".py":
            mods = {m for m, _ in _imports(p)}
            assert not mods & {"paper_1912_03565_amd", "torch", "ctypes"}, (p, mods)


def test_bench_imports_the_oracle_only_in_its_cpu_baseline():
    where = {f for m, f in _imports(ROOT / "bench.py") if m == "oracle"}
    assert where == {"cpu_baseline"}, where


def test_package_import_fails_without_the_library(tmp_path):
    env = dict(os.environ, CS3D_LIBRARY=str(tmp_path / "missing" / "libcs3d.so"))
    r = subprocess.run([sys.executable, "-c", "import paper_1912_03565_amd"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "libcs3d" in r.stderr or "missing" in r.stderr, r.stderr[-2000:]
