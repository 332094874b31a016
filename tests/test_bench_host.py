"""Host-side helpers of bench.py (no GPU).

- The hash that ties the committed HBM-traffic counter runs to the kernel code ignores
  comments and layout and follows every change of the code.
- The algorithmic bytes per pass add up to the design's 88 + 8/nrhs bytes per unknown
  and right-hand side (five passes, c' written once per plan).
"""
import importlib.util
import os
import shutil

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_text_drops_comments_keeps_literals():
    b = _bench()
    src = 'int a = 1;  // note\n/* block\n comment */ const char* s = "x // y /* z */";\nchar q = \'"\';'
    assert b._code_text(src) == 'int a = 1; const char* s = "x // y /* z */"; char q = \'"\';'


def test_source_hash_follows_code_not_comments(tmp_path):
    b = _bench()
    csrc = tmp_path / "paper_1912_03565_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_1912_03565_amd", "csrc"), csrc)
    b.ROOT = str(tmp_path)
    h0 = b.kernel_source_hash()
    k = csrc / "kernels.hpp"
    text = k.read_text()
    k.write_text("// an added comment line\n" + text.replace("\n", "\n\n", 3))
    assert b.kernel_source_hash() == h0
    assert "kBlockY = 256" in text
    k.write_text(text.replace("kBlockY = 256", "kBlockY = 128"))
    assert b.kernel_source_hash() != h0


def test_stage_bytes_design_total():
    b = _bench()
    n, nrhs = 1023, 4
    total = sum(b.stage_bytes(n, n, n, nrhs))
    closed = (n + 2) ** 3
    n3 = n ** 3
    # K0 reads the closed grid: 8 (n+2)^3 instead of 8 n^3
    expect = nrhs * (88 * n3 + 8 * (closed - n3)) + 8 * n3
    assert total == expect
