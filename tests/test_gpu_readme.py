"""The Python example of README.md runs as written and solves its system: the FP64
27-point residual of the returned u (the library's residual pass, a kernel separate from
the solve) is at rounding level relative to the right-hand side."""
import os
import re

import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_python_example():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    text = open(os.path.join(ROOT, "README.md")).read()
    code = re.search(r"```python\n(.*?)```", text, re.S).group(1)
    ns = {}
    exec(compile(code, "README.md example", "exec"), ns)
    plan, f, u = ns["plan"], ns["f"], ns["u"]
    n = plan.nx
    assert tuple(u.shape) == (1, n, n, n) and torch.isfinite(u).all()
    r = plan.residual(f, u)
    rhs = plan.residual(f, torch.zeros_like(u))  # F - A 0 = F
    rel = (r.norm() / rhs.norm()).item()
    print(f"README example: {n}^3, relative residual {rel:.2e}, "
          f"min pivot {plan.stats()['min_abs_pivot']:.3e}", flush=True)
    assert rel < 1e-12, rel
    plan.close()
