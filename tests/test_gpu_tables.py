"""The paper's convergence tables reproduced by the HIP path (FP64), through the C ABI.

Section 5.2.2, Tables 4 and 5 (2nd and 4th order, variable k(z) = a - b sin(cz)) and the
convection-diffusion table of Section 5.2.3: max-error and L2-error of every printed row
to all printed digits.  Table 6 (6th order): the paper does not define its discrete
derivatives of f (reading R11), so its rows are matched in magnitude, the HIP path's
errors equal the oracle's, and the observed order between the two printed sizes is at
least six (the printed rows give 6.0; this discrete right-hand side gives 7.0 there, its
N = 125 error carrying a larger h^7 part).
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def cs3d():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_03565_amd as m
    return m


@pytest.fixture(scope="module")
def tables(golden_dir):
    with open(os.path.join(golden_dir, "paper_tables.json")) as fh:
        return json.load(fh)


def _printed_match(ours, printed, digits=8):
    """|ours - printed| within 0.75 unit of the last printed digit."""
    e = math.floor(math.log10(abs(printed)))
    return abs(ours - printed) <= 0.75 * 10.0 ** (e - (digits - 1))


def _gpu(cs3d, p):
    plan = cs3d.plan_for_problem(p, device=DEV)
    gl = None if p.g_lo is None else p.g_lo.to(DEV)
    gh = None if p.g_hi is None else p.g_hi.to(DEV)
    u = plan.solve(p.f.to(DEV), gl, gh).cpu().numpy()[0]
    st = plan.stats()
    plan.close()
    assert st["bad_pivots"] == 0
    return u


@pytest.mark.parametrize("scheme,key", [("helm2", "table4_helm2"), ("helm4", "table5_helm4")])
@pytest.mark.parametrize("row", [0, 1])
def test_tables_4_5_all_digits(cs3d, tables, scheme, key, row):
    ref = tables[key]["rows"][row]
    p = WL.paper_variable_k(ref["n"], scheme)
    u = _gpu(cs3d, p)
    e = O.error_norms(u, p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1])
    print(f"{key} N={ref['n']}: max {e['max_err']:.8e} (printed {ref['max_err']:.8e}), "
          f"l2 {e['l2_err_U']:.8e} (printed {ref['l2_err']:.8e})", flush=True)
    assert _printed_match(e["max_err"], ref["max_err"])
    assert _printed_match(e["l2_err_U"], ref["l2_err"])


@pytest.mark.parametrize("row", [0, 1])
def test_cd_table_all_digits(cs3d, tables, row):
    ref = tables["cd_table"]["rows"][row]
    p = WL.paper_cd(ref["n"])
    u = _gpu(cs3d, p)
    e = O.error_norms(u, p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1])
    print(f"cd N={ref['n']}: max {e['max_err']:.8e} (printed {ref['max_err']:.8e}), "
          f"l2 {e['l2_err_u']:.8e} (printed {ref['l2_err']:.8e})", flush=True)
    assert _printed_match(e["max_err"], ref["max_err"])
    assert _printed_match(e["l2_err_u"], ref["l2_err"])


def test_table6_magnitude_order_and_oracle(cs3d, tables):
    errs = []
    for ref in tables["table6_helm6"]["rows"]:
        p = WL.paper_variable_k(ref["n"], "helm6")
        u = _gpu(cs3d, p)
        ue = p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1]
        e = O.error_norms(u, ue)
        res = O.solve(p.scheme, p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma,
                      None if p.g_lo is None else p.g_lo[0].numpy(),
                      None if p.g_hi is None else p.g_hi[0].numpy())
        eo = O.error_norms(res.U, ue)
        print(f"table6 N={ref['n']}: max {e['max_err']:.6e} (oracle {eo['max_err']:.6e}, printed "
              f"{ref['max_err']:.6e})", flush=True)
        assert abs(e["max_err"] - eo["max_err"]) <= 1e-12
        assert ref["max_err"] / 3 <= e["max_err"] <= 3 * ref["max_err"]
        errs.append((ref["n"], e["max_err"]))
    (n1, e1), (n2, e2) = errs
    order = math.log(e1 / e2) / math.log((n2 + 1) / (n1 + 1))
    print(f"table6 observed order {order:.2f}", flush=True)
    assert order >= 5.5
