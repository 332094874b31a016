"""Write oracle_tables.json: the oracle's errors on the paper's convergence problems.

    python tests/golden/make_oracle_tables.py [--max-n 512]

Calls only the oracle (``oracle/``) and the problem definitions (``workloads/``, which
hold no solver arithmetic).  The GPU table tests compare the HIP path's errors with these
values for the rows the oracle is too slow to rerun inside a test (N = 500 of Section 5.2.2,
Tables 4-6; N = 256, 512 of the convection-diffusion table of Section 5.2.3).  Sizes up to
512 take about a minute each and 20-25 GB of host memory.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as WL  # noqa: E402

CASES = [("table4_helm2", "helm2", (125, 250, 500)),
         ("table5_helm4", "helm4", (125, 250, 500)),
         ("table6_helm6", "helm6", (125, 250, 500)),
         ("cd_table", "cd4", (64, 128, 256, 512))]


def oracle_errors(scheme, n):
    p = WL.paper_cd(n) if scheme == "cd4" else WL.paper_variable_k(n, scheme)
    res = O.solve(p.scheme, p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma,
                  p.g_lo[0].numpy(), p.g_hi[0].numpy())
    e = O.error_norms(res.U, p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1])
    return {"n": n, "max_err": e["max_err"], "l2_err_U": e["l2_err_U"], "l2_err_u": e["l2_err_u"],
            "min_abs_pivot": res.minpiv}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-n", type=int, default=512)
    args = ap.parse_args()
    out = {"_source": "written by tests/golden/make_oracle_tables.py from the FP64 oracle on the "
                      "paper's convergence problems (Section 5.2.2 variable k, Section 5.2.3 "
                      "convection-diffusion); errors against the exact solution"}
    for key, scheme, sizes in CASES:
        rows = []
        for n in sizes:
            if n > args.max_n:
                continue
            t = time.time()
            rows.append(oracle_errors(scheme, n))
            print(key, rows[-1], f"{time.time() - t:.1f} s", flush=True)
        out[key] = {"scheme": scheme, "rows": rows}
    with open(os.path.join(HERE, "oracle_tables.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
