"""Pins of the CPU oracle against things other than itself.

* printed numbers of the paper (Tables 4-5 and the convection-diffusion table to
  all printed digits; Table 6 in magnitude and order),
* the PDE itself (truncation order of every weight table + RHS operator applied
  to analytic solutions),
* brute force (assembled 27-diagonal matrix + dense LU) on tiny grids,
* closed forms (orthonormal sine matrix, DST eigenvectors of the 9-point blocks,
  constant-k Toeplitz systems solved by a 3-D sine transform),
* a library banded solver for the Thomas recurrence,
* discrete manufactured solutions at any size.

A plausible slip in the oracle (a dropped term, a wrong sign or index, a swapped
x/y weight) changes at least one of these.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import paper_problems as PP
import workloads as WL


def _np(t):
    return None if t is None else t.numpy()


def _solve_problem(p, r=0):
    f = p.f[r].numpy()
    gl = None if p.g_lo is None else p.g_lo[r].numpy()
    gh = None if p.g_hi is None else p.g_hi[r].numpy()
    res = O.solve(p.scheme, f, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma, gl, gh)
    return res, gl, gh


def _printed_match(ours, printed, digits=8):
    """|ours - printed| within 0.75 unit of the last printed digit."""
    e = math.floor(math.log10(abs(printed)))
    ulp = 10.0 ** (e - (digits - 1))
    return abs(ours - printed) <= 0.75 * ulp


@pytest.fixture(scope="module")
def tables(golden_dir):
    with open(os.path.join(golden_dir, "paper_tables.json")) as fh:
        return json.load(fh)


# ---------------------------------------------------------------------------
# P1/P2: the paper's printed tables
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme,key", [("helm2", "table4_helm2"), ("helm4", "table5_helm4")])
@pytest.mark.parametrize("row", [0, 1])
def test_paper_tables_2nd_4th_order_all_digits(tables, scheme, key, row):
    ref = tables[key]["rows"][row]
    p = WL.paper_variable_k(ref["n"], scheme)
    res, _, _ = _solve_problem(p)
    ue = p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1]
    e = O.error_norms(res.U, ue)
    assert _printed_match(e["max_err"], ref["max_err"]), (e, ref)
    assert _printed_match(e["l2_err_U"], ref["l2_err"]), (e, ref)
    assert res.bad == 0


@pytest.mark.parametrize("row", [0, 1])
def test_paper_cd_table_all_digits(tables, row):
    ref = tables["cd_table"]["rows"][row]
    p = WL.paper_cd(ref["n"])
    res, _, _ = _solve_problem(p)
    ue = p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1]
    e = O.error_norms(res.U, ue)
    assert _printed_match(e["max_err"], ref["max_err"]), (e, ref)
    assert _printed_match(e["l2_err_u"], ref["l2_err"]), (e, ref)


def test_paper_table6_magnitude(tables):
    ref = tables["table6_helm6"]["rows"][0]
    p = WL.paper_variable_k(ref["n"], "helm6")
    res, gl, gh = _solve_problem(p)
    ue = p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1]
    e = O.error_norms(res.U, ue, res.W, res.F, gl, gh)
    # same magnitude as the printed 2.19e-6 (the paper's discrete f-derivatives are unspecified)
    assert 1e-6 <= e["max_err"] <= 6e-6, e
    assert 1e-6 <= e["l2_err_U"] <= 6e-6, e
    # direct-solve residual at the level the paper reports (~1e-13 .. 1e-12 absolute)
    assert e["l2_res"] < 2e-11, e


# ---------------------------------------------------------------------------
# The largest printed rows: 500^3 of Tables 4-6 and 256^3 / 512^3 of the
# convection-diffusion table.  A 3-D oracle solve at these sizes takes 20-40 s and
# about 20 GB, so its errors are stored in tests/golden/oracle_tables.json (written by
# tests/golden/make_oracle_tables.py, which calls only the oracle) and pinned here.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme,key", [("helm2", "table4_helm2"), ("helm4", "table5_helm4"),
                                        ("cd4", "cd_table")])
def test_paper_tables_by_single_mode_reduction(tables, golden_dir, scheme, key):
    """Tables 4 and 5 (125^3 .. 500^3) and the convection-diffusion table (64^3 .. 512^3)
    from the one-mode reduction (extended precision, no transforms): every printed digit
    within 0.75 of the last one, plus the FP64 bound cond * eps * max|u| of the excited
    mode.  That bound is below one printed unit up to 128^3 (125^3) and reaches 6.5e-13
    at 500^3 and 4.2e-12 at 512^3 (mode condition numbers 2.9e3 and 9.5e3), where the
    printed eighth digit lies below what any FP64 solve resolves.  The stored errors of
    the 3-D FP64 oracle agree with the exact discrete ones within the same bound."""
    stored = {r["n"]: r for r in PP.oracle_tables(golden_dir)[key]["rows"]}
    l2key = "l2_err_u" if scheme == "cd4" else "l2_err_U"  # reading R12
    for ref in tables[key]["rows"]:
        n = ref["n"]
        m = PP.single_mode(scheme, n)
        b = PP.fp64_bound(m)
        assert abs(m["max_err"] - ref["max_err"]) <= PP.printed_bar(ref["max_err"], b["max_err"]), (n, m, ref)
        assert abs(m[l2key] - ref["l2_err"]) <= PP.printed_bar(ref["l2_err"], b["l2"]), (n, m, ref)
        o = stored[n]
        assert abs(o["max_err"] - m["max_err"]) <= b["max_err"], (n, o, m)
        assert abs(o[l2key] - m[l2key]) <= b["l2"], (n, o, m)


def test_stored_oracle_tables_match_a_fresh_oracle_run(golden_dir):
    """The stored rows of the two smallest sizes agree with the oracle run now."""
    stored = PP.oracle_tables(golden_dir)
    for key, scheme in (("table5_helm4", "helm4"), ("table6_helm6", "helm6"), ("cd_table", "cd4")):
        ref = stored[key]["rows"][0]
        p = WL.paper_cd(ref["n"]) if scheme == "cd4" else WL.paper_variable_k(ref["n"], scheme)
        res, _, _ = _solve_problem(p)
        e = O.error_norms(res.U, p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1])
        assert e["max_err"] == pytest.approx(ref["max_err"], rel=1e-9, abs=1e-14)
        assert e["l2_err_U"] == pytest.approx(ref["l2_err_U"], rel=1e-9, abs=1e-14)


def test_table6_order_from_250_to_500(tables, golden_dir):
    """Table 6 (Section 5.2.2): the paper's ratios are 62.6 and 63.3, order 6.0 on both
    intervals.  The oracle's ratio is 122 from 125 to 250 (its N = 125 maximum sits on the
    first interior layer, where the one-sided fourth differences of reading R10 leave an
    error that decays faster than h^6) and 63.9 from 250 to 500: order 6.0 once the h^6
    term dominates.  Magnitudes at 250 and 500 within 15 % of the printed ones."""
    rows = {r["n"]: r for r in PP.oracle_tables(golden_dir)["table6_helm6"]["rows"]}
    printed = {r["n"]: r for r in tables["table6_helm6"]["rows"]}
    order = math.log(rows[250]["max_err"] / rows[500]["max_err"]) / math.log(501 / 251)
    assert 5.8 <= order <= 6.2, order
    for n in (250, 500):
        assert 0.8 <= rows[n]["max_err"] / printed[n]["max_err"] <= 1.2, (n, rows[n], printed[n])
    order_first = math.log(rows[125]["max_err"] / rows[250]["max_err"]) / math.log(251 / 126)
    assert order_first > order


def test_helm6_observed_order_six_under_h_halving():
    prof = WL.problems.KProfile(lambda z: 4.0 + np.sin(2 * np.pi * z),
                                lambda z: 2 * np.pi * np.cos(2 * np.pi * z),
                                lambda z: -4 * np.pi ** 2 * np.sin(2 * np.pi * z))
    errs = []
    for n in (15, 31, 63):
        p = WL.manufactured_sin3(n, n, n, "helm6", prof)
        res, _, _ = _solve_problem(p)
        errs.append(np.abs(res.U - p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1]).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 5.5 < orders[-1] < 6.8, (errs, orders)


@pytest.mark.parametrize("scheme,lo,hi", [("helm4", 3.7, 4.4), ("cd4", 3.7, 4.4)])
def test_fourth_order_observed_order_under_h_halving(scheme, lo, hi):
    prof = WL.problems.KProfile(lambda z: 4.0 + np.sin(2 * np.pi * z),
                                lambda z: 2 * np.pi * np.cos(2 * np.pi * z),
                                lambda z: -4 * np.pi ** 2 * np.sin(2 * np.pi * z))
    errs = []
    for n in (15, 31, 63):
        if scheme == "cd4":
            # u* with gamma u_z forcing: f = lap u* + gamma u*_z
            p = WL.manufactured_sin3(n, n, n, "cd4", WL.problems.k_const(0.0))
            gamma = -20.0
            z = p.hz * np.arange(n + 2)
            x = p.hx * np.arange(n + 2)
            y = p.hy * np.arange(n + 2)
            uz = 3 * np.pi * np.cos(3 * np.pi * z)
            extra = gamma * uz[:, None, None] * np.sin(2 * np.pi * y)[None, :, None] * np.sin(np.pi * x)[None, None, :]
            f = p.f[0].numpy() + extra
            res = O.solve("cd4", f, p.hx, p.hy, p.hz, gamma=gamma)
        else:
            p = WL.manufactured_sin3(n, n, n, scheme, prof, box=(1.0, 1.5, 0.8))
            res, _, _ = _solve_problem(p)
        errs.append(np.abs(res.U - p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1]).max())
    order = math.log2(errs[1] / errs[2])
    assert lo < order < hi, (errs, order)


# ---------------------------------------------------------------------------
# P3: truncation order of every weight table + RHS against the PDE itself
# ---------------------------------------------------------------------------
def _trunc_residual(scheme, h, ratios=(1.0, 1.0, 1.0), gamma=0.0, n=10, centre=(0.31, -0.17, 0.23)):
    hx, hy, hz = h * ratios[0], h * ratios[1], h * ratios[2]
    # the grid is centred on a fixed physical point, so the residual there is C h^p + ...
    ic = (n + 1) // 2
    x = centre[0] + hx * (np.arange(n + 2) - ic)
    y = centre[1] + hy * (np.arange(n + 2) - ic)
    z = centre[2] + hz * (np.arange(n + 2) - ic)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    # analytic u with all derivatives non-trivial
    ph = 1.3 * X - 0.8 * Y + 1.1 * Z
    u = np.exp(0.4 * X + 0.2 * Z) * np.sin(ph) + np.cos(0.7 * Y + 0.5 * Z)
    # derivatives of u
    e = np.exp(0.4 * X + 0.2 * Z)
    s, c = np.sin(ph), np.cos(ph)
    uxx = e * ((0.16 - 1.69) * s + 2 * 0.4 * 1.3 * c)
    uyy = e * (-0.64 * s) - 0.49 * np.cos(0.7 * Y + 0.5 * Z)
    uzz = e * ((0.04 - 1.21) * s + 2 * 0.2 * 1.1 * c) - 0.25 * np.cos(0.7 * Y + 0.5 * Z)
    uz = e * (0.2 * s + 1.1 * c) - 0.5 * np.sin(0.7 * Y + 0.5 * Z)
    kz = 3.0 + np.sin(2.0 * z)
    k2 = kz ** 2
    k2z = 2 * kz * 2 * np.cos(2.0 * z)
    k2zz = 2 * (2 * np.cos(2.0 * z)) ** 2 + 2 * kz * (-4 * np.sin(2.0 * z))
    if scheme == "cd4":
        f = uxx + uyy + uzz + gamma * uz
    else:
        f = uxx + uyy + uzz + k2[:, None, None] * u
    W = O.stencil_weights(scheme, n, hx, hy, hz, k2, k2z, k2zz, gamma)
    F = O.rhs(scheme, f, hx, hy, hz, k2, k2z, gamma)
    r = O.apply_operator(W, u) - F
    return abs(r[ic - 1, ic - 1, ic - 1])


@pytest.mark.parametrize("scheme,ratios,expect", [
    ("helm2", (1.0, 1.3, 0.8), 4),
    ("helm4", (1.0, 1.3, 0.8), 6),
    ("cd4", (1.0, 1.3, 0.8), 6),
    ("helm6", (1.0, 1.0, 1.0), 8),
])
@pytest.mark.parametrize("centre", [(0.31, -0.17, 0.23), (1.1, 0.4, -0.6)])
def test_truncation_order_of_scaled_row(scheme, ratios, expect, centre):
    hs = (0.16, 0.08, 0.04)
    r = [_trunc_residual(scheme, h, ratios, gamma=-3.0, centre=centre) for h in hs]
    orders = [math.log2(r[i] / r[i + 1]) for i in range(2)]
    assert all(abs(o - expect) < 0.15 for o in orders), (r, orders)


@pytest.mark.parametrize("mistake", ["drop_k2f", "drop_k2z_fz", "biharmonic", "swap_bc",
                                     "sign_k2z_weight"])
def test_truncation_pin_detects_planted_mistakes(monkeypatch, mistake):
    """Each plausible slip, planted in the oracle on the CPU, lowers the observed order."""
    scheme, ratios = ("helm6", (1.0, 1.0, 1.0))
    orig_rhs, orig_w = O.rhs, O.stencil_weights
    if mistake == "swap_bc":
        scheme, ratios = ("helm4", (1.0, 1.3, 0.8))

    def bad_rhs(sch, f, hx, hy, hz, k2=None, k2_z=None, gamma=0.0):
        F = orig_rhs(sch, f, hx, hy, hz, k2, k2_z, gamma)
        nz = f.shape[0] - 2
        inner = f[1:-1, 1:-1, 1:-1]
        k0 = np.asarray(k2)[1:nz + 1][:, None, None]
        kz = np.asarray(k2_z)[1:nz + 1][:, None, None]
        h = hz
        if mistake == "drop_k2f":
            F = F + h ** 4 * k0 * inner / 20.0
        if mistake == "drop_k2z_fz":
            F = F - h ** 5 * kz * 0.5 * (f[2:, 1:-1, 1:-1] - f[:-2, 1:-1, 1:-1]) / 60.0
        if mistake == "biharmonic":
            # cross fourth derivatives counted twice (nabla^4 read as the biharmonic)
            F = F + h ** 2 * (2.0 / 360.0) * (O.cs3d_oracle._d2d2(f, 1, 2) + O.cs3d_oracle._d2d2(f, 0, 2)
                                              + O.cs3d_oracle._d2d2(f, 0, 1))
        return F

    def bad_w(*a, **k):
        W = orig_w(*a, **k)
        if mistake == "swap_bc":
            W[:, :, [1, 2]] = W[:, :, [2, 1]]
        if mistake == "sign_k2z_weight":
            W[:, [0, 2]] = W[:, [2, 0]]
        return W

    monkeypatch.setattr(O, "rhs", bad_rhs)
    monkeypatch.setattr(O, "stencil_weights", bad_w)
    r = [_trunc_residual(scheme, h, ratios, gamma=-3.0) for h in (0.08, 0.04)]
    expect = 8 if scheme == "helm6" else 6
    assert math.log2(r[0] / r[1]) < expect - 1.0, r


def test_helm6_needs_uniform_h():
    with pytest.raises(ValueError):
        O.stencil_weights("helm6", 4, 0.1, 0.1, 0.2, np.ones(6), np.zeros(6), np.zeros(6))


# ---------------------------------------------------------------------------
# P5: the sine transform and the eigen-structure of the 9-point blocks
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 7, 31, 50])
def test_sine_matrix_orthonormal_symmetric(n):
    S = O.sine_matrix(n)
    assert np.allclose(S, S.T, atol=0)
    assert np.abs(S @ S - np.eye(n)).max() < 1e-14


def test_dst_modes_are_eigenvectors_of_plane_blocks():
    rng = np.random.default_rng(5)
    nx, ny = 7, 5
    W = rng.uniform(-1, 1, size=(1, 3, 4))
    lam = O.modal_eigenvalues(W, nx, ny)
    for (m, n) in [(1, 1), (2, 5), (5, 3), (4, 7)]:
        mode = np.outer(np.sin(np.pi * m * np.arange(ny + 2) / (ny + 1)),
                        np.sin(np.pi * n * np.arange(nx + 2) / (nx + 1)))
        for o in range(3):
            Ucl = np.zeros((3, ny + 2, nx + 2))
            Ucl[o] = mode
            out = O.apply_operator(W, Ucl)[0]
            assert np.abs(out - lam[0, o, m - 1, n - 1] * mode[1:-1, 1:-1]).max() < 1e-13


def test_dst2_matches_naive_double_sum():
    rng = np.random.default_rng(6)
    F = rng.standard_normal((2, 5, 6))
    Fb = O.dst2(F)
    ny, nx = 5, 6
    for l in range(2):
        for m in range(1, ny + 1):
            for n in range(1, nx + 1):
                s = 0.0
                for j in range(1, ny + 1):
                    for i in range(1, nx + 1):
                        s += (2 / math.sqrt((nx + 1) * (ny + 1)) * math.sin(math.pi * n * i / (nx + 1))
                              * math.sin(math.pi * m * j / (ny + 1)) * F[l, j - 1, i - 1])
                assert abs(s - Fb[l, m - 1, n - 1]) < 1e-13


# ---------------------------------------------------------------------------
# Thomas against a library banded solver
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["dominant", "indefinite"])
def test_thomas_vs_banded_solver(kind):
    rng = np.random.default_rng(7)
    nz = 40
    lam = rng.uniform(-1, 1, size=(nz, 3, 3, 4))
    if kind == "dominant":
        lam[:, 1] += 4.0 * np.sign(lam[:, 1])
    else:
        lam[:, 1] = rng.uniform(-2.2, 2.2, size=(nz, 3, 4))
    F = rng.standard_normal((nz, 3, 4))
    Wm, minpiv, bad = O.thomas(lam, F)
    assert bad == 0
    for m in range(3):
        for n in range(4):
            ab = np.zeros((3, nz))
            ab[0, 1:] = lam[:-1, 2, m, n]
            ab[1] = lam[:, 1, m, n]
            ab[2, :-1] = lam[1:, 0, m, n]
            ref = scipy.linalg.solve_banded((1, 1), ab, F[:, m, n])
            tol = 1e-12 * max(1.0, np.abs(ref).max()) * (1.0 if kind == "dominant" else 1e3)
            assert np.abs(ref - Wm[:, m, n]).max() < tol


def test_thomas_flags_zero_pivot():
    lam = np.zeros((2, 3, 1, 1))
    lam[:, 1] = 1.0
    lam[0, 1] = 0.0
    _, minpiv, bad = O.thomas(lam, np.ones((2, 1, 1)))
    assert bad >= 1 and minpiv == 0.0


# ---------------------------------------------------------------------------
# P6: brute force on tiny grids (assembled matrix + dense partial-pivot LU)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme,dims", [
    ("helm2", (4, 5, 6)), ("helm4", (4, 5, 6)), ("helm4", (7, 7, 7)), ("cd4", (5, 4, 6)),
    ("helm6", (4, 6, 5)), ("helm6", (7, 7, 7)), ("helm4", (3, 2, 1)), ("cd4", (1, 1, 5)),
])
def test_solve_matches_dense_lu(scheme, dims):
    nx, ny, nz = dims
    if scheme == "helm6" or min(dims) >= 1:
        pass
    p = WL.noise_problem(nx, ny, nz, scheme, seed=11 + nx + ny * nz)
    f = p.f[0].numpy()
    gl, gh = p.g_lo[0].numpy(), p.g_hi[0].numpy()
    W = O.stencil_weights(scheme, nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma)
    if scheme == "helm6":
        F = O.rhs(scheme, f, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.gamma)
    else:
        F = O.rhs(scheme, f, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.gamma)
    Fl = O.lift(W, F, gl, gh)
    ref = O.dense_solve(W, Fl)
    res = O.solve(scheme, f, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma, gl, gh)
    assert np.abs(res.U - ref).max() <= 1e-13 * np.abs(ref).max()
    # the residual path (direct operator application, boundary planes included) agrees
    r = F - O.apply_operator(W, O.closed(res.U, gl, gh))
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(Fl)


def test_dense_assembly_matches_operator_application():
    rng = np.random.default_rng(3)
    nx, ny, nz = 3, 4, 5
    W = rng.standard_normal((nz, 3, 4))
    U = rng.standard_normal((nz, ny, nx))
    A = O.assemble_dense(W, nx, ny, nz)
    assert np.abs(A @ U.reshape(-1) - O.apply_operator(W, O.closed(U)).reshape(-1)).max() < 1e-13


# ---------------------------------------------------------------------------
# P7: discrete manufactured solution at a size dense LU cannot reach
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme,dims", [("helm4", (31, 17, 23)), ("helm6", (20, 24, 19)),
                                         ("cd4", (16, 33, 12))])
def test_discrete_manufactured_solution(scheme, dims):
    nx, ny, nz = dims
    p = WL.noise_problem(nx, ny, nz, scheme, seed=21)
    W = O.stencil_weights(scheme, nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma)
    rng = np.random.default_rng(9)
    Ustar = rng.uniform(-1, 1, size=(nz, ny, nx))
    gl, gh = p.g_lo[0].numpy(), p.g_hi[0].numpy()
    F = O.apply_operator(W, O.closed(Ustar, gl, gh))
    res = O.solve(scheme, None, p.hx, p.hy, p.hz, W=W, F=F, g_lo=gl, g_hi=gh)
    assert np.abs(res.U - Ustar).max() < 1e-11


# ---------------------------------------------------------------------------
# P8: closed forms
# ---------------------------------------------------------------------------
def test_constant_k_matches_3d_sine_transform_closed_form():
    nx, ny, nz = 9, 6, 11
    p = WL.noise_problem(nx, ny, nz, "helm4", seed=31, prof=WL.problems.k_const(7.0), boundary=False)
    f = p.f[0].numpy()
    res = O.solve("helm4", f, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz)
    W = res.W
    assert np.allclose(W[:, 0], W[:, 2]) and np.allclose(W, W[0:1])
    lam = O.modal_eigenvalues(W[:1], nx, ny)[0]      # (3, ny, nx)
    cz = np.cos(np.pi * np.arange(1, nz + 1) / (nz + 1))[:, None, None]
    Lam = lam[1][None] + 2.0 * lam[0][None] * cz      # eigenvalues of the Toeplitz tridiagonals
    Sx, Sy, Sz = O.sine_matrix(nx), O.sine_matrix(ny), O.sine_matrix(nz)
    F = res.F
    Fh = np.einsum("pl,mj,ni,lji->pmn", Sz, Sy, Sx, F)
    U = np.einsum("pl,mj,ni,pmn->lji", Sz, Sy, Sx, Fh / Lam)
    assert np.abs(U - res.U).max() < 1e-12 * np.abs(U).max()


def test_single_plane_is_a_diagonal_modal_solve():
    nx, ny = 6, 5
    p = WL.noise_problem(nx, ny, 1, "helm2", seed=41, boundary=False)
    res = O.solve("helm2", p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz)
    lam0 = O.modal_eigenvalues(res.W, nx, ny)[0, 1]
    U = O.dst2(O.dst2(res.F) / lam0[None])
    assert np.abs(U - res.U).max() < 1e-13 * np.abs(U).max()


# ---------------------------------------------------------------------------
# Input generator: SplitMix64 published outputs
# ---------------------------------------------------------------------------
def test_splitmix64_reference_outputs(golden_dir):
    with open(os.path.join(golden_dir, "splitmix64.json")) as fh:
        g = json.load(fh)
    out = WL.splitmix64_u64(g["seed"], len(g["outputs_hex"]))
    got = [format(int(v) & ((1 << 64) - 1), "016x") for v in out]
    assert got == g["outputs_hex"]


def test_uniform_chunking_is_consistent():
    a = WL.uniform01(77, (1000,))
    b = WL.uniform01(77, (400,), offset=600)
    assert np.array_equal(a[600:].numpy(), b.numpy())
    assert float(a.min()) >= 0.0 and float(a.max()) < 1.0


# ---------------------------------------------------------------------------
# Extended-precision mode: same discrete system, residual far below the FP64 level
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme,dims", [("helm6", (63, 40, 33)), ("cd4", (20, 17, 9))])
def test_extended_precision_solve_has_tiny_residual(scheme, dims):
    nx, ny, nz = dims
    p = WL.noise_problem(nx, ny, nz, scheme, seed=55)
    gl, gh = p.g_lo[0].numpy(), p.g_hi[0].numpy()
    r64 = O.solve(scheme, p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma, gl, gh)
    rld = O.solve(scheme, p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma, gl, gh,
                  dtype=np.longdouble)
    Fl = O.lift(r64.W, r64.F, gl, gh).astype(np.longdouble)
    Wld = r64.W.astype(np.longdouble)

    def res(U):
        # residual of the interior system in extended precision, U given in FP64
        return float(np.linalg.norm((Fl - O.apply_operator(Wld, O.closed(U.astype(np.longdouble))))
                                    .astype(np.float64)) / np.linalg.norm(Fl.astype(np.float64)))

    assert res(rld.U) <= res(r64.U) + 1e-16
    assert res(rld.U) < 5e-16
    assert np.linalg.norm(rld.U - r64.U) / np.linalg.norm(rld.U) < 1e-10
    # extended mode matches brute force exactly on a tiny grid
    q = WL.noise_problem(4, 5, 6, scheme, seed=56)
    ql, qh = q.g_lo[0].numpy(), q.g_hi[0].numpy()
    rq = O.solve(scheme, q.f[0].numpy(), q.hx, q.hy, q.hz, q.k2, q.k2_z, q.k2_zz, q.gamma, ql, qh,
                 dtype=np.longdouble)
    ref = O.dense_solve(rq.W, O.lift(rq.W, rq.F, ql, qh))
    assert np.abs(rq.U - ref).max() <= 1e-13 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# Complex k(z) (absorbing media; reading R16)
# ---------------------------------------------------------------------------
def _csolve(p, dtype=np.float64, k2=None, f=None, g=True):
    gl = p.g_lo[0].numpy() if (g and p.g_lo is not None) else None
    gh = p.g_hi[0].numpy() if (g and p.g_hi is not None) else None
    k2 = p.k2 if k2 is None else k2
    return O.solve(p.scheme, p.f[0].numpy() if f is None else f, p.hx, p.hy, p.hz, k2, p.k2_z, p.k2_zz,
                   p.gamma, gl, gh, dtype=dtype), gl, gh


@pytest.mark.parametrize("scheme,n", [("helm2", (6, 5, 7)), ("helm4", (7, 4, 6)), ("helm6", (5, 6, 7)),
                                      ("helm4", (3, 2, 1))])
def test_complex_k_matches_dense_lu(scheme, n):
    p = WL.complex_noise_problem(*n, scheme, seed=31 + sum(n))
    assert np.iscomplexobj(p.k2)
    res, gl, gh = _csolve(p)
    ref = O.dense_solve(res.W, O.lift(res.W, res.F, gl, gh))
    assert np.iscomplexobj(res.U) and np.abs(ref.imag).max() > 1e-3
    assert np.abs(res.U - ref).max() <= 1e-12 * np.abs(ref).max()
    # extended-precision transforms and Thomas on the same complex system
    rl, _, _ = _csolve(p, dtype=np.longdouble)
    assert np.abs(rl.U - ref).max() <= 1e-12 * np.abs(ref).max()


def test_complex_k_conjugate_medium_gives_conjugate_solution():
    p = WL.complex_noise_problem(9, 8, 7, "helm6", seed=5, boundary=False)
    f = p.f[0].numpy().real.copy()
    r1, _, _ = _csolve(p, f=f)
    r2 = O.solve("helm6", f, p.hx, p.hy, p.hz, np.conj(p.k2), np.conj(p.k2_z), np.conj(p.k2_zz))
    assert np.abs(r2.U - np.conj(r1.U)).max() <= 1e-13 * np.abs(r1.U).max()
    assert np.abs(r1.U.imag).max() > 1e-3 * np.abs(r1.U).max()


def test_complex_data_with_real_k_splits_into_real_solves():
    p = WL.noise_problem(9, 7, 8, "helm4", seed=6)
    f = p.f[0].numpy()
    fi = WL.uniform_pm1(99, tuple(p.f.shape[1:])).numpy()
    k2c = p.k2.astype(np.complex128)
    rc = O.solve("helm4", f + 1j * fi, p.hx, p.hy, p.hz, k2c)
    rr = O.solve("helm4", f, p.hx, p.hy, p.hz, p.k2)
    ri = O.solve("helm4", fi, p.hx, p.hy, p.hz, p.k2)
    assert np.abs(rc.U - (rr.U + 1j * ri.U)).max() <= 1e-13 * np.abs(rc.U).max()


@pytest.mark.parametrize("scheme,lo,hi", [("helm4", 3.7, 4.4), ("helm6", 5.5, 6.8)])
def test_complex_k_observed_order_under_h_halving(scheme, lo, hi):
    errs = []
    for n in (15, 31, 63):
        p = WL.manufactured_sin3(n, n, n, scheme, WL.K_ABSORB)
        assert np.iscomplexobj(p.k2)
        res, _, _ = _csolve(p)
        errs.append(np.abs(res.U - p.u_exact[0].numpy()[1:-1, 1:-1, 1:-1]).max())
    order = math.log2(errs[1] / errs[2])
    assert lo < order < hi, (errs, order)
