"""Pins of the oracle's Robin z faces (reading R22: alpha u_z + beta u = g on the z faces,
Section 1, eq. bc), against things other than itself.

* the ghost-plane formula against the exact ghost value of a smooth solution: its error
  falls as h^5 (a dropped term or a sign slip changes that);
* the modal solve (DST, changed first and last tridiagonal rows) against a dense LU of the
  (nz+2)-plane system assembled entry by entry with the ghost planes substituted;
* observed orders under h-halving on a manufactured solution: 2 (HELM2), 4 (HELM4) and 4
  (HELM6, whose closure near the faces is of fourth order);
* planted mistakes in the closure that these pins must catch.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.cs3d_oracle as OC
import workloads as WL


def _solve(p, **kw):
    return O.solve_robin(p.scheme, p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.robin[0],
                         p.robin[1], p.g_lo[0].numpy(), p.g_hi[0].numpy(), **kw)


def _orders(scheme, sizes=(15, 31, 63)):
    errs = []
    for n in sizes:
        p = WL.manufactured_robin(n, scheme)
        r = _solve(p)
        errs.append(np.abs(r.U - p.u_exact[0].numpy()[:, 1:-1, 1:-1]).max())
    return errs, [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_ghost_formula_matches_the_exact_ghost_plane():
    """U_{-1} = U_1 + (c0 + c1 D) U_0 + R_lo must reproduce u(z = -h) of a smooth solution of
    the equation to O(h^5) (and the top face likewise u(1 + h)): ratio ~32 per halving."""
    prof = WL.problems.KProfile(lambda z: 4.0 + np.sin(2 * np.pi * z), lambda z: 2 * np.pi * np.cos(2 * np.pi * z),
                                lambda z: -4 * np.pi ** 2 * np.sin(2 * np.pi * z))
    errs = []
    for n in (15, 31, 63):
        p = WL.manufactured_robin(n, "helm4", prof=prof)
        h = p.hz
        z = np.array([-h, 1.0 + h])
        Z = np.cos(1.3 * z) + 0.5 * np.sin(2.1 * z)
        x = h * np.arange(n + 2)
        S = np.outer(np.sin(2 * np.pi * x), np.sin(np.pi * x))[1:-1, 1:-1]
        (c_lo, c_hi), (R_lo, R_hi) = O.robin_ghost(n, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.robin[0], p.robin[1],
                                                   p.f[0].numpy(), p.g_lo[0].numpy(), p.g_hi[0].numpy())
        u = p.u_exact[0].numpy()
        ue = u[:, 1:-1, 1:-1]
        lapD = lambda P: OC._plane_lap(P, p.hx, p.hy)  # noqa: E731
        gl = ue[1] + c_lo[0] * ue[0] + c_lo[1] * lapD(u[0]) + R_lo
        gh = ue[-2] + c_hi[0] * ue[-1] + c_hi[1] * lapD(u[-1]) + R_hi
        errs.append(max(np.abs(gl - Z[0] * S).max(), np.abs(gh - Z[1] * S).max()))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(26 < r < 40 for r in ratios), (errs, ratios)


@pytest.mark.parametrize("scheme,dims", [("helm2", (5, 4, 4)), ("helm4", (4, 6, 5)), ("helm6", (5, 5, 4)),
                                         ("helm4", (3, 2, 4))])
def test_robin_modal_solve_matches_dense_lu(scheme, dims):
    nx, ny, nz = dims
    p = WL.robin_noise_problem(nx, ny, nz, scheme, seed=41 + nx + ny + nz)
    r = _solve(p)
    A = O.assemble_dense_robin(scheme, nx, ny, nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.robin[0], p.robin[1])
    Ud = np.linalg.solve(A, r.F.reshape(-1)).reshape(nz + 2, ny, nx)
    assert np.abs(Ud - r.U).max() <= 1e-13 * np.abs(Ud).max()
    assert r.bad == 0


@pytest.mark.parametrize("scheme,lo,hi", [("helm2", 1.9, 2.1), ("helm4", 3.7, 4.3), ("helm6", 3.7, 4.3)])
def test_robin_observed_orders(scheme, lo, hi):
    errs, orders = _orders(scheme)
    assert lo < orders[-1] < hi, (errs, orders)


def test_robin_extended_precision_agrees():
    p = WL.robin_noise_problem(31, 17, 9, "helm6", seed=5)
    a = _solve(p).U
    b = _solve(p, dtype=np.longdouble).U
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def _no_h3(nz, hx, hy, hz, k2, k2_z, alpha, beta, f, g_lo, g_hi):
    """A plausible slip: the closure of the central difference only (no u_zzz term)."""
    (a0, a1), (b0, b1) = alpha, beta
    h = hz
    gl, gh = np.asarray(g_lo, float), np.asarray(g_hi, float)
    return ((2 * h * b0 / a0, 0.0), (-2 * h * b1 / a1, 0.0)), (-2 * h * gl[1:-1, 1:-1] / a0, 2 * h * gh[1:-1, 1:-1] / a1)


def _flipped_top(nz, hx, hy, hz, k2, k2_z, alpha, beta, f, g_lo, g_hi):
    """A plausible slip: the top face takes the bottom face's formula (outward normal mixed up)."""
    (c_lo, c_hi), (R_lo, R_hi) = _ORIG(nz, hx, hy, hz, k2, k2_z, alpha, beta, f, g_lo, g_hi)
    (a0, a1), (b0, b1) = alpha, beta
    h = hz
    kh, kzh = np.asarray(k2)[-2], np.asarray(k2_z)[-2]
    c_hi = ((h ** 3 / 3.0) * kzh - (b1 / a1) * (-2.0 * h + (h ** 3 / 3.0) * kh), -(b1 / a1) * (h ** 3 / 3.0))
    return (c_lo, c_hi), (R_lo, -R_hi)


_ORIG = O.robin_ghost


@pytest.mark.parametrize("mistake,scheme", [(_no_h3, "helm4"), (_flipped_top, "helm4"), (_no_h3, "helm6")])
def test_robin_pins_catch_planted_mistakes(monkeypatch, mistake, scheme):
    monkeypatch.setattr(OC, "robin_ghost", mistake)
    errs, orders = _orders(scheme)
    assert not (3.7 < orders[-1] < 4.3), (errs, orders)
