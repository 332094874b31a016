"""Pins of the oracle's Neumann-sides path (reading R21: du/dn = 0 on the x and y faces,
closed by even reflection, solved with a DCT-I in place of the DST-I).

* the DCT-I itself: C C = (M/2) I, and C x equals scipy's type-1 DCT (a library routine);
* the modal angles and the mirror rule: the cosine vectors are eigenvectors of the
  reflected 9-point plane blocks as assembled entry by entry, with the eigenvalues of
  Section 3.6 at theta_n = n pi/M;
* brute force: the transform solve equals dense LU of the assembled reflected matrix on
  tiny grids, for every scheme, with z-face data;
* the PDE: on u = cos(pi x) cos(2 pi y) (sin 3 pi z + cos(pi z)/2) the observed orders
  under h-halving are 2, 4 and 6, and a wrong mirror rule breaks them.
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle as O
import workloads as WL

PROF = WL.problems.KProfile(lambda z: 4.0 + np.sin(2 * np.pi * z),
                            lambda z: 2 * np.pi * np.cos(2 * np.pi * z),
                            lambda z: -4 * np.pi ** 2 * np.sin(2 * np.pi * z))


def _solve(p, r=0, dtype=np.float64):
    gl = None if p.g_lo is None else p.g_lo[r].numpy()
    gh = None if p.g_hi is None else p.g_hi[r].numpy()
    return O.solve(p.scheme, p.f[r].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma, gl, gh,
                   dtype=dtype, sides="neumann"), gl, gh


@pytest.mark.parametrize("nodes", [2, 3, 8, 33, 65, 130])
def test_cosine_matrix_squares_to_half_M_and_matches_scipy(nodes):
    C = O.cosine_matrix(nodes)
    M = nodes - 1
    assert np.abs(C @ C - 0.5 * M * np.eye(nodes)).max() < 1e-12 * M
    x = np.random.default_rng(nodes).standard_normal(nodes)
    # scipy's unnormalised DCT-I is twice the e-weighted sum
    assert np.abs(C @ x - 0.5 * scipy.fft.dct(x, type=1)).max() < 1e-12 * np.abs(x).sum()


@pytest.mark.parametrize("nx,ny", [(3, 5), (6, 4), (9, 9)])
def test_cosine_modes_are_eigenvectors_of_reflected_plane_blocks(nx, ny):
    rng = np.random.default_rng(nx * 10 + ny)
    W = rng.standard_normal((1, 3, 4))
    A = O.assemble_dense(W, nx, ny, 1, sides="neumann")  # one plane: the offset-0 block
    lam = O.modal_eigenvalues(W, nx, ny, sides="neumann")[0, 1]
    i, j = np.arange(nx), np.arange(ny)
    for n in range(nx):
        for m in range(ny):
            v = np.outer(np.cos(np.pi * m * j / (ny - 1)), np.cos(np.pi * n * i / (nx - 1))).reshape(-1)
            assert np.abs(A @ v - lam[m, n] * v).max() < 1e-12 * (1 + np.abs(lam[m, n]))


def test_reflected_assembly_matches_operator_application():
    rng = np.random.default_rng(5)
    nx, ny, nz = 4, 5, 3  # nodes per line
    W = rng.standard_normal((nz, 3, 4))
    U = rng.standard_normal((nz, ny, nx))
    A = O.assemble_dense(W, nx, ny, nz, sides="neumann")
    AU = O.apply_operator(W, O.closed(U, sides="neumann"), sides="neumann")
    assert np.abs(A @ U.reshape(-1) - AU.reshape(-1)).max() < 1e-13
    # a side node couples twice to its inner neighbour: the mirrored entry
    r = 0  # node (0, 0, 0)
    a, b, c, d = W[0, 1]
    assert math.isclose(A[r, 1], 2 * b, rel_tol=1e-14)      # x-neighbour 1 and its mirror -1
    assert math.isclose(A[r, nx], 2 * c, rel_tol=1e-14)     # y-neighbour
    assert math.isclose(A[r, nx + 1], 4 * a, rel_tol=1e-14)  # corner: four mirror images


@pytest.mark.parametrize("scheme,dims", [
    ("helm2", (4, 5, 6)), ("helm4", (3, 4, 5)), ("helm4", (1, 2, 1)), ("cd4", (5, 3, 4)),
    ("helm6", (4, 5, 6)), ("helm6", (6, 4, 4)),
])
def test_neumann_solve_matches_dense_lu(scheme, dims):
    nx, ny, nz = dims
    p = WL.neumann_noise_problem(nx, ny, nz, scheme, seed=31 + nx + 3 * ny + 7 * nz)
    f, gl, gh = p.f[0].numpy(), p.g_lo[0].numpy(), p.g_hi[0].numpy()
    W = O.stencil_weights(scheme, nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma)
    F = O.rhs(scheme, f, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.gamma, sides="neumann")
    assert F.shape == (nz, ny + 2, nx + 2)
    Fl = O.lift(W, F, gl, gh, sides="neumann")
    ref = O.dense_solve(W, Fl, sides="neumann")
    res, _, _ = _solve(p)
    assert res.U.shape == (nz, ny + 2, nx + 2)
    assert np.abs(res.U - ref).max() <= 1e-12 * np.abs(ref).max()
    # the residual path (mirrored operator application with the z-face planes)
    r = F - O.apply_operator(W, O.closed(res.U, gl, gh, sides="neumann"), sides="neumann")
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(Fl)


def test_neumann_rhs_equals_dirichlet_formula_on_the_mirrored_grid_interior():
    """Away from the sides the Neumann RHS is the Dirichlet one: same f, same formula."""
    p = WL.neumann_noise_problem(9, 8, 7, "helm6", seed=3)
    f = p.f[0].numpy()
    Fn = O.rhs("helm6", f, p.hx, p.hy, p.hz, p.k2, p.k2_z, sides="neumann")
    Fd = O.rhs("helm6", f, p.hx, p.hy, p.hz, p.k2, p.k2_z)
    # Dirichlet interior node (i, j) = Neumann node (i, j); the fourth differences of the
    # Dirichlet path are one-sided on its first and last layers, so compare two layers in
    assert np.abs(Fn[:, 3:-3, 3:-3] - Fd[:, 2:-2, 2:-2]).max() < 1e-15 * np.abs(Fd).max()


@pytest.mark.parametrize("scheme,lo,hi", [("helm2", 1.8, 2.3), ("helm4", 3.7, 4.4), ("helm6", 5.5, 6.8)])
def test_neumann_observed_order_under_h_halving(scheme, lo, hi):
    errs = []
    for n in (15, 31, 63):
        p = WL.manufactured_cos2(n, n, n, scheme, PROF)
        res, _, _ = _solve(p)
        errs.append(np.abs(res.U - p.u_exact[0].numpy()[1:-1]).max())
    order = math.log2(errs[1] / errs[2])
    assert lo < order < hi, (errs, order)


def test_neumann_order_pin_detects_a_wrong_mirror(monkeypatch):
    """Mirroring about the half-cell (u_{-1} = u_0) instead of the side node is a plausible
    slip; it leaves a first-order closure that the observed-order pin rejects."""
    def half_cell(a, width):
        pad = [(0, 0)] * (a.ndim - 2) + [(width, width), (width, width)]
        return np.pad(a, pad, mode="symmetric")
    errs = []
    monkeypatch.setattr(O.cs3d_oracle, "mirror_pad", half_cell)
    for n in (15, 31, 63):
        p = WL.manufactured_cos2(n, n, n, "helm4", PROF)
        res, _, _ = _solve(p)
        errs.append(np.abs(res.U - p.u_exact[0].numpy()[1:-1]).max())
    order = math.log2(errs[1] / errs[2])
    assert not (3.7 < order < 4.4), (errs, order)


def test_neumann_constant_mode_of_a_pure_z_problem():
    """f and the z-face data independent of x and y: U is constant over every plane and
    the plane values solve the 1-D problem of mode (0, 0), whose eigenvalues are the row
    sums 4a + 2b + 2c + d (a check of the n = 0 angle)."""
    nx, ny, nz = 6, 5, 9
    p = WL.neumann_noise_problem(nx, ny, nz, "helm4", seed=8)
    zprof = np.random.default_rng(2).uniform(-1, 1, nz + 2)
    f = np.broadcast_to(zprof[:, None, None], p.f[0].shape).copy()
    gl = np.full(p.g_lo[0].shape, 0.3)
    gh = np.full(p.g_hi[0].shape, -0.7)
    res = O.solve("helm4", f, p.hx, p.hy, p.hz, p.k2, gamma=0.0, g_lo=gl, g_hi=gh, sides="neumann")
    U = res.U
    assert np.abs(U - U[:, :1, :1]).max() < 1e-13 * np.abs(U).max()
    W = O.stencil_weights("helm4", nz, p.hx, p.hy, p.hz, p.k2)
    s = 4 * W[..., 0] + 2 * W[..., 1] + 2 * W[..., 2] + W[..., 3]  # (nz, 3)
    F = O.rhs("helm4", f, p.hx, p.hy, p.hz, p.k2, sides="neumann")[:, 0, 0].copy()
    F[0] -= s[0, 0] * 0.3
    F[-1] -= s[-1, 2] * -0.7
    T = np.diag(s[:, 1]) + np.diag(s[1:, 0], -1) + np.diag(s[:-1, 2], 1)
    assert np.abs(np.linalg.solve(T, F) - U[:, 0, 0]).max() < 1e-12 * np.abs(U).max()
