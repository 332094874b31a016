"""Plain, slow, obviously correct FP64 oracle of the compact 27-point FFT direct solver.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``; never by the product path.

Paper: Gonzales, Gryazin & Lee, "Scalable Algorithms for High-Order
Approximations on Three-Dimensional Compact Stencils" (arXiv 1912.03565).

What it computes.  The grid has N_alpha interior points per axis and
h_alpha = L_alpha/(N_alpha+1) (Section 2).  Row (i, j, l) of the 27-diagonal system
A U = F holds, for each plane offset o = -1, 0, +1, four weights (a, b, c, d)
multiplying the corner, x-edge, y-edge and centre points of plane l+o (eq.
stencil27, Figure 1).  The weights of every scheme are functions of the row l
only (Sections 3.2 - 3.5).  The solve is Section 3.6: an orthonormal 2-D DST-I
diagonalises every in-plane 9-point block, leaving N_x N_y independent
tridiagonal systems along z that are solved by LU without pivoting (Thomas).

Arrays are numpy float64 indexed [z, y, x] (x fastest), matching the paper's row
index i + N_x j + N_x N_y l.  Interior arrays have shape (nz, ny, nx); closed-grid
arrays have shape (nz+2, ny+2, nx+2); z-face data are closed planes (ny+2, nx+2).

Readings taken where the paper is silent, garbled or inconsistent (each one is
listed with its justification in the design notes of the repository):
  R1  "N^3" counts interior points.
  R2  the b-term of eq. stencil27 multiplies the two x-neighbours (Figure 1).
  R3  modal angles theta_n = n pi/(N_x+1), n = 1..N_x (the eigenvector indices).
  R4  weights depend on the row l; the modal tridiagonal is non-symmetric.
  R5  non-zero Dirichlet data on the z faces are moved to the right-hand side
      through the plane-offset weights of rows 1 and N_z.
  R6-R8 the 6th-order RHS carries -(h^2/20) k_l^2 f + (h^4/60) (k^2)_z f_z (the two
      terms hidden in the garbled Delta_h(k^2 U)); its "nabla^4 f" is the sum of the
      three pure fourth derivatives.
  R10 6th-order derivatives of f by explicit central differences on the closed
      grid; the fourth differences of the first and last interior layer are the
      one-sided 6-point formula (2, -9, 16, -14, 6, -1)/h^4.
  R14 the convection-diffusion d_{l+-1} has an unbalanced parenthesis; read as
      2/3 - (R_zx+R_zy)/6 +- (h_z gamma/12)(4 - R_zx - R_zy +- h_z gamma).
  R15 "LU decomposition" of each tridiagonal = Thomas without pivoting.
  R16 k may be complex (Section 1 allows it): the weights, the modal eigenvalues, the
      right-hand side and U are then complex; the sine transforms are real and act on
      the real and imaginary parts alike, so only the tridiagonal solves are complex.
  R21 Neumann sides (Section 1 names the extension to Neumann conditions on the sides,
      without a discretisation): du/dn = 0 on the x and y faces is closed by even
      reflection.  The side nodes i = 0, N_x+1 (j = 0, N_y+1) become unknowns, every
      node carries the scheme's own row, and a value beyond a side is the mirror image
      about it: U_{-1} = U_1, U_{N+2} = U_N, and the same for f in the right-hand side,
      whose x and y differences are then all central.  The reflected 9-point plane
      blocks are diagonalised by the cosine vectors cos(pi n i/M), n, i = 0..M = N+1,
      with the eigenvalue formula of Section 3.6 at theta_n = n pi/M, so a DCT-I takes
      the place of the DST-I.  The scheme keeps its order for solutions whose odd
      normal derivatives vanish on the sides (the cosine class), as the Dirichlet
      reading keeps it when the even derivatives of f vanish there.

Neumann arrays (sides="neumann"): the unknowns form arrays of shape (nz, ny+2, nx+2)
(every x/y node of a plane); f and the z-face planes keep their closed-grid shapes.
"""
import numpy as np

SCHEMES = ("helm2", "helm4", "helm6", "cd4")


def _num(x):
    """x as a float64 array, or complex128 when x holds complex values (complex k)."""
    a = np.asarray(x)
    return a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)


def _complex_of(dtype):
    """The complex type of a real working precision."""
    return np.clongdouble if dtype == np.longdouble else np.complex128

__all__ = [
    "SCHEMES", "stencil_weights", "rhs", "lift", "sine_matrix", "dst2", "cosine_matrix", "dct2",
    "mirror_pad",
    "modal_eigenvalues", "thomas", "solve_modal", "solve", "apply_operator",
    "assemble_dense", "dense_solve", "error_norms", "OracleResult", "closed",
    "ROBIN_SCHEMES", "robin_weights", "robin_rhs", "robin_ghost", "solve_robin", "assemble_dense_robin",
]


# ----------------------------------------------------------------------------
# Stencil weights, Sections 3.2 - 3.5.
# W[l-1, o+1] = (a, b, c, d) of row l for plane offset o.
# ----------------------------------------------------------------------------
def stencil_weights(scheme, nz, hx, hy, hz, k2=None, k2_z=None, k2_zz=None, gamma=0.0):
    """Weights of every row, shape (nz, 3, 4).

    k2, k2_z, k2_zz are samples of k^2, (k^2)_z, (k^2)_zz at the planes z_0..z_{nz+1}.
    """
    cplx = any(v is not None and np.iscomplexobj(np.asarray(v)) for v in (k2, k2_z, k2_zz))
    W = np.zeros((nz, 3, 4), dtype=np.complex128 if cplx else np.float64)
    rzx = hz * hz / (hx * hx)
    rzy = hz * hz / (hy * hy)
    ls = np.arange(1, nz + 1)
    if scheme in ("helm2", "helm4", "helm6"):
        k2 = _num(k2)
        km, k0, kp = k2[ls - 1], k2[ls], k2[ls + 1]
    if scheme == "helm2":
        # Section 3.2: five non-zero weights.
        W[:, 0, 3] = 1.0
        W[:, 2, 3] = 1.0
        W[:, 1, 1] = rzx
        W[:, 1, 2] = rzy
        W[:, 1, 3] = -2.0 * (rzx + rzy + 1.0) + hz * hz * k0
    elif scheme == "helm4":
        # Section 3.3.
        for o, kk in ((0, km), (2, kp)):
            W[:, o, 1] = (1.0 + rzx) / 12.0
            W[:, o, 2] = (1.0 + rzy) / 12.0
            W[:, o, 3] = 2.0 / 3.0 - (rzx + rzy) / 6.0 + hz * hz * kk / 12.0
        W[:, 1, 0] = (rzx + rzy) / 12.0
        W[:, 1, 1] = (4.0 * rzx - rzy - 1.0 + hz * hz * k0 / 2.0) / 6.0
        W[:, 1, 2] = (4.0 * rzy - rzx - 1.0 + hz * hz * k0 / 2.0) / 6.0
        W[:, 1, 3] = -4.0 * (1.0 + rzx + rzy) / 3.0 + hz * hz * k0 / 2.0
    elif scheme == "helm6":
        # Section 3.4 (uniform h).
        if not (np.isclose(hx, hz, rtol=1e-13, atol=0) and np.isclose(hy, hz, rtol=1e-13, atol=0)):
            raise ValueError("6th-order scheme needs hx == hy == hz")
        h = hz
        kz = _num(k2_z)[ls]
        kzz = _num(k2_zz)[ls]
        for o, s, kk in ((0, -1.0, km), (2, 1.0, kp)):
            W[:, o, 0] = 1.0 / 30.0
            bc = 1.0 / 10.0 + h ** 2 * kk / 90.0 + s * h ** 3 * kz / 120.0
            W[:, o, 1] = bc
            W[:, o, 2] = bc
            W[:, o, 3] = (7.0 / 15.0 - h ** 2 * kk / 90.0
                          + s * (h ** 3 * kz / 20.0) * (1.0 / 3.0 + h ** 2 * kk / 6.0))
        W[:, 1, 0] = 1.0 / 10.0 + h ** 2 * k0 / 90.0
        W[:, 1, 1] = 7.0 / 15.0 - h ** 2 * k0 / 90.0
        W[:, 1, 2] = 7.0 / 15.0 - h ** 2 * k0 / 90.0
        W[:, 1, 3] = (-64.0 / 15.0 + 14.0 * h ** 2 * k0 / 15.0 - h ** 4 * k0 ** 2 / 20.0
                      + h ** 4 * kzz / 20.0)
    elif scheme == "cd4":
        # Section 3.5, with reading R14 of the unbalanced d_{l+-1}.
        t = hz * gamma
        for o, s in ((0, -1.0), (2, 1.0)):
            W[:, o, 1] = (1.0 + rzx) * (2.0 + s * t) / 24.0
            W[:, o, 2] = (1.0 + rzy) * (2.0 + s * t) / 24.0
            W[:, o, 3] = 2.0 / 3.0 - (rzx + rzy) / 6.0 + s * (t / 12.0) * (4.0 - rzx - rzy + s * t)
        W[:, 1, 0] = (rzx + rzy) / 12.0
        W[:, 1, 1] = (4.0 * rzx - rzy - 1.0) / 6.0
        W[:, 1, 2] = (4.0 * rzy - rzx - 1.0) / 6.0
        W[:, 1, 3] = -4.0 * (1.0 + rzx + rzy) / 3.0 - t * t / 6.0
    else:
        raise ValueError(f"unknown scheme {scheme}")
    return W


# ----------------------------------------------------------------------------
# Right-hand sides F (interior), Sections 2.1, 3.2 - 3.5.
# ----------------------------------------------------------------------------
def _d2(f, axis):
    """Second difference f_{-1} - 2 f_0 + f_{+1} on the interior of a closed-grid array."""
    sl = [slice(1, -1)] * 3
    lo, mid, hi = list(sl), list(sl), list(sl)
    lo[axis] = slice(0, -2)
    hi[axis] = slice(2, None)
    return f[tuple(lo)] - 2.0 * f[tuple(mid)] + f[tuple(hi)]


def _d1(f, axis):
    """Centred first difference (f_{+1} - f_{-1})/2 on the interior."""
    sl = [slice(1, -1)] * 3
    lo, hi = list(sl), list(sl)
    lo[axis] = slice(0, -2)
    hi[axis] = slice(2, None)
    return 0.5 * (f[tuple(hi)] - f[tuple(lo)])


def _d4(f, axis):
    """Fourth difference on the interior (reading R10).

    Central (1, -4, 6, -4, 1) where both neighbours at distance 2 exist; on the
    first and last interior layer the one-sided (2, -9, 16, -14, 6, -1) formula
    built from the boundary point and the next five points.
    """
    g = np.moveaxis(f, axis, 0)
    n = g.shape[0] - 2
    out = np.empty((n,) + g.shape[1:], dtype=g.dtype)
    if n < 4:
        raise ValueError("the fourth differences need at least 4 interior points per axis")
    out[1:n - 1] = g[0:n - 2] - 4 * g[1:n - 1] + 6 * g[2:n] - 4 * g[3:n + 1] + g[4:n + 2]
    out[0] = 2 * g[0] - 9 * g[1] + 16 * g[2] - 14 * g[3] + 6 * g[4] - g[5]
    out[n - 1] = 2 * g[n + 1] - 9 * g[n] + 16 * g[n - 1] - 14 * g[n - 2] + 6 * g[n - 3] - g[n - 4]
    out = np.moveaxis(out, 0, axis)
    # restrict the two transverse axes to the interior
    sl = [slice(1, -1)] * 3
    sl[axis] = slice(None)
    return out[tuple(sl)]


def _d2d2(f, a, b):
    """Product of second differences along axes a and b (a 9-point plane stencil)."""
    g = np.moveaxis(f, (a, b), (0, 1))
    s = g[:-2] - 2.0 * g[1:-1] + g[2:]
    s = s[:, :-2] - 2.0 * s[:, 1:-1] + s[:, 2:]
    s = np.moveaxis(s, (0, 1), (a, b))
    sl = [slice(1, -1)] * 3
    sl[a] = slice(None)
    sl[b] = slice(None)
    return s[tuple(sl)]


def mirror_pad(a, width):
    """Extend the last two axes (y, x) of a by ``width`` mirrored layers on each side:
    a value beyond a side is the one at the same distance inside (reading R21)."""
    pad = [(0, 0)] * (a.ndim - 2) + [(width, width), (width, width)]
    return np.pad(a, pad, mode="reflect")


def rhs(scheme, f, hx, hy, hz, k2=None, k2_z=None, gamma=0.0, sides="dirichlet"):
    """F on the interior from f on the closed grid (shape (nz+2, ny+2, nx+2)).

    sides="neumann" (reading R21): F on every x/y node, shape (nz, ny+2, nx+2); f is
    mirrored about the sides by two layers and the Dirichlet formula evaluated on the
    extended grid, whose one-sided side differences then fall outside what is kept.

    helm2: F = h_z^2 f (Section 3.2).
    helm4: F = h_z^2 (1 + sum_alpha h_alpha^2 delta_alpha^2/12) f (eq. scheme4, Section 3.3).
    cd4:   F = h_z^2 [f + h_x^2/12 f_xx + h_y^2/12 f_yy + h_z^2/12 (gamma f_z + f_zz)] with
           the derivatives replaced by centred differences (eq. cd_rhs).
    helm6: F = h^2 [f + h^2/12 sum d2 + h^4/360 sum d4 + h^4/90 sum d2d2
                    - h^2/20 k_l^2 f + h^4/60 (k^2)_z f_z]   (eq. scheme6, readings R6-R10),
           where sum_alpha h^2 delta^2 f is corrected by -1/240 h^4 delta^4 so that the h^4
           coefficient of f_{alpha alpha alpha alpha} is 1/360.
    """
    f = _num(f)
    if sides == "neumann":
        return rhs(scheme, mirror_pad(f, 2), hx, hy, hz, k2, k2_z, gamma)[:, 1:-1, 1:-1]
    nz = f.shape[0] - 2
    inner = f[1:-1, 1:-1, 1:-1]
    if scheme == "helm2":
        return hz * hz * inner
    if scheme == "helm4":
        return hz * hz * (inner + (_d2(f, 2) + _d2(f, 1) + _d2(f, 0)) / 12.0)
    if scheme == "cd4":
        return hz * hz * (inner + _d2(f, 2) / 12.0 + _d2(f, 1) / 12.0
                          + (hz * gamma * _d1(f, 0) + _d2(f, 0)) / 12.0)
    if scheme == "helm6":
        h = hz
        k0 = _num(k2)[1:nz + 1][:, None, None]
        kz = _num(k2_z)[1:nz + 1][:, None, None]
        s2 = _d2(f, 0) + _d2(f, 1) + _d2(f, 2)
        s4 = _d4(f, 0) + _d4(f, 1) + _d4(f, 2)
        sx = _d2d2(f, 1, 2) + _d2d2(f, 0, 2) + _d2d2(f, 0, 1)
        return h * h * (inner + s2 / 12.0 - s4 / 240.0 + sx / 90.0
                        - h * h * k0 * inner / 20.0 + h ** 3 * kz * _d1(f, 0) / 60.0)
    raise ValueError(f"unknown scheme {scheme}")


# ----------------------------------------------------------------------------
# In-plane 9-point application and the z-face lift (reading R5).
# ----------------------------------------------------------------------------
def _plane9(w, P):
    """Apply weights w = (a, b, c, d) to the interior of a closed plane P (ny+2, nx+2)."""
    a, b, c, d = w
    return (a * (P[:-2, :-2] + P[:-2, 2:] + P[2:, :-2] + P[2:, 2:])
            + b * (P[1:-1, :-2] + P[1:-1, 2:])
            + c * (P[:-2, 1:-1] + P[2:, 1:-1])
            + d * P[1:-1, 1:-1])


def lift(W, F, g_lo=None, g_hi=None, sides="dirichlet"):
    """F_1 -= (plane -1 weights of row 1) * g_lo;  F_Nz -= (plane +1 weights of row Nz) * g_hi.

    Neumann sides: the planes are mirrored by one layer, so every node of a plane takes part."""
    parts = [F, W] + [g for g in (g_lo, g_hi) if g is not None]
    F = np.array(F, dtype=np.result_type(*[_num(x) for x in parts]), copy=True)
    ext = (lambda g: mirror_pad(_num(g), 1)) if sides == "neumann" else _num
    if g_lo is not None:
        F[0] -= _plane9(W[0, 0], ext(g_lo))
    if g_hi is not None:
        F[-1] -= _plane9(W[-1, 2], ext(g_hi))
    return F


def apply_operator(W, U_closed, sides="dirichlet"):
    """(A U)_{i,j,l} = sum_o sum of the in-plane 9-point weights of plane l+o (eq. stencil27).

    U_closed holds the solution on the closed grid including its boundary values (Neumann
    sides: shape (nz+2, ny+2, nx+2), the nodes of every plane, mirrored by one layer here).
    This is the residual path: it shares nothing with the transform solve.
    """
    U = np.asarray(U_closed)
    if U.dtype not in (np.longdouble, np.clongdouble):
        U = _num(U)
    if sides == "neumann":
        U = mirror_pad(U, 1)
    nz = U.shape[0] - 2
    out = np.zeros((nz, U.shape[1] - 2, U.shape[2] - 2), dtype=np.result_type(U, W))
    for l in range(1, nz + 1):
        for o in (-1, 0, 1):
            out[l - 1] += _plane9(W[l - 1, o + 1], U[l + o])
    return out


# ----------------------------------------------------------------------------
# The orthonormal sine transform, Section 3.6: V = S_y (x) S_x with
# S[n-1, i-1] = sqrt(2/(N+1)) sin(pi n i/(N+1)), symmetric and its own inverse.
# ----------------------------------------------------------------------------
def _pi(dtype):
    """pi to the working precision (4 atan 1 in that precision)."""
    return 4 * np.arctan(np.ones((), dtype=dtype))


def sine_matrix(n, dtype=np.float64):
    """The product k*i is reduced modulo 2(N+1) in integers first, so every entry is
    sin(pi r/(N+1)) with 0 <= r < 2(N+1): no argument rounding for large k*i."""
    k = np.arange(1, n + 1)
    r = (np.outer(k, k) % (2 * (n + 1))).astype(dtype)
    two = np.asarray(2, dtype=dtype)
    return np.sqrt(two / (n + 1)) * np.sin(_pi(dtype) * r / (n + 1))


def dst2(F, dtype=None):
    """Fbar_l = V^T F_l for every plane: sums over x then over y (dense products)."""
    if np.iscomplexobj(F):  # the transform is real: real and imaginary parts alike
        re = dst2(np.real(F), dtype)
        return re + 1j * dst2(np.imag(F), dtype)
    dtype = F.dtype if dtype is None else dtype
    F = np.asarray(F, dtype=dtype)
    nz, ny, nx = F.shape
    Sx, Sy = sine_matrix(nx, dtype), sine_matrix(ny, dtype)
    G = np.matmul(F, Sx.T)          # x-sums:  G[l, j, n] = sum_i F[l, j, i] Sx[n, i]
    return np.matmul(Sy, G)         # y-sums:  Fbar[l, m, n] = sum_j Sy[m, j] G[l, j, n]


def cosine_matrix(nodes, dtype=np.float64):
    """DCT-I of a line of ``nodes`` = M + 1 values (reading R21):
    C[k, i] = e_i cos(pi k i/M), k, i = 0..M, e_0 = e_M = 1/2, e_i = 1 otherwise.
    C C = (M/2) I; the product k*i is reduced modulo 2M in integers first."""
    M = nodes - 1
    k = np.arange(nodes)
    r = (np.outer(k, k) % (2 * M)).astype(dtype)
    C = np.cos(_pi(dtype) * r / M)
    C[:, 0] *= 0.5
    C[:, M] *= 0.5
    return C


def dct2(F, dtype=None, inverse=False):
    """Per plane: C_y F C_x^T (x sums, then y sums); inverse=True also scales by
    (2/M_x)(2/M_y), which makes it the inverse transform."""
    if np.iscomplexobj(F):
        return dct2(np.real(F), dtype, inverse) + 1j * dct2(np.imag(F), dtype, inverse)
    dtype = F.dtype if dtype is None else dtype
    F = np.asarray(F, dtype=dtype)
    nz, ny, nx = F.shape
    Cx, Cy = cosine_matrix(nx, dtype), cosine_matrix(ny, dtype)
    out = np.matmul(Cy, np.matmul(F, Cx.T))
    if inverse:
        out = out * (np.asarray(4, dtype=dtype) / ((nx - 1) * (ny - 1)))
    return out


# ----------------------------------------------------------------------------
# Modal tridiagonal systems, Section 3.6.
# ----------------------------------------------------------------------------
def modal_eigenvalues(W, nx, ny, dtype=np.float64, sides="dirichlet"):
    """lam[l-1, o+1, m-1, n-1] = 4a cos(th_n) cos(ph_m) + 2b cos(th_n) + 2c cos(ph_m) + d.

    Dirichlet: th_n = n pi/(nx+1), n = 1..nx.  Neumann (nx, ny = nodes per line, R21):
    th_n = n pi/(nx-1), n = 0..nx-1."""
    pi = _pi(dtype)
    if sides == "neumann":
        ct = np.cos(pi * np.arange(nx, dtype=dtype) / (nx - 1))[None, :]
        cp = np.cos(pi * np.arange(ny, dtype=dtype) / (ny - 1))[:, None]
    else:
        ct = np.cos(pi * np.arange(1, nx + 1, dtype=dtype) / (nx + 1))[None, :]
        cp = np.cos(pi * np.arange(1, ny + 1, dtype=dtype) / (ny + 1))[:, None]
    W = np.asarray(W, dtype=_complex_of(dtype) if np.iscomplexobj(W) else dtype)
    a, b, c, d = (W[..., q][:, :, None, None] for q in range(4))
    return 4.0 * a * cp * ct + 2.0 * b * ct + 2.0 * c * cp + d


def thomas(lam, Fbar):
    """Solve lam^-_l W_{l-1} + lam^0_l W_l + lam^+_l W_{l+1} = Fbar_l, W_0 = W_{Nz+1} = 0.

    LU without pivoting (Thomas), every (m, n) column at once.  Returns
    (W, min |pivot|, number of zero or non-finite pivots).
    """
    nz = Fbar.shape[0]
    cp = np.empty_like(Fbar)
    dp = np.empty_like(Fbar)
    minpiv = np.inf
    bad = 0
    prev_c = np.zeros_like(Fbar[0])
    prev_d = np.zeros_like(Fbar[0])
    with np.errstate(divide="ignore", invalid="ignore"):
        for l in range(nz):
            piv = lam[l, 1] - lam[l, 0] * prev_c
            ap = np.abs(piv)
            ap = ap[np.isfinite(ap)]
            if ap.size:
                minpiv = min(minpiv, float(ap.min()))
            bad += int(np.count_nonzero(~np.isfinite(piv) | (piv == 0)))
            cp[l] = lam[l, 2] / piv
            dp[l] = (Fbar[l] - lam[l, 0] * prev_d) / piv
            prev_c, prev_d = cp[l], dp[l]
    Wm = np.empty_like(Fbar)
    Wm[nz - 1] = dp[nz - 1]
    for l in range(nz - 2, -1, -1):
        Wm[l] = dp[l] - cp[l] * Wm[l + 1]
    return Wm, minpiv, bad


def solve_modal(W, Fbar, sides="dirichlet"):
    nz, ny, nx = Fbar.shape
    real = np.real(Fbar[:1, :1, :1]).dtype
    lam = modal_eigenvalues(W, nx, ny, real, sides)
    if np.iscomplexobj(lam) and not np.iscomplexobj(Fbar):
        Fbar = Fbar.astype(_complex_of(real))
    return thomas(lam, Fbar)


class OracleResult:
    def __init__(self, U, W, F, minpiv, bad):
        self.U, self.W, self.F, self.minpiv, self.bad = U, W, F, minpiv, bad


def solve(scheme, f, hx, hy, hz, k2=None, k2_z=None, k2_zz=None, gamma=0.0,
          g_lo=None, g_hi=None, W=None, F=None, dtype=np.float64, sides="dirichlet"):
    """U = A^{-1}(F - lift): weights -> F -> lift -> DST -> Thomas -> inverse DST (Section 3.6).

    Either f (closed grid) with a scheme, or an assembled interior F with explicit W.
    The weights and the right-hand side are formed in FP64 (they define the discrete
    system); the transforms and the tridiagonal solves run in ``dtype``.  With
    dtype=np.longdouble (x87 extended, 64-bit significand) the oracle's own rounding
    stays far below the FP64 level even where small pivots amplify it, so the result is
    the FP64 system's solution to about 1e-16.  U is returned in FP64.

    sides="neumann" (reading R21): U on every node of each plane, the DCT-I in place of
    the DST-I.
    """
    if W is None:
        nz = np.asarray(f).shape[0] - 2
        W = stencil_weights(scheme, nz, hx, hy, hz, k2, k2_z, k2_zz, gamma)
    if F is None:
        F = rhs(scheme, f, hx, hy, hz, k2, k2_z, gamma, sides)
    Fl = lift(W, F, g_lo, g_hi, sides)
    if sides == "neumann":
        What, minpiv, bad = solve_modal(W, dct2(Fl, dtype), sides)
        U = dct2(What, inverse=True)
    else:
        Fbar = dst2(Fl, dtype)
        What, minpiv, bad = solve_modal(W, Fbar)
        U = dst2(What)    # V is its own inverse
    U = U.astype(np.complex128 if np.iscomplexobj(U) else np.float64)
    return OracleResult(U, W, F, minpiv, bad)


# ----------------------------------------------------------------------------
# Brute force for tiny grids: the assembled 27-diagonal matrix (eq. stencil27)
# and a dense partial-pivot LU solve.
# ----------------------------------------------------------------------------
def assemble_dense(W, nx, ny, nz, sides="dirichlet"):
    """The 27-diagonal matrix row by row (eq. stencil27).  Neumann sides (nx, ny = nodes
    per line, R21): a neighbour beyond a side is its mirror image, whose entry takes the
    weight (the two neighbours of a side node then add up on one column)."""
    n = nx * ny * nz
    A = np.zeros((n, n), dtype=np.result_type(W, np.float64))
    for l in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = i + nx * (j + ny * l)
                for o in (-1, 0, 1):
                    ll = l + o
                    if not 0 <= ll < nz:
                        continue
                    a, b, c, d = W[l, o + 1]
                    for di in (-1, 0, 1):
                        for dj in (-1, 0, 1):
                            ii, jj = i + di, j + dj
                            if sides == "neumann":
                                ii = -ii if ii < 0 else (2 * (nx - 1) - ii if ii >= nx else ii)
                                jj = -jj if jj < 0 else (2 * (ny - 1) - jj if jj >= ny else jj)
                            if not (0 <= ii < nx and 0 <= jj < ny):
                                continue
                            w = (a if (di and dj) else b if di else c if dj else d)
                            A[r, ii + nx * (jj + ny * ll)] += w
    return A


def dense_solve(W, Fl, sides="dirichlet"):
    nz, ny, nx = Fl.shape
    A = assemble_dense(W, nx, ny, nz, sides)
    return np.linalg.solve(A, Fl.reshape(-1)).reshape(nz, ny, nx)


# ----------------------------------------------------------------------------
# Error measures, Section 5.1 (with reading R12 for the two L2 normalisations).
# ----------------------------------------------------------------------------
def closed(U, g_lo=None, g_hi=None, sides="dirichlet"):
    """U with its z-face planes (and, for Dirichlet sides, the zero x/y ring)."""
    nz, ny, nx = U.shape
    if sides == "neumann":
        C = np.zeros((nz + 2, ny, nx), dtype=U.dtype)
        C[1:-1] = U
    else:
        C = np.zeros((nz + 2, ny + 2, nx + 2), dtype=U.dtype)
        C[1:-1, 1:-1, 1:-1] = U
    if g_lo is not None:
        C[0] = g_lo
    if g_hi is not None:
        C[-1] = g_hi
    return C


def error_norms(U, u_exact_interior, W=None, F=None, g_lo=None, g_hi=None, sides="dirichlet"):
    e = u_exact_interior - U
    out = {
        "max_err": float(np.max(np.abs(e))),
        "l2_err_U": float(np.linalg.norm(e) / np.linalg.norm(U)),
        "l2_err_u": float(np.linalg.norm(e) / np.linalg.norm(u_exact_interior)),
    }
    if W is not None and F is not None:
        r = F - apply_operator(W, closed(U, g_lo, g_hi, sides), sides)
        out["l2_res"] = float(np.linalg.norm(r))
        out["rel_res"] = float(np.linalg.norm(r) / np.linalg.norm(lift(W, F, g_lo, g_hi, sides)))
    return out


# ----------------------------------------------------------------------------
# Robin z faces (reading R22).  Section 1 states alpha u_z + beta u = g on the z faces but
# not its discretisation (the paper cites earlier work for it).  The closure here: the
# z-face nodes z_0 and z_{Nz+1} become unknowns and carry the scheme's own row; the ghost
# plane beyond each face is eliminated by the Taylor expansion
#     u(z_0 - h) = u(z_0 + h) - 2h u_z - (h^3/3) u_zzz + O(h^5)
# with u_z = (g - beta u)/alpha from the boundary condition and u_zzz from the z-derivative
# of the equation, u_zzz = f_z - (k^2)_z u - (k^2 + D) u_z, D = delta_x^2 + delta_y^2 on
# the face plane (Dirichlet sides).  The ghost value is then the neighbouring plane plus
# in-plane operators of the face plane and of g, so every modal system stays tridiagonal
# (N_z + 2 rows; only the first and last rows change).  Local error O(h^5) in the ghost
# plane: fourth order near the faces (HELM2 stays second order, HELM6 drops to fourth).
# The boundary rows' right-hand sides take the scheme's operator with one-sided z
# differences (second order for delta_z^2 and delta_z, first order for delta_z^4).
#
# Arrays: U, F of shape (nz+2, ny, nx) for the planes z_0..z_{nz+1}; f on the closed grid
# (nz+2, ny+2, nx+2); g_lo, g_hi closed planes (ny+2, nx+2) with a zero ring; k2, k2_z,
# k2_zz sampled at the nz+4 planes z_{-1}..z_{nz+2}.
# ----------------------------------------------------------------------------
ROBIN_SCHEMES = ("helm2", "helm4", "helm6")


def robin_weights(scheme, nz, hx, hy, hz, k2, k2_z=None, k2_zz=None):
    """Weights of the rows of planes z_0..z_{nz+1}, shape (nz+2, 3, 4)."""
    if scheme not in ROBIN_SCHEMES:
        raise ValueError("Robin z faces: Helmholtz schemes only")
    return stencil_weights(scheme, nz + 2, hx, hy, hz, k2, k2_z, k2_zz)


def _plane_lap(P, hx, hy):
    """delta_x^2 + delta_y^2 of the interior of a closed plane (Dirichlet sides)."""
    return ((P[1:-1, :-2] - 2.0 * P[1:-1, 1:-1] + P[1:-1, 2:]) / (hx * hx)
            + (P[:-2, 1:-1] - 2.0 * P[1:-1, 1:-1] + P[2:, 1:-1]) / (hy * hy))


def _robin_face_rhs(scheme, f, hx, hy, hz, k2f, k2zf, side):
    """The scheme's RHS operator at the face nodes (interior x/y) from f on the closed grid,
    z differences one-sided into the box: delta_z^2 (2, -5, 4, -1), delta_z^4
    (3, -14, 26, -24, 11, -2), delta_z as (-3, 4, -1)/2 (raw, unscaled differences)."""
    g = f if side == "lo" else f[::-1]
    s = 1.0 if side == "lo" else -1.0
    fp = [g[q] for q in range(6)]
    inner = fp[0][1:-1, 1:-1]
    d2z = 2 * fp[0] - 5 * fp[1] + 4 * fp[2] - fp[3]
    d4z = 3 * fp[0] - 14 * fp[1] + 26 * fp[2] - 24 * fp[3] + 11 * fp[4] - 2 * fp[5]
    d1z = s * (-3 * fp[0] + 4 * fp[1] - fp[2]) / 2.0
    P = fp[0]
    d2x = P[1:-1, :-2] - 2.0 * P[1:-1, 1:-1] + P[1:-1, 2:]
    d2y = P[:-2, 1:-1] - 2.0 * P[1:-1, 1:-1] + P[2:, 1:-1]
    if scheme == "helm2":
        return hz * hz * inner
    if scheme == "helm4":
        return hz * hz * (inner + (d2x + d2y + d2z[1:-1, 1:-1]) / 12.0)
    # helm6 (uniform h): the interior formula of rhs() with the z parts one-sided
    h = hz
    # fourth differences of the face plane in x and y, with the one-sided R10 formula on
    # the first and last interior lines (as rhs() does for the interior planes)
    fx = _d4(np.stack([P] * 3), 2)[0]
    fy = _d4(np.stack([P] * 3), 1)[0]
    d2xz = d2z[1:-1, :-2] - 2.0 * d2z[1:-1, 1:-1] + d2z[1:-1, 2:]
    d2yz = d2z[:-2, 1:-1] - 2.0 * d2z[1:-1, 1:-1] + d2z[2:, 1:-1]
    d2xy = (P[:-2, :-2] - 2 * P[:-2, 1:-1] + P[:-2, 2:]
            - 2 * (P[1:-1, :-2] - 2 * P[1:-1, 1:-1] + P[1:-1, 2:])
            + P[2:, :-2] - 2 * P[2:, 1:-1] + P[2:, 2:])
    s2 = d2x + d2y + d2z[1:-1, 1:-1]
    s4 = fx + fy + d4z[1:-1, 1:-1]
    sx = d2xy + d2xz + d2yz
    return h * h * (inner + s2 / 12.0 - s4 / 240.0 + sx / 90.0
                    - h * h * k2f * inner / 20.0 + h ** 3 * k2zf * d1z[1:-1, 1:-1] / 60.0)


def robin_rhs(scheme, f, hx, hy, hz, k2, k2_z=None):
    """F on the planes z_0..z_{nz+1} (shape (nz+2, ny, nx)): interior planes as rhs(), the
    face planes by _robin_face_rhs.  k2, k2_z sampled at z_{-1}..z_{nz+2}."""
    f = _num(f)
    nz = f.shape[0] - 2
    k2 = _num(k2)
    k2z = None if k2_z is None else _num(k2_z)
    F = np.empty((nz + 2, f.shape[1] - 2, f.shape[2] - 2), dtype=f.dtype)
    F[1:-1] = rhs(scheme, f, hx, hy, hz, k2[1:-1], None if k2z is None else k2z[1:-1])
    kz0 = 0.0 if k2z is None else k2z[1]
    kz1 = 0.0 if k2z is None else k2z[-2]
    F[0] = _robin_face_rhs(scheme, f, hx, hy, hz, k2[1], kz0, "lo")
    F[-1] = _robin_face_rhs(scheme, f, hx, hy, hz, k2[-2], kz1, "hi")
    return F


def robin_ghost(nz, hx, hy, hz, k2, k2_z, alpha, beta, f, g_lo, g_hi):
    """The ghost-plane eliminations of both faces.

    Bottom: U_{-1} = U_1 + c_lo(D) U_0 + R_lo, top: U_{nz+2} = U_nz + c_hi(D) U_{nz+1} + R_hi,
    with c(D) = c0 + c1 D an in-plane operator of the face plane:
      c_lo = (h^3/3) k2_z(z_0) - (beta/alpha)(-2h + (h^3/3)(k2(z_0) + D))
      c_hi = -(h^3/3) k2_z(z_{nz+1}) - (beta/alpha)(2h - (h^3/3)(k2(z_{nz+1}) + D))
      R_lo = (1/alpha)(-2h + (h^3/3)(k2 + D)) g_lo - (h^3/3) f_z(z_0)
      R_hi = (1/alpha)(2h - (h^3/3)(k2 + D)) g_hi + (h^3/3) f_z(z_{nz+1})
    f_z one-sided of second order.  Returns ((c0, c1) per face, (R_lo, R_hi) interior planes)."""
    h = hz
    (a0, a1), (b0, b1) = alpha, beta
    k2 = _num(k2)
    k2z = np.zeros_like(k2) if k2_z is None else _num(k2_z)
    f = _num(f)
    kl, kh = k2[1], k2[-2]
    kzl, kzh = k2z[1], k2z[-2]
    c_lo = ((h ** 3 / 3.0) * kzl - (b0 / a0) * (-2.0 * h + (h ** 3 / 3.0) * kl), -(b0 / a0) * (h ** 3 / 3.0))
    c_hi = (-(h ** 3 / 3.0) * kzh - (b1 / a1) * (2.0 * h - (h ** 3 / 3.0) * kh), (b1 / a1) * (h ** 3 / 3.0))
    fz_lo = (-3.0 * f[0] + 4.0 * f[1] - f[2]) / (2.0 * h)
    fz_hi = (3.0 * f[-1] - 4.0 * f[-2] + f[-3]) / (2.0 * h)
    gl, gh = _num(g_lo), _num(g_hi)
    R_lo = ((-2.0 * h + (h ** 3 / 3.0) * kl) * gl[1:-1, 1:-1] + (h ** 3 / 3.0) * _plane_lap(gl, hx, hy)) / a0 \
        - (h ** 3 / 3.0) * fz_lo[1:-1, 1:-1]
    R_hi = ((2.0 * h - (h ** 3 / 3.0) * kh) * gh[1:-1, 1:-1] - (h ** 3 / 3.0) * _plane_lap(gh, hx, hy)) / a1 \
        + (h ** 3 / 3.0) * fz_hi[1:-1, 1:-1]
    return (c_lo, c_hi), (R_lo, R_hi)


def _plane9_open(w, P):
    """9-point weights applied to an interior plane P (zero beyond its edges)."""
    Z = np.zeros((P.shape[0] + 2, P.shape[1] + 2), dtype=P.dtype)
    Z[1:-1, 1:-1] = P
    return _plane9(w, Z)


def solve_robin(scheme, f, hx, hy, hz, k2, k2_z=None, k2_zz=None, alpha=(1.0, 1.0), beta=(0.0, 0.0),
                g_lo=None, g_hi=None, dtype=np.float64, W=None):
    """U on the planes z_0..z_{nz+1} for Robin z faces (reading R22): weights -> F -> ghost
    eliminations -> DST -> modal Thomas with changed first and last rows -> inverse DST.

    Row 0:      (lam^0 + c_lo(mu) lam^-) W_0 + (lam^+ + lam^-) W_1 = Fbar_0 - lam^- Rbar_lo
    Row nz+1:   (lam^- + lam^+) W_nz + (lam^0 + c_hi(mu) lam^+) W_{nz+1} = Fbar_{nz+1} - lam^+ Rbar_hi
    where mu = -(2 - 2 cos th)/hx^2 - (2 - 2 cos ph)/hy^2 is the eigenvalue of D on the mode.
    The lifts lam^- Rbar are applied in physical space (the plane-offset weights on R).
    W: the rows' weights, if given (else robin_weights)."""
    f = _num(f)
    nz = f.shape[0] - 2
    ny, nx = f.shape[1] - 2, f.shape[2] - 2
    if W is None:
        W = robin_weights(scheme, nz, hx, hy, hz, k2, k2_z, k2_zz)
    F = robin_rhs(scheme, f, hx, hy, hz, k2, k2_z)
    z = np.zeros((ny + 2, nx + 2))
    (c_lo, c_hi), (R_lo, R_hi) = robin_ghost(nz, hx, hy, hz, k2, k2_z, alpha, beta, f,
                                             z if g_lo is None else g_lo, z if g_hi is None else g_hi)
    F = np.array(F, copy=True)
    F[0] -= _plane9_open(W[0, 0], R_lo)
    F[-1] -= _plane9_open(W[-1, 2], R_hi)
    Fbar = dst2(F, dtype)
    real = np.real(Fbar[:1, :1, :1]).dtype
    lam = modal_eigenvalues(W, nx, ny, real)
    pi = _pi(real)
    ct = np.cos(pi * np.arange(1, nx + 1, dtype=real) / (nx + 1))[None, :]
    cp = np.cos(pi * np.arange(1, ny + 1, dtype=real) / (ny + 1))[:, None]
    mu = -(2 - 2 * ct) / (hx * hx) - (2 - 2 * cp) / (hy * hy)
    lam = np.array(lam, copy=True)
    lm0, lp0 = lam[0, 0].copy(), lam[0, 2].copy()
    lam[0, 1] = lam[0, 1] + (c_lo[0] + c_lo[1] * mu) * lm0
    lam[0, 2] = lp0 + lm0
    lm1, lp1 = lam[-1, 0].copy(), lam[-1, 2].copy()
    lam[-1, 0] = lm1 + lp1
    lam[-1, 1] = lam[-1, 1] + (c_hi[0] + c_hi[1] * mu) * lp1
    What, minpiv, bad = thomas(lam, Fbar)
    U = dst2(What).astype(np.float64)
    return OracleResult(U, W, F, minpiv, bad)


def assemble_dense_robin(scheme, nx, ny, nz, hx, hy, hz, k2, k2_z=None, k2_zz=None, alpha=(1.0, 1.0),
                         beta=(0.0, 0.0)):
    """The (nz+2)-plane system with the ghost planes substituted, entry by entry: each row
    is eq. stencil27 with the neighbours beyond a face replaced by the ghost formulas of
    robin_ghost (in-plane operators c0 + c1 D of the face plane, D the 5-point in-plane
    second differences), as a dense matrix (no transform involved)."""
    W = robin_weights(scheme, nz, hx, hy, hz, k2, k2_z, k2_zz)
    npl = nx * ny
    nzz = nz + 2
    A = np.zeros((npl * nzz, npl * nzz))

    def plane_op(w):
        """Matrix of the 9-point in-plane operator with weights w (Dirichlet sides)."""
        M = np.zeros((npl, npl))
        a, b, c, d = w
        for j in range(ny):
            for i in range(nx):
                r = i + nx * j
                for dj in (-1, 0, 1):
                    for di in (-1, 0, 1):
                        ii, jj = i + di, j + dj
                        if 0 <= ii < nx and 0 <= jj < ny:
                            M[r, ii + nx * jj] += (a if (di and dj) else b if di else c if dj else d)
        return M

    D = plane_op((0.0, 1.0 / (hx * hx), 1.0 / (hy * hy), -2.0 / (hx * hx) - 2.0 / (hy * hy)))
    (c_lo, c_hi), _ = robin_ghost(nz, hx, hy, hz, k2, k2_z, alpha, beta, np.zeros((nz + 2, 3, 3)),
                                  np.zeros((3, 3)), np.zeros((3, 3)))
    I = np.eye(npl)
    blk = lambda l, ll: (slice(l * npl, (l + 1) * npl), slice(ll * npl, (ll + 1) * npl))  # noqa: E731
    for l in range(nzz):
        for o in (-1, 0, 1):
            M = plane_op(W[l, o + 1])
            ll = l + o
            if 0 <= ll < nzz:
                A[blk(l, ll)] += M
            elif ll < 0:      # U_{-1} = U_1 + (c0 + c1 D) U_0 (+ data)
                A[blk(l, 1)] += M
                A[blk(l, 0)] += M @ (c_lo[0] * I + c_lo[1] * D)
            else:             # U_{nz+2} = U_nz + (c0 + c1 D) U_{nz+1} (+ data)
                A[blk(l, nz)] += M
                A[blk(l, nz + 1)] += M @ (c_hi[0] * I + c_hi[1] * D)
    return A
