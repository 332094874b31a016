"""Analytic test problems and synthetic workload configurations.

Every problem is the Helmholtz equation  u_xx + u_yy + u_zz + k(z)^2 u = f
(or the convection-diffusion equation u_xx + u_yy + u_zz + gamma u_z = f) on a
box with N_alpha interior grid points per axis and h_alpha = L_alpha/(N_alpha+1)
(paper, Section 2).  Fields are float64 torch tensors on the closed grid,
indexed [z, y, x] (x fastest), so interior point (i, j, l) is element
[l, j, i] with 1 <= i <= N_x etc.  Dirichlet data on the two z faces is given as
whole closed planes [y, x]; the x and y faces are homogeneous.

The samples k2 = k^2, k2_z = (k^2)_z and k2_zz = (k^2)_zz are taken at the
N_z + 2 planes z_0 .. z_{N_z+1}, from the analytic k(z).
"""
import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import torch

from .gen import gaussian, uniform01, uniform_pm1


@dataclass
class KProfile:
    """k(z) with its first two derivatives (all callables on numpy arrays; complex values
    describe an absorbing medium)."""

    k: Callable
    dk: Callable
    d2k: Callable
    name: str = ""

    def samples(self, z):
        k, dk, d2k = self.k(z), self.dk(z), self.d2k(z)
        k2 = k * k
        k2_z = 2.0 * k * dk
        k2_zz = 2.0 * dk * dk + 2.0 * k * d2k
        dt = np.complex128 if np.iscomplexobj(k2) else np.float64  # complex k: absorbing media
        return (np.ascontiguousarray(k2, dtype=dt),
                np.ascontiguousarray(k2_z, dtype=dt),
                np.ascontiguousarray(k2_zz, dtype=dt))


def k_const(k0):
    return KProfile(lambda z: np.full_like(z, k0, dtype=np.float64),
                    lambda z: np.zeros_like(z, dtype=np.float64),
                    lambda z: np.zeros_like(z, dtype=np.float64), f"k={k0}")


@dataclass
class Problem:
    name: str
    scheme: str                     # "helm2" | "helm4" | "helm6" | "cd4"
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    f: torch.Tensor                 # [nrhs, nz+2, ny+2, nx+2]
    g_lo: Optional[torch.Tensor] = None   # [nrhs, ny+2, nx+2] or None (zero)
    g_hi: Optional[torch.Tensor] = None
    k2: Optional[np.ndarray] = None       # [nz+2]
    k2_z: Optional[np.ndarray] = None
    k2_zz: Optional[np.ndarray] = None
    gamma: float = 0.0
    u_exact: Optional[torch.Tensor] = None  # [nrhs, nz+2, ny+2, nx+2] or None
    meta: dict = field(default_factory=dict)
    # "dirichlet": u = 0 on the x/y faces; "neumann": du/dn = 0 there, and every x/y node of
    # the closed grid is an unknown
    sides: str = "dirichlet"
    # Robin z faces: ((alpha_lo, alpha_hi), (beta_lo, beta_hi)) of alpha u_z + beta u = g, or
    # None (Dirichlet).  Then g_lo/g_hi are the data g, the k^2 samples cover z_{-1}..z_{nz+2}
    # and the unknowns include the z-face nodes (nz + 2 planes)
    robin: Optional[tuple] = None

    @property
    def nrhs(self):
        return self.f.shape[0]

    @property
    def unknowns(self):
        if self.sides == "neumann":
            return (self.nx + 2) * (self.ny + 2) * self.nz
        if self.robin is not None:
            return self.nx * self.ny * (self.nz + 2)
        return self.nx * self.ny * self.nz


def _axis(n, h, lo=0.0, device="cpu"):
    return lo + h * torch.arange(n + 2, dtype=torch.float64, device=device)


def _outer3(fz, fy, fx):
    return fz[:, None, None] * fy[None, :, None] * fx[None, None, :]


def _zsamples(prob_nz, hz, prof):
    z = hz * np.arange(prob_nz + 2, dtype=np.float64)
    return prof.samples(z)


# ----------------------------------------------------------------------------
# The paper's variable-coefficient test problem (Section 5.1 and the tables of
# Section 5.2.2): k(z) = a - b sin(c z), u = sin(beta x) sin(gamma y) e^{-k/c},
# f = -b(2a + c) sin(cz) e^{-k/c} sin(beta x) sin(gamma y), on [0, pi]^3.
# ----------------------------------------------------------------------------
def paper_variable_k(n, scheme, a=10.0, b=9.0, c=10.0, beta=10.0, gam=9.0, device="cpu"):
    h = math.pi / (n + 1)
    prof = KProfile(lambda z: a - b * np.sin(c * z),
                    lambda z: -b * c * np.cos(c * z),
                    lambda z: b * c * c * np.sin(c * z), "a-b sin(cz)")
    k2, k2z, k2zz = _zsamples(n, h, prof)
    x = _axis(n, h, device=device)
    z = x
    kz = a - b * torch.sin(c * z)
    ez = torch.exp(-kz / c)
    sx, sy = torch.sin(beta * x), torch.sin(gam * x)
    u = _outer3(ez, sy, sx)
    f = _outer3(-b * (2 * a + c) * torch.sin(c * z) * ez, sy, sx)
    return Problem(f"paper_vark_{scheme}_{n}", scheme, n, n, n, h, h, h,
                   f=f[None], g_lo=u[0][None].clone(), g_hi=u[-1][None].clone(),
                   k2=k2, k2_z=k2z, k2_zz=k2zz, u_exact=u[None])


# ----------------------------------------------------------------------------
# The paper's convection-diffusion test problem (Section 5.2.3): gamma = -100
# on [0, sqrt 2]^2 x [0, 1], f = 0, u = S at z = 0 and 2S at z = 1 with
# S = sin(pi x/sqrt 2) sin(pi y/sqrt 2).
# ----------------------------------------------------------------------------
def paper_cd(n, gamma=-100.0, device="cpu"):
    L = math.sqrt(2.0)
    hx = L / (n + 1)
    hz = 1.0 / (n + 1)
    x = _axis(n, hx, device=device)
    z = _axis(n, hz, device=device)
    s = torch.sin(math.pi * x / L)
    sigma = math.sqrt(math.pi ** 2 + gamma * gamma / 4.0)
    ez = (torch.exp(-gamma * z / 2) * (2 * math.exp(gamma / 2) * torch.sinh(sigma * z)
                                       + torch.sinh(sigma * (1 - z))) / math.sinh(sigma))
    u = _outer3(ez, s, s)
    f = torch.zeros_like(u)
    plane = _outer3(torch.ones(1, dtype=torch.float64, device=device), s, s)[0]
    return Problem(f"paper_cd_{n}", "cd4", n, n, n, hx, hx, hz, f=f[None],
                   g_lo=plane[None].clone(), g_hi=(2 * plane)[None].clone(),
                   gamma=gamma, u_exact=u[None])


# ----------------------------------------------------------------------------
# Manufactured smooth solution on the unit cube, homogeneous on every face:
# u* = sin(pi x) sin(2 pi y) sin(3 pi z), f* = (k(z)^2 - 14 pi^2) u*.
# ----------------------------------------------------------------------------
def manufactured_sin3(nx, ny, nz, scheme, prof, device="cpu", box=None, planes=None):
    """``planes`` restricts the fields to the closed-grid z-planes 0..planes-1."""
    if box is None:
        box = (1.0, 1.0, 1.0)
    hx, hy, hz = box[0] / (nx + 1), box[1] / (ny + 1), box[2] / (nz + 1)
    x, y, z = _axis(nx, hx, device=device), _axis(ny, hy, device=device), _axis(nz, hz, device=device)
    if planes is not None:
        z = z[:planes]
    sx = torch.sin(math.pi * x / box[0])
    sy = torch.sin(2 * math.pi * y / box[1])
    sz = torch.sin(3 * math.pi * z / box[2])
    lap = -math.pi ** 2 * (1.0 / box[0] ** 2 + 4.0 / box[1] ** 2 + 9.0 / box[2] ** 2)
    k2, k2z, k2zz = _zsamples(nz, hz, prof)
    k2t = torch.as_tensor(k2[: z.shape[0]], device=device)
    u = _outer3(sz, sy, sx)
    f = _outer3((k2t + lap) * sz, sy, sx)
    return Problem(f"sin3_{scheme}_{nx}x{ny}x{nz}", scheme, nx, ny, nz, hx, hy, hz,
                   f=f[None], k2=k2, k2_z=k2z, k2_zz=k2zz, u_exact=u[None])


def manufactured_cos2(nx, ny, nz, scheme, prof, device="cpu", box=None):
    """Neumann sides: u = cos(pi x/Lx) cos(2 pi y/Ly) (sin(3 pi z/Lz) + cos(pi z/Lz)/2).

    du/dn = 0 on the x and y faces (every odd x/y derivative vanishes there) and non-zero
    Dirichlet data u(x, y, 0), u(x, y, Lz) on the z faces."""
    if box is None:
        box = (1.0, 1.0, 1.0)
    hx, hy, hz = box[0] / (nx + 1), box[1] / (ny + 1), box[2] / (nz + 1)
    x, y, z = _axis(nx, hx, device=device), _axis(ny, hy, device=device), _axis(nz, hz, device=device)
    cx = torch.cos(math.pi * x / box[0])
    cy = torch.cos(2 * math.pi * y / box[1])
    a, b = 3 * math.pi / box[2], math.pi / box[2]
    gz = torch.sin(a * z) + 0.5 * torch.cos(b * z)
    gzz = -a * a * torch.sin(a * z) - 0.5 * b * b * torch.cos(b * z)
    lapxy = -math.pi ** 2 * (1.0 / box[0] ** 2 + 4.0 / box[1] ** 2)
    k2, k2z, k2zz = _zsamples(nz, hz, prof)
    k2t = torch.as_tensor(k2, device=device)
    u = _outer3(gz, cy, cx)
    f = _outer3((k2t + lapxy) * gz + gzz, cy, cx)
    return Problem(f"cos2_{scheme}_{nx}x{ny}x{nz}", scheme, nx, ny, nz, hx, hy, hz,
                   f=f[None], g_lo=u[None, 0].clone(), g_hi=u[None, -1].clone(), k2=k2, k2_z=k2z,
                   k2_zz=k2zz, u_exact=u[None], sides="neumann")


def neumann_noise_problem(nx, ny, nz, scheme, seed, device="cpu", nrhs=1, boundary=True):
    """Neumann sides, random f on every node of the closed grid and random z-face planes
    (all nodes); k(z) = 6 + 2 sin 3z; the grids of ``noise_problem``."""
    p = noise_problem(nx, ny, nz, scheme, seed, device=device, boundary=False, nrhs=nrhs)
    if boundary:
        p.g_lo = uniform_pm1(seed + 1, (nrhs, ny + 2, nx + 2), device=device)
        p.g_hi = uniform_pm1(seed + 2, (nrhs, ny + 2, nx + 2), device=device)
    p.sides = "neumann"
    p.name = f"neu_{scheme}_{nx}x{ny}x{nz}_s{seed}"
    return p


def _zero_ring_(f):
    """Set the x and y faces of closed-grid fields to zero (homogeneous Dirichlet)."""
    f[..., 0, :] = 0
    f[..., -1, :] = 0
    f[..., :, 0] = 0
    f[..., :, -1] = 0
    return f


K_CONFIG2 = KProfile(lambda z: 20.0 * (1 + 0.5 * np.sin(2 * np.pi * z)),
                     lambda z: 20.0 * np.pi * np.cos(2 * np.pi * z),
                     lambda z: -40.0 * np.pi ** 2 * np.sin(2 * np.pi * z), "20(1+0.5 sin 2 pi z)")
K_CONFIG3 = KProfile(lambda z: 50.0 * (1 + 0.3 * z),
                     lambda z: np.full_like(z, 15.0),
                     lambda z: np.zeros_like(z), "50(1+0.3z)")
K_CONFIG5 = KProfile(lambda z: 80.0 * np.exp(-z),
                     lambda z: -80.0 * np.exp(-z),
                     lambda z: 80.0 * np.exp(-z), "80 exp(-z)")


def config1(device="cpu"):
    """4th-order compact Helmholtz, k = 10, unit cube, 63^3, RHS from u*."""
    p = manufactured_sin3(63, 63, 63, "helm4", k_const(10.0), device=device)
    p.name = "helm4_k10_63"
    return p


def _noise_rhs(p, seeds, kind, scale_smooth=1.0, device="cpu"):
    shape = tuple(p.f.shape[1:])
    base = p.f[0]
    p.u_exact = None
    out = torch.empty((len(seeds),) + shape, dtype=torch.float64, device=device)
    for r, s in enumerate(seeds):
        xi = uniform_pm1(s, shape, device=device) if kind == "uniform" else gaussian(s, shape, device=device)
        torch.add(xi, base, alpha=scale_smooth, out=out[r])
        del xi
    p.f = out
    return p


def config2(n=255, device="cpu"):
    """6th-order, k = 20(1 + 0.5 sin 2 pi z), f = f*(u*) + U[-1, 1] noise (seed 102)."""
    p = manufactured_sin3(n, n, n, "helm6", K_CONFIG2, device=device)
    p.name = f"helm6_ksin_{n}"
    return _noise_rhs(p, [102], "uniform", device=device)


def config3(n=511, device="cpu"):
    """6th-order, k = 50(1 + 0.3 z), f ~ N(0, 1) (seed 103)."""
    p = manufactured_sin3(n, n, n, "helm6", K_CONFIG3, device=device)
    p.name = f"helm6_klin_{n}"
    return _noise_rhs(p, [103], "gauss", scale_smooth=0.0, device=device)


def config5(n=1023, nrhs=4, device="cpu", planes=None):
    """6th-order, k = 80 exp(-z), f_r = f*(u*) + U[-1, 1] noise (seeds 105000 + r).

    ``planes`` keeps only the closed-grid z-planes 0..planes-1 (same values)."""
    p = manufactured_sin3(n, n, n, "helm6", K_CONFIG5, device=device, planes=planes)
    p.name = f"helm6_kexp_{n}_x{nrhs}"
    return _noise_rhs(p, [105000 + r for r in range(nrhs)], "uniform", device=device)


K_CONFIG5_ABSORB = KProfile(lambda z: 80.0 * (1.0 + 0.05j) * np.exp(-z),
                            lambda z: -80.0 * (1.0 + 0.05j) * np.exp(-z),
                            lambda z: 80.0 * (1.0 + 0.05j) * np.exp(-z), "80(1+0.05i) exp(-z)")


def config5_absorbing(n=1023, nrhs=2, device="cpu"):
    """The 1023^3 workload in an absorbing medium: k = 80 (1 + 0.05 i) exp(-z); complex
    right-hand sides f_r = f*(u*) + U[-1, 1] noise + i U[-1, 1] noise (seeds 105100 + r,
    105200 + r)."""
    p = manufactured_sin3(n, n, n, "helm6", K_CONFIG5_ABSORB, device=device)
    p.name = f"helm6_kexp_absorbing_{n}_x{nrhs}"
    base = p.f[0]
    p.u_exact = None
    shape = tuple(base.shape)
    out = torch.empty((nrhs,) + shape, dtype=torch.complex128, device=device)
    for r in range(nrhs):
        out[r] = base + torch.complex(uniform_pm1(105100 + r, shape, device=device),
                                      uniform_pm1(105200 + r, shape, device=device))
    p.f = out
    return p


def noise_problem(nx, ny, nz, scheme, seed, device="cpu", box=None, gamma=-7.5,
                  prof=None, boundary=True, nrhs=1):
    """Random RHS and z-face data on a (possibly non-cubic) grid; variable k(z)."""
    if box is None:
        box = (1.0, 1.3, 0.9) if scheme != "helm6" else None
    if scheme == "helm6":
        h = 1.0 / (nz + 1)
        box = ((nx + 1) * h, (ny + 1) * h, 1.0)
    hx, hy, hz = box[0] / (nx + 1), box[1] / (ny + 1), box[2] / (nz + 1)
    if prof is None:
        prof = KProfile(lambda z: 6.0 + 2.0 * np.sin(3.0 * z),
                        lambda z: 6.0 * np.cos(3.0 * z),
                        lambda z: -18.0 * np.sin(3.0 * z), "6+2 sin 3z")
    k2, k2z, k2zz = _zsamples(nz, hz, prof)
    shape = (nrhs, nz + 2, ny + 2, nx + 2)
    f = uniform_pm1(seed, shape, device=device)
    g_lo = g_hi = None
    if boundary:
        g_lo = _zero_ring_(uniform_pm1(seed + 1, (nrhs, ny + 2, nx + 2), device=device))
        g_hi = _zero_ring_(uniform_pm1(seed + 2, (nrhs, ny + 2, nx + 2), device=device))
    return Problem(f"noise_{scheme}_{nx}x{ny}x{nz}_s{seed}", scheme, nx, ny, nz, hx, hy, hz,
                   f=f, g_lo=g_lo, g_hi=g_hi, k2=k2, k2_z=k2z, k2_zz=k2zz,
                   gamma=gamma if scheme == "cd4" else 0.0)


# absorbing medium: complex k(z) = 6 + 2 sin 3z + i (1 + 0.5 cos 2z)
K_ABSORB = KProfile(lambda z: (6.0 + 2.0 * np.sin(3.0 * z)) + 1j * (1.0 + 0.5 * np.cos(2.0 * z)),
                    lambda z: 6.0 * np.cos(3.0 * z) - 1j * np.sin(2.0 * z),
                    lambda z: -18.0 * np.sin(3.0 * z) - 2j * np.cos(2.0 * z), "6+2 sin 3z + i(1+0.5 cos 2z)")


def complex_noise_problem(nx, ny, nz, scheme, seed, device="cpu", boundary=True, nrhs=1, prof=None):
    """Complex k(z) (absorbing medium, default ``K_ABSORB``), complex random right-hand
    sides and z-face data (complex128 tensors; real and imaginary parts U[-1, 1])."""
    p = noise_problem(nx, ny, nz, scheme, seed, device=device, boundary=False, nrhs=nrhs,
                      prof=K_ABSORB if prof is None else prof)
    shape = tuple(p.f.shape)
    p.f = torch.complex(p.f, uniform_pm1(seed + 7, shape, device=device))
    if boundary:
        pl = (nrhs, ny + 2, nx + 2)
        p.g_lo = _zero_ring_(torch.complex(uniform_pm1(seed + 1, pl, device=device),
                                           uniform_pm1(seed + 8, pl, device=device)))
        p.g_hi = _zero_ring_(torch.complex(uniform_pm1(seed + 2, pl, device=device),
                                           uniform_pm1(seed + 9, pl, device=device)))
    p.name = f"cplx_{scheme}_{nx}x{ny}x{nz}_s{seed}"
    return p


def batch_members(seed=104, count=64, sizes=(63, 127, 255), device="cpu", make_fields=True):
    """Uneven batch: per-axis sizes drawn from ``sizes``; schemes HELM4/HELM6/CD4 in turn.

    Helmholtz members have constant k0 ~ U[5, 60]; CD members gamma ~ U[-100, -5].
    HELM4 and CD4 live on the unit cube (per-axis h); HELM6 needs one h, so its box is
    [0, (N_x+1)h] x [0, (N_y+1)h] x [0, 1] with h = 1/(N_z+1).  f ~ U[-1, 1], zero z-face data.
    """
    draws = uniform01(seed, (count, 5)).numpy()
    schemes = ("helm4", "helm6", "cd4")
    out = []
    for i in range(count):
        nx, ny, nz = (sizes[min(int(draws[i, a] * len(sizes)), len(sizes) - 1)] for a in range(3))
        scheme = schemes[i % 3]
        if scheme == "helm6":
            h = 1.0 / (nz + 1)
            hx = hy = hz = h
        else:
            hx, hy, hz = 1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1)
        k0 = 5.0 + 55.0 * draws[i, 3]
        gamma = -100.0 + 95.0 * draws[i, 4]
        prof = k_const(k0)
        k2, k2z, k2zz = _zsamples(nz, hz, prof)
        sub = seed * 1000 + i
        f = (uniform_pm1(sub, (1, nz + 2, ny + 2, nx + 2), device=device) if make_fields
             else None)
        out.append(Problem(f"batch{i}_{scheme}_{nx}x{ny}x{nz}", scheme, nx, ny, nz, hx, hy, hz,
                           f=f, k2=None if scheme == "cd4" else k2,
                           k2_z=None if scheme == "cd4" else k2z,
                           k2_zz=None if scheme == "cd4" else k2zz,
                           gamma=gamma if scheme == "cd4" else 0.0,
                           meta={"k0": k0 if scheme != "cd4" else None, "seed": sub}))
    return out


# ----------------------------------------------------------------------------
# Robin z faces: alpha u_z + beta u = g on z = 0 and z = L_z (Section 1, eq. bc).
# The k^2 samples then cover z_{-1}..z_{nz+2} (the rows of the face nodes reach one plane
# beyond each face).
# ----------------------------------------------------------------------------
ROBIN_DEFAULT = ((1.0, 0.7), (2.0, -1.5))


def _zsamples_robin(nz, hz, prof):
    z = hz * np.arange(-1, nz + 3, dtype=np.float64)
    return prof.samples(z)


def robin_noise_problem(nx, ny, nz, scheme, seed, device="cpu", nrhs=1, robin=ROBIN_DEFAULT, prof=None):
    """Random f on the closed grid and random face data g (zero ring), Robin z faces,
    k(z) = 6 + 2 sin 3z by default; the grids of ``noise_problem``."""
    p = noise_problem(nx, ny, nz, scheme, seed, device=device, boundary=True, nrhs=nrhs, prof=prof)
    if prof is None:
        prof = KProfile(lambda z: 6.0 + 2.0 * np.sin(3.0 * z), lambda z: 6.0 * np.cos(3.0 * z),
                        lambda z: -18.0 * np.sin(3.0 * z), "6+2 sin 3z")
    p.k2, p.k2_z, p.k2_zz = _zsamples_robin(nz, p.hz, prof)
    p.robin = robin
    p.name = f"robin_{scheme}_{nx}x{ny}x{nz}_s{seed}"
    return p


def manufactured_robin(n, scheme, robin=ROBIN_DEFAULT, prof=None, device="cpu"):
    """u = sin(pi x) sin(2 pi y) Z(z), Z = cos(1.3 z) + sin(2.1 z)/2 on the unit cube with
    Robin data g = alpha Z'(z_face) + beta Z(z_face) (times the x/y factor) on both z faces,
    f = Z'' + (k^2 - 5 pi^2) Z (times the factor); u_exact on the planes z_0..z_{n+1}."""
    if prof is None:
        prof = KProfile(lambda z: 4.0 + np.sin(2 * np.pi * z), lambda z: 2 * np.pi * np.cos(2 * np.pi * z),
                        lambda z: -4 * np.pi ** 2 * np.sin(2 * np.pi * z), "4 + sin 2 pi z")
    h = 1.0 / (n + 1)
    (a0, a1), (b0, b1) = robin
    x = _axis(n, h, device=device)
    z = x
    k2, k2z, k2zz = _zsamples_robin(n, h, prof)
    Z = torch.cos(1.3 * z) + 0.5 * torch.sin(2.1 * z)
    Zz = -1.3 * torch.sin(1.3 * z) + 1.05 * torch.cos(2.1 * z)
    Zzz = -1.69 * torch.cos(1.3 * z) - 2.205 * torch.sin(2.1 * z)
    sx, sy = torch.sin(math.pi * x), torch.sin(2 * math.pi * x)
    k2t = torch.as_tensor(k2[1:-1], device=device)
    u = _outer3(Z, sy, sx)
    f = _outer3(Zzz + (k2t - 5.0 * math.pi ** 2) * Z, sy, sx)
    one = torch.ones(1, dtype=torch.float64, device=device)
    g_lo = _outer3((a0 * Zz[0] + b0 * Z[0]) * one, sy, sx)[0]
    g_hi = _outer3((a1 * Zz[-1] + b1 * Z[-1]) * one, sy, sx)[0]
    return Problem(f"robin_sin_{scheme}_{n}", scheme, n, n, n, h, h, h, f=f[None], g_lo=g_lo[None],
                   g_hi=g_hi[None], k2=k2, k2_z=k2z, k2_zz=k2zz, u_exact=u[None], robin=robin)
