"""Shared pieces of the paper-table tests (CPU pins and GPU runs): the one-mode reduction
of the paper's test problems and the bars against printed digits.

Test infrastructure: uses the oracle's weight formulas (Sections 3.2-3.5) and numpy/scipy.
"""
import json
import math
import os

import numpy as np
import scipy.linalg

import oracle as O

EPS = np.finfo(np.float64).eps


def oracle_tables(golden_dir):
    """Errors of the oracle on the paper's problems, stored by make_oracle_tables.py."""
    with open(os.path.join(golden_dir, "oracle_tables.json")) as fh:
        return json.load(fh)


def printed_unit(v, digits=8):
    """One unit of the last of ``digits`` printed significant digits of v."""
    return 10.0 ** (math.floor(math.log10(abs(v))) - (digits - 1))


def _tridiag_solve_ld(lo, di, up, F):
    """Tridiagonal solve in extended precision: an FP64 banded LU, then two refinement
    steps with the residual formed in extended precision (exact to far below 1e-16)."""
    ab = np.array([np.r_[0.0, np.asarray(up[:-1], np.float64)], np.asarray(di, np.float64),
                   np.r_[np.asarray(lo[1:], np.float64), 0.0]])
    w = scipy.linalg.solve_banded((1, 1), ab, np.asarray(F, np.float64)).astype(np.longdouble)
    for _ in range(2):
        r = F - di * w
        r[1:] -= lo[1:] * w[:-1]
        r[:-1] -= up[:-1] * w[1:]
        w = w + scipy.linalg.solve_banded((1, 1), ab, np.asarray(r, np.float64)).astype(np.longdouble)
    return w


def single_mode(scheme, n):
    """Exact discrete errors of the paper's test problems by a reduction to one sine mode.

    * HELM2/HELM4 (Section 5.2.2, Tables 4 and 5): on [0, pi]^3 with h = pi/(n+1), f and u
      are Z(z) sin(10 x) sin(9 y), and the samples sin(beta x_i) are the DST-I mode beta of
      Section 3.6.
    * CD4 (Section 5.2.3): f = 0 and the z-face data are S and 2S with
      S = sin(pi x/sqrt 2) sin(pi y/sqrt 2), mode (1, 1) on [0, sqrt 2]^2.

    The in-plane 9-point blocks act on the mode by the eigenvalue formula of Section 3.6,
    and the in-plane second differences of the HELM4 right-hand side (eq. scheme4) by
    -(2 - 2 cos theta).  So the 3-D discrete solution is w_l times the mode, with w the
    solution of that mode's tridiagonal system, solved here in extended precision without
    any transform.

    Returns max_err, l2_err_U (normalised by U), l2_err_u (by u), cond (inf-norm condition
    number of the mode's tridiagonal matrix) and umax = max |u|.  An FP64 direct solve can
    move U by up to about cond * eps * umax, which bounds how many printed digits any FP64
    code can reproduce."""
    ld = np.longdouble
    if scheme == "cd4":
        gamma = -100.0
        L = math.sqrt(2.0)
        hx = L / (n + 1)
        hz = 1.0 / (n + 1)
        W = O.stencil_weights("cd4", n, hx, hx, hz, gamma=gamma).astype(ld)
        th = ph = ld(np.pi) / ld(n + 1)
        F = np.zeros(n, dtype=ld)
        z = np.arange(n + 2) * hz
        sigma = math.sqrt(math.pi ** 2 + gamma * gamma / 4)
        uz = (np.exp(-gamma * z / 2) * (2 * math.exp(gamma / 2) * np.sinh(sigma * z)
                                         + np.sinh(sigma * (1 - z))) / math.sinh(sigma))
        g_lo, g_hi = 1.0, 2.0
        i = np.arange(1, n + 1)
        sx = sy = np.sin(math.pi * i / (n + 1))
    else:
        a, b, c, beta, gam = 10.0, 9.0, 10.0, 10, 9
        h = math.pi / (n + 1)
        z = np.arange(n + 2) * h
        k = a - b * np.sin(c * z)
        W = O.stencil_weights(scheme, n, h, h, h, k * k).astype(ld)
        th, ph = ld(beta) * ld(h), ld(gam) * ld(h)
        uz = np.exp(-(a - b * np.sin(c * z)) / c)                 # u / (sin sin)
        fz = (-b * (2 * a + c) * np.sin(c * z) * uz).astype(ld)   # f / (sin sin)
        hh = ld(h) * ld(h)
        if scheme == "helm2":
            F = hh * fz[1:-1]
        else:
            p2 = (2 - 2 * np.cos(th)) + (2 - 2 * np.cos(ph))
            F = hh * (fz[1:-1] + (fz[:-2] - 2 * fz[1:-1] + fz[2:] - p2 * fz[1:-1]) / 12)
        g_lo, g_hi = uz[0], uz[-1]
        i = np.arange(1, n + 1)
        sx, sy = np.sin(beta * i * h), np.sin(gam * i * h)
    lam = (4 * W[..., 0] * np.cos(th) * np.cos(ph) + 2 * W[..., 1] * np.cos(th)
           + 2 * W[..., 2] * np.cos(ph) + W[..., 3])
    F = np.array(F, dtype=ld)
    F[0] -= lam[0, 0] * ld(g_lo)
    F[-1] -= lam[-1, 2] * ld(g_hi)
    w = _tridiag_solve_ld(lam[:, 0], lam[:, 1], lam[:, 2], F)
    smax = float(np.max(np.abs(sx)) * np.max(np.abs(sy)))
    e = w - uz[1:-1].astype(ld)
    u = uz[1:-1].astype(ld)
    A = (np.diag(np.asarray(lam[:, 1], np.float64)) + np.diag(np.asarray(lam[1:, 0], np.float64), -1)
         + np.diag(np.asarray(lam[:-1, 2], np.float64), 1))
    return {"max_err": float(np.max(np.abs(e))) * smax,
            "l2_err_U": float(np.sqrt(np.sum(e * e) / np.sum(w * w))),
            "l2_err_u": float(np.sqrt(np.sum(e * e) / np.sum(u * u))),
            "cond": float(np.linalg.cond(A, np.inf)),
            "umax": float(np.max(np.abs(uz))) * smax}


def fp64_bound(mode):
    """How far rounding in an FP64 direct solve can move the printed errors: max-err by
    cond eps umax (absolute); the L2 errors (norms relative to U or u) by cond eps."""
    return {"max_err": mode["cond"] * EPS * mode["umax"], "l2": mode["cond"] * EPS}


def printed_bar(printed, bound):
    """0.75 of the last printed digit, plus the FP64 bound of the problem (the printed
    eighth digit of the largest rows lies below what an FP64 solve resolves)."""
    return 0.75 * printed_unit(printed) + bound
