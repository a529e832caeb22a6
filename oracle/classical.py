"""The classical fast Ewald method (Methods, "Classical fast Ewald methods",
eqs. cem and cemparameters) as a plain reference, for the same-hardware
baseline: the Gaussian splitting kernel with the cardinal B-spline of order P
as spreading/interpolation window, through the same five steps as the ESP
reference (spread, DFT, diagonal scaling, inverse DFT, interpolation with the
analytic window derivative).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never does.

  * Splitting kernel: chi(t) = 2 sqrt(alpha/pi) exp(-alpha t^2) with t = r/rc
    (oracle.split.GaussianSplit; the paper's constant written without its
    square root is read as this, the normalisation that makes int chi = 1),
    so S^(k) = exp(-k^2 rc^2/(4 alpha))/k^2, classical Ewald with
    beta = sqrt(alpha)/rc, and S(0) = chi(0)/(4 pi rc).
  * Window: the centred cardinal B-spline B_P (support [-P/2, P/2]) in grid
    units, written out by its truncated-power formula
        B_P(x) = 1/(P-1)! sum_{k=0..P} (-1)^k C(P, k) (x + P/2 - k)_+^(P-1),
    with derivative B_P'(x) = B_{P-1}(x + 1/2) - B_{P-1}(x - 1/2). Its
    transform in physical units is h (sin(xi h/2)/(xi h/2))^P (eq. cem).
  * Placement as in the ESP reference: the P points l0 .. l0 + P - 1 with
    l0 = floor(u - P/2) + 1, weight B_P(u - l).
  * Influence function as in the ESP reference: p_m = h^6 S^(k)/(L^3 phi^(k)^2).
  * Parameters (eq. cemparameters): alpha = log(1/eps),
    n_f = 2 ceil(alpha L/(pi rc)).
"""
from __future__ import annotations

import math

import numpy as np

from .fivestep import dft3
from .split import GaussianSplit, S_hat


def bspline(x, P):
    """Centred cardinal B-spline of order P at x (grid units)."""
    x = np.asarray(x, np.float64) + 0.5 * P
    out = np.zeros_like(x)
    for k in range(P + 1):
        out += (-1) ** k * math.comb(P, k) * np.maximum(x - k, 0.0) ** (P - 1)
    out /= math.factorial(P - 1)
    return np.where((x > 0) & (x < P), out, 0.0)


def dbspline(x, P):
    x = np.asarray(x, np.float64)
    return bspline(x + 0.5, P - 1) - bspline(x - 0.5, P - 1)


def parameters(L, tol, rc):
    """alpha and the minimal grid of eq. cemparameters."""
    alpha = math.log(1.0 / tol)
    return alpha, 2 * math.ceil(alpha * L / (math.pi * rc))


def window(u, P, n):
    """Grid indices (mod n), weights and d(weight)/du for one axis."""
    l0 = np.floor(u - P / 2.0).astype(np.int64) + 1
    pts = l0[:, None] + np.arange(P)[None, :]
    disp = u[:, None] - pts
    return np.mod(pts, n), bspline(disp, P), dbspline(disp, P)


def phi_hat_1d(xi, P, h):
    x = np.asarray(xi, np.float64) * h / 2.0
    return h * np.sinc(x / math.pi) ** P


def influence(n, L, P, alpha, rc):
    h = L / n
    split = GaussianSplit(alpha, rc)
    k = np.arange(n)
    m = np.where(k < n // 2, k, k - n).astype(np.float64)
    ph = phi_hat_1d(2 * math.pi * m / L, P, h)
    m2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    m2[0, 0, 0] = 1.0
    S = S_hat(split, 2 * math.pi * np.sqrt(m2) / L)
    phi2 = (ph[:, None, None] * ph[None, :, None] * ph[None, None, :]) ** 2
    p = h ** 6 * S / (L ** 3 * phi2)
    p[0, 0, 0] = 0.0
    return p


def spread(pos, q, L, n, P, chunk=20000):
    u = np.mod(np.asarray(pos, np.float64), L) * (n / L)
    b = np.zeros(n ** 3)
    for s in range(0, len(u), chunk):
        us, qs = u[s:s + chunk], q[s:s + chunk]
        ix, wx, _ = window(us[:, 0], P, n)
        iy, wy, _ = window(us[:, 1], P, n)
        iz, wz, _ = window(us[:, 2], P, n)
        flat = (ix[:, :, None, None] * n + iy[:, None, :, None]) * n + iz[:, None, None, :]
        w = qs[:, None, None, None] * wx[:, :, None, None] * wy[:, None, :, None] * wz[:, None, None, :]
        b += np.bincount(flat.ravel(), weights=w.ravel(), minlength=n ** 3)
    return b.reshape(n, n, n)


def interpolate(pos, L, n, P, cgrid, chunk=20000):
    u = np.mod(np.asarray(pos, np.float64), L) * (n / L)
    cf = cgrid.ravel()
    ut = np.zeros(len(u))
    g = np.zeros((len(u), 3))
    for s in range(0, len(u), chunk):
        us = u[s:s + chunk]
        ix, wx, dx = window(us[:, 0], P, n)
        iy, wy, dy = window(us[:, 1], P, n)
        iz, wz, dz = window(us[:, 2], P, n)
        flat = (ix[:, :, None, None] * n + iy[:, None, :, None]) * n + iz[:, None, None, :]
        cv = cf[flat]
        ut[s:s + chunk] = np.einsum("iabc,ia,ib,ic->i", cv, wx, wy, wz)
        g[s:s + chunk, 0] = np.einsum("iabc,ia,ib,ic->i", cv, dx, wy, wz)
        g[s:s + chunk, 1] = np.einsum("iabc,ia,ib,ic->i", cv, wx, dy, wz)
        g[s:s + chunk, 2] = np.einsum("iabc,ia,ib,ic->i", cv, wx, wy, dz)
    return ut, g * (n / L)


def five_step_classical(pos, q, L, n, P, alpha, rc):
    """All stages of the classical method; returns a dict like five_step."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    b = spread(pos, q, L, n, P)
    bhat = dft3(b, +1)
    p = influence(n, L, P, alpha, rc)
    chat = p * bhat
    cgrid = np.real(dft3(chat, -1))
    ut, grad = interpolate(pos, L, n, P, cgrid)
    s0 = GaussianSplit(alpha, rc).S0()
    phi = ut - q * s0
    F = -q[:, None] * grad
    E = 0.5 * float(np.einsum("i,i->", q, phi, optimize=False))
    return dict(b=b, bhat=bhat, p=p, chat=chat, c=cgrid, phi=phi, F=F, E=E, s0=s0,
                Ek=0.5 * float(np.sum(p * np.abs(bhat) ** 2)))
