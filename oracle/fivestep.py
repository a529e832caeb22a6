"""The five-step method for the spectral part (Methods, "Fast algorithm for the
spectral part", eqs. spread, FFT, diagonal scaling, IFFT, interp; eq. pk),
written out stage by stage in FP64 with the exact window (no piecewise
polynomials) and a plain matrix DFT (no FFT), so that each stage can be
compared with the GPU pipeline.

Notation: n = n_f grid points per side, h = L/n, grid point l sits at h*l
(l taken mod n), u = r/h in grid units. The SI kernel is
phi(x) = prod_d psi_0^{c1}(2 x_d/(P h)) (eq. pswf), supported on |x_d| < P h/2.

Readings (listed in the design notes):
  * Window placement: particle at u couples to the P points
    l0 .. l0+P-1 with l0 = floor(u - P/2) + 1 (for even P: floor(u)-P/2+1;
    for odd P: the P points centred on round(u)).
  * Influence function (eq. pk): with the unnormalised DFT pair as written,
    Poisson summation gives p_m = h^6 S^(k) / (L^3 phi^(k)^2), k = 2 pi m/L,
    where phi^ is the transform of phi in physical units,
    phi^(xi) = prod_d (P h/2) int_{-1}^{1} psi^{c1}(t) cos(xi_d P h t/2) dt.
    p_0 = 0 (m = 0 dropped, tin-foil boundary).
  * Forces by the AD route: F_i = -q_i grad u~(r_i), differentiating the
    window analytically (five_step), or by the "ik" route (five_step_ik):
    the scaled spectrum is multiplied by the spectral derivative of the
    inverse transform, c_l = sum_k exp(-2 pi i k.l/n) c^_k, i.e. by
    -2 pi i m_d / L along axis d (m_d = k_d or k_d - n), with the factor 0 at
    the Nyquist index k_d = n/2, whose two signed images cancel; each
    gradient grid is then interpolated with the window itself.
  * Self term: phi_i = u~_i - q_i S(0); E = (1/2) sum_i q_i phi_i.
"""
from __future__ import annotations

import math

import numpy as np

from .pswf import pswf
from .split import PSWFSplit, S_hat


def window(u, P, n, psi1):
    """Grid indices (mod n), weights and d(weight)/du for one axis."""
    l0 = np.floor(u - P / 2.0).astype(np.int64) + 1
    pts = l0[:, None] + np.arange(P)[None, :]
    disp = u[:, None] - pts
    x = 2.0 * disp / P
    return np.mod(pts, n), psi1(x), psi1.deriv(x) * (2.0 / P)


def phi_hat_1d(xi, P, h, c1):
    psi1 = pswf(c1)
    return 0.5 * P * h * psi1.ft(np.asarray(xi) * P * h / 2.0)


def influence(n, L, P, c, rc, c1):
    """p_m on the full n^3 index grid (index k in [0,n) means m = k or k-n)."""
    h = L / n
    split = PSWFSplit(c, rc)
    k = np.arange(n)
    m = np.where(k < n // 2, k, k - n).astype(np.float64)
    kk = 2 * math.pi * m / L
    ph = phi_hat_1d(kk, P, h, c1)
    m2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    m2[0, 0, 0] = 1.0
    S = S_hat(split, 2 * math.pi * np.sqrt(m2) / L)
    phi2 = (ph[:, None, None] * ph[None, :, None] * ph[None, None, :]) ** 2
    p = h ** 6 * S / (L ** 3 * phi2)
    p[0, 0, 0] = 0.0
    return p


def dft_matrix(n, sign):
    k = np.arange(n)
    return np.exp(sign * 2j * math.pi * np.outer(k, k) / n)


def dft3(a, sign):
    """sum_l exp(sign 2 pi i k.l/n) a_l along all three axes (numpy's own
    summation loops, without BLAS)."""
    F = dft_matrix(a.shape[0], sign)
    out = np.einsum("kl,lmn->kmn", F, a, optimize=False)
    out = np.einsum("kl,mln->mkn", F, out, optimize=False)
    out = np.einsum("kl,mnl->mnk", F, out, optimize=False)
    return out


def spread(pos, q, L, n, P, c1, chunk=20000):
    """b_l = sum_j phi~(r_j - h l) q_j  (eq. spread)."""
    psi1 = pswf(c1)
    u = np.mod(np.asarray(pos, np.float64), L) * (n / L)
    b = np.zeros(n ** 3)
    for s in range(0, len(u), chunk):
        us, qs = u[s:s + chunk], q[s:s + chunk]
        ix, wx, _ = window(us[:, 0], P, n, psi1)
        iy, wy, _ = window(us[:, 1], P, n, psi1)
        iz, wz, _ = window(us[:, 2], P, n, psi1)
        flat = (ix[:, :, None, None] * n + iy[:, None, :, None]) * n + iz[:, None, None, :]
        w = qs[:, None, None, None] * wx[:, :, None, None] * wy[:, None, :, None] * wz[:, None, None, :]
        b += np.bincount(flat.ravel(), weights=w.ravel(), minlength=n ** 3)
    return b.reshape(n, n, n)


def interpolate(pos, L, n, P, c1, cgrid, chunk=20000):
    """u~_i = sum_l phi~(r_i - h l) c_l (eq. interp) and its gradient (physical units)."""
    psi1 = pswf(c1)
    u = np.mod(np.asarray(pos, np.float64), L) * (n / L)
    cf = cgrid.ravel()
    ut = np.zeros(len(u))
    g = np.zeros((len(u), 3))
    for s in range(0, len(u), chunk):
        us = u[s:s + chunk]
        ix, wx, dx = window(us[:, 0], P, n, psi1)
        iy, wy, dy = window(us[:, 1], P, n, psi1)
        iz, wz, dz = window(us[:, 2], P, n, psi1)
        flat = (ix[:, :, None, None] * n + iy[:, None, :, None]) * n + iz[:, None, None, :]
        cv = cf[flat]
        ut[s:s + chunk] = np.einsum("iabc,ia,ib,ic->i", cv, wx, wy, wz)
        g[s:s + chunk, 0] = np.einsum("iabc,ia,ib,ic->i", cv, dx, wy, wz)
        g[s:s + chunk, 1] = np.einsum("iabc,ia,ib,ic->i", cv, wx, dy, wz)
        g[s:s + chunk, 2] = np.einsum("iabc,ia,ib,ic->i", cv, wx, wy, dz)
    return ut, g * (n / L)


def _finite(name, a):
    """Every stage of a finite input is finite; name the first one that is not."""
    if not np.all(np.isfinite(a)):
        raise FloatingPointError(f"five-step reference: stage {name} holds "
                                 f"{int(np.count_nonzero(~np.isfinite(a)))} non-finite values")
    return a


def five_step(pos, q, L, n, P, c, rc, c1):
    """All stages of the five-step method; returns a dict."""
    pos = _finite("positions", np.asarray(pos, np.float64))
    q = _finite("charges", np.asarray(q, np.float64))
    b = _finite("b (spread)", spread(pos, q, L, n, P, c1))
    bhat = _finite("b^ (forward DFT)", dft3(b, +1))
    p = _finite("p (influence)", influence(n, L, P, c, rc, c1))
    chat = p * bhat
    cgrid = _finite("c (inverse DFT)", np.real(dft3(chat, -1)))
    ut, grad = interpolate(pos, L, n, P, c1, cgrid)
    _finite("u~ (interpolation)", ut)
    _finite("grad u~ (interpolation)", grad)
    s0 = PSWFSplit(c, rc).S0()
    phi = ut - q * s0
    F = -q[:, None] * grad
    E = 0.5 * float(np.einsum("i,i->", q, phi, optimize=False))
    Ek = 0.5 * float(np.sum(p * np.abs(bhat) ** 2))
    return dict(b=b, bhat=bhat, p=p, chat=chat, c=cgrid, u_tilde=ut, grad=grad,
                phi=phi, F=F, E=E, Ek=Ek, s0=s0)


def ik_factors(n, L):
    """Spectral derivative factors of one axis, index k in [0, n): the
    derivative of exp(-2 pi i m x/L) is -2 pi i m/L times it (m = k or k - n);
    0 at the Nyquist index n/2."""
    k = np.arange(n)
    m = np.where(k <= n // 2, k, k - n).astype(np.float64)
    d = -2j * math.pi * m / L
    d[n // 2] = 0.0
    return d


def five_step_ik(pos, q, L, n, P, c, rc, c1):
    """Five-step method with forces by the "ik" route (Methods, force
    paragraph): the potentials and energy are those of five_step; the force
    on particle i is -q_i times the window interpolation of the three
    gradient grids IFFT(d_ax c^)."""
    base = five_step(pos, q, L, n, P, c, rc, c1)
    d = ik_factors(n, L)
    grids, grad = [], np.zeros((len(q), 3))
    for ax in range(3):
        shape = [1, 1, 1]
        shape[ax] = n
        g = dft3(base["chat"] * d.reshape(shape), -1)
        grids.append(np.real(g))
        grad[:, ax], _ = interpolate(pos, L, n, P, c1, np.real(g))
    out = dict(base)
    out["grad"] = grad
    out["grad_grids"] = grids
    out["F"] = -np.asarray(q, np.float64)[:, None] * grad
    return out
