"""Orthorhombic boxes (sides Lx, Ly, Lz) for the reference: classical Ewald,
the local sum and the ESP five-step method.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never does.

The five-step method runs on a cubic index grid n^3 with per-axis spacing
h_d = L_d/n (reading: the paper presents the cubic case; an orthorhombic box
scales each axis of the same grid). In grid units the window is the same
function on every axis, so spreading and interpolation are the cubic ones
with per-axis scaling; the influence function (eq. pk) becomes
    p_m = (h_x h_y h_z)^2 S^(|k|) / (V phi^_x(k_x)^2 phi^_y(k_y)^2 phi^_z(k_z)^2),
k_d = 2 pi m_d / L_d, V = L_x L_y L_z, phi^_d the window's transform at
spacing h_d. Classical Ewald and the local sum take the nearest image along
each axis.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .fivestep import dft3, interpolate, phi_hat_1d, spread
from .split import L_and_dL, PSWFSplit, S_hat


def _phase(x, m, L):
    return np.exp((2j * math.pi / L) * np.multiply.outer(x, m))


def _modes(pos, q, box, ms, W, targets, chunk=256):
    """u_i = Re sum_m W_m e^{-i k.r_i} with W = w * rho(m), and grad u."""
    mx, my, mz = ms
    rho = np.zeros((len(mx), len(my) * len(mz)), dtype=np.complex128)
    for s in range(0, len(pos), chunk):
        p = pos[s:s + chunk]
        ex = _phase(p[:, 0], mx, box[0]) * q[s:s + chunk, None]
        eyz = (_phase(p[:, 1], my, box[1])[:, :, None] * _phase(p[:, 2], mz, box[2])[:, None, :]).reshape(len(p), -1)
        rho += np.einsum("ja,jb->ab", ex, eyz, optimize=False)
    A = W.reshape(len(mx), -1) * rho
    kx, ky, kz = (2 * math.pi * np.asarray(m, np.float64) / L for m, L in zip(ms, box))
    kyf = np.repeat(ky, len(mz))
    kzf = np.tile(kz, len(my))
    pt = pos[targets]
    u = np.zeros(len(pt))
    g = np.zeros((len(pt), 3))
    for s in range(0, len(pt), chunk):
        p = pt[s:s + chunk]
        exc = np.conj(_phase(p[:, 0], mx, box[0]))
        eyz = np.conj((_phase(p[:, 1], my, box[1])[:, :, None] * _phase(p[:, 2], mz, box[2])[:, None, :])
                      .reshape(len(p), -1))
        B = np.einsum("ia,ab->ib", exc, A, optimize=False)
        Bx = np.einsum("ia,ab->ib", exc * (-1j * kx)[None, :], A, optimize=False)
        u[s:s + chunk] = np.real(np.sum(B * eyz, axis=1))
        g[s:s + chunk, 0] = np.real(np.sum(Bx * eyz, axis=1))
        g[s:s + chunk, 1] = np.real(np.sum(B * eyz * (-1j * kyf)[None, :], axis=1))
        g[s:s + chunk, 2] = np.real(np.sum(B * eyz * (-1j * kzf)[None, :], axis=1))
    return u, g


def ewald_box(pos, q, box, beta=None, targets=None):
    """Classical Ewald in an orthorhombic box: erfc real-space sum over nearest
    images, Gaussian k-space sum, self term; beta = 11.8/min(L_d) so that the
    real-space sum needs nearest images only."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    beta = 11.8 / box.min() if beta is None else beta
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    ur = np.zeros(len(idx))
    gr = np.zeros((len(idx), 3))
    c2 = 2 * beta / math.sqrt(math.pi)
    for s in range(0, len(idx), 256):
        ii = idx[s:s + 256]
        d = pos[ii, None, :] - pos[None, :, :]
        d -= box * np.round(d / box)
        r2 = np.einsum("abk,abk->ab", d, d)
        self_mask = ii[:, None] == np.arange(len(pos))[None, :]
        r2 = np.where(self_mask, 1.0, r2)
        r = np.sqrt(r2)
        e = np.where(self_mask, 0.0, erfc(beta * r) / (4 * math.pi * r))
        ur[s:s + 256] = np.einsum("ab,b->a", e, q, optimize=False)
        dr = -(erfc(beta * r) / r2 + c2 * np.exp(-beta * beta * r2) / r) / (4 * math.pi)
        dr = np.where(self_mask, 0.0, dr) / r
        gr[s:s + 256] = np.einsum("ab,abk->ak", dr * q[None, :], d)
    ms = [np.arange(-M, M + 1) for M in (int(math.ceil(12.2 * beta * L / (2 * math.pi))) for L in box)]
    k2 = (2 * math.pi * ms[0] / box[0])[:, None, None] ** 2 + (2 * math.pi * ms[1] / box[1])[None, :, None] ** 2 \
        + (2 * math.pi * ms[2] / box[2])[None, None, :] ** 2
    zero = tuple(len(m) // 2 for m in ms)
    k2[zero] = 1.0
    w = np.exp(-k2 / (4 * beta * beta)) / k2 / np.prod(box)
    w[zero] = 0.0
    uk, gk = _modes(pos, q, box, ms, w, idx)
    u = ur + uk - q[idx] * beta / (2 * math.pi ** 1.5)
    F = -q[idx, None] * (gr + gk)
    E = 0.5 * float(np.einsum("i,i->", q[idx], u, optimize=False)) if targets is None else None
    return u, F, E


def local_sum_box(pos, q, box, split, chunk=256):
    """u^l_i = sum_{j != i, r < rc} q_j L(r_ij) over nearest images, and grad."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    if split.support > box.min() / 2 + 1e-12:
        raise ValueError("local kernel support exceeds the half box; minimum image invalid")
    u = np.zeros(len(pos))
    g = np.zeros((len(pos), 3))
    allj = np.arange(len(pos))
    for s in range(0, len(pos), chunk):
        ii = allj[s:s + chunk]
        d = pos[ii, None, :] - pos[None, :, :]
        d -= box * np.round(d / box)
        r = np.sqrt(np.einsum("abk,abk->ab", d, d))
        a, b = np.nonzero((r < split.support) & (ii[:, None] != allj[None, :]))
        Lr, dLr = L_and_dL(split, r[a, b])
        np.add.at(u, s + a, q[b] * Lr)
        np.add.at(g, s + a, (q[b] * dLr / r[a, b])[:, None] * d[a, b])
    return u, g


def influence_box(n, box, P, c, rc, c1):
    """p_m on the full n^3 index grid (index k in [0, n): m = k or k - n)."""
    box = np.asarray(box, np.float64)
    h = box / n
    split = PSWFSplit(c, rc)
    k = np.arange(n)
    m = np.where(k < n // 2, k, k - n).astype(np.float64)
    kd = [2 * math.pi * m / L for L in box]
    ph = [phi_hat_1d(kd[a], P, h[a], c1) for a in range(3)]
    k2 = kd[0][:, None, None] ** 2 + kd[1][None, :, None] ** 2 + kd[2][None, None, :] ** 2
    k2[0, 0, 0] = 1.0
    S = S_hat(split, np.sqrt(k2))
    phi2 = (ph[0][:, None, None] * ph[1][None, :, None] * ph[2][None, None, :]) ** 2
    p = np.prod(h) ** 2 * S / (np.prod(box) * phi2)
    p[0, 0, 0] = 0.0
    return p


def five_step_box(pos, q, box, n, P, c, rc, c1):
    """All stages of the five-step method in an orthorhombic box."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    b = spread(pos, q, box, n, P, c1)
    bhat = dft3(b, +1)
    p = influence_box(n, box, P, c, rc, c1)
    cgrid = np.real(dft3(p * bhat, -1))
    ut, grad = interpolate(pos, box, n, P, c1, cgrid)
    s0 = PSWFSplit(c, rc).S0()
    phi = ut - q * s0
    F = -q[:, None] * grad
    E = 0.5 * float(np.einsum("i,i->", q, phi, optimize=False))
    return dict(b=b, bhat=bhat, p=p, c=cgrid, phi=phi, F=F, E=E, s0=s0)
