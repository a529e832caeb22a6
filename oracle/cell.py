"""Triclinic cells for the reference: classical Ewald, the local sum and the
ESP five-step method.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never does.

A cell is the upper-triangular matrix H whose columns are the lattice vectors
a = (Lx, 0, 0), b = (xy, Ly, 0), c = (xz, yz, Lz); fractional coordinates are
s = H^-1 r. The five-step method runs on an n^3 index grid over fractional
coordinates (u = n s; reading: the paper presents the cubic case), where the
window is the cubic one along each lattice direction. With the volume per grid
point V/n^3 in place of h^3, the influence function (eq. pk) becomes
    p_m = S^(|k|)/V prod_d 1/f^(2 pi m_d/n)^2,   k = 2 pi H^-T m,
f^ the window's transform in grid units, and the forces are
F_i = -q_i n H^-T grad_u u~. Ewald and the local sum take the nearest image
among the 27 neighbouring cells of the wrapped fractional displacement (exact
when the cutoff is below half the smallest lattice-plane spacing).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .fivestep import dft3, ik_factors, interpolate, phi_hat_1d, spread
from . import classical
from .split import GaussianSplit, L_and_dL, PSWFSplit, S_hat


def cell_matrix(Lx, Ly, Lz, xy=0.0, xz=0.0, yz=0.0):
    return np.array([[Lx, xy, xz], [0.0, Ly, yz], [0.0, 0.0, Lz]], np.float64)


def plane_spacings(H):
    """Distances between consecutive lattice planes of each family (1/|row of H^-1|)."""
    return 1.0 / np.linalg.norm(np.linalg.inv(H), axis=1)


_SHIFTS = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)], np.float64)


def _nearest_images(d, H, Hinv):
    """Nearest-image displacements for an (..., 3) array of displacements."""
    s = np.einsum("...k,jk->...j", d, Hinv, optimize=False)
    s -= np.round(s)
    best = None
    for t in _SHIFTS:
        c = np.einsum("...k,jk->...j", s + t, H, optimize=False)
        r2 = np.einsum("...k,...k->...", c, c)
        if best is None:
            best, bd = r2, c
        else:
            m = r2 < best
            best = np.where(m, r2, best)
            bd = np.where(m[..., None], c, bd)
    return bd


def ewald_cell(pos, q, H, beta=None, targets=None):
    """Classical Ewald in a triclinic cell: erfc real-space sum over nearest
    images, Gaussian k-space sum over k = 2 pi H^-T m, self term; beta = 11.8
    over the smallest plane spacing, so nearest images suffice in real space."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    H = np.asarray(H, np.float64)
    Hinv = np.linalg.inv(H)
    V = abs(np.linalg.det(H))
    beta = 11.8 / plane_spacings(H).min() if beta is None else beta
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    ur = np.zeros(len(idx))
    gr = np.zeros((len(idx), 3))
    c2 = 2 * beta / math.sqrt(math.pi)
    for s in range(0, len(idx), 128):
        ii = idx[s:s + 128]
        d = _nearest_images(pos[ii, None, :] - pos[None, :, :], H, Hinv)
        r2 = np.einsum("abk,abk->ab", d, d)
        self_mask = ii[:, None] == np.arange(len(pos))[None, :]
        r2 = np.where(self_mask, 1.0, r2)
        r = np.sqrt(r2)
        ur[s:s + 128] = np.einsum("ab,b->a", np.where(self_mask, 0.0, erfc(beta * r) / (4 * math.pi * r)), q,
                                  optimize=False)
        dr = -(erfc(beta * r) / r2 + c2 * np.exp(-beta * beta * r2) / r) / (4 * math.pi)
        dr = np.where(self_mask, 0.0, dr) / r
        gr[s:s + 128] = np.einsum("ab,abk->ak", dr * q[None, :], d)
    # modes with |k| <= k_max, k_max where exp(-k^2/4 beta^2) < 1e-16
    kmax = 2 * beta * math.sqrt(16 * math.log(10))
    M = [int(math.ceil(kmax * np.linalg.norm(H[:, d]) / (2 * math.pi))) for d in range(3)]
    ms = np.array(np.meshgrid(*[np.arange(-m, m + 1) for m in M], indexing="ij")).reshape(3, -1).T
    ms = ms[np.any(ms != 0, axis=1)]
    k = 2 * math.pi * np.einsum("mj,jk->mk", ms, Hinv, optimize=False)  # k = 2 pi H^-T m, as rows
    k2 = np.einsum("mk,mk->m", k, k)
    keep = k2 <= kmax * kmax
    k, k2 = k[keep], k2[keep]
    w = np.exp(-k2 / (4 * beta * beta)) / k2 / V
    uk = np.zeros(len(idx))
    gk = np.zeros((len(idx), 3))
    for s in range(0, len(k), 2048):
        ks = k[s:s + 2048]
        ph = np.einsum("ik,mk->im", pos, ks, optimize=False)   # N x modes
        rho = (q[:, None] * np.exp(1j * ph)).sum(0)
        e = np.exp(-1j * ph[idx]) * (w[s:s + 2048] * rho)[None, :]
        uk += np.real(e.sum(1))
        gk += np.real(np.einsum("im,mk->ik", e * -1j, ks, optimize=False))
    u = ur + uk - q[idx] * beta / (2 * math.pi ** 1.5)
    F = -q[idx, None] * (gr + gk)
    E = 0.5 * float(np.einsum("i,i->", q[idx], u, optimize=False)) if targets is None else None
    return u, F, E


def local_sum_cell(pos, q, H, split, targets=None, chunk=128):
    """u^l_i = sum_{j != i, r < rc} q_j L(r_ij) over nearest images, and grad."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    H = np.asarray(H, np.float64)
    Hinv = np.linalg.inv(H)
    if split.support > plane_spacings(H).min() / 2 + 1e-12:
        raise ValueError("local kernel support exceeds half the smallest plane spacing")
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    u = np.zeros(len(idx))
    g = np.zeros((len(idx), 3))
    allj = np.arange(len(pos))
    for s in range(0, len(idx), chunk):
        ii = idx[s:s + chunk]
        d = _nearest_images(pos[ii, None, :] - pos[None, :, :], H, Hinv)
        r = np.sqrt(np.einsum("abk,abk->ab", d, d))
        a, b = np.nonzero((r < split.support) & (ii[:, None] != allj[None, :]))
        Lr, dLr = L_and_dL(split, r[a, b])
        np.add.at(u, s + a, q[b] * Lr)
        np.add.at(g, s + a, (q[b] * dLr / r[a, b])[:, None] * d[a, b])
    return u, g


def _influence_on_index_grid(n, H, split, f):
    """p_m = S^(|k|)/V / prod_d f_d^2 on the full n^3 index grid (index k in
    [0, n): m = k or k - n), k = 2 pi H^-T m, f the window's transform in grid
    units per axis (an array over the index).

    Reading: in a tilted cell p depends on the signs of m, and an index at the
    Nyquist frequency n/2 stands for both signs; p there is the mean over the
    sign choices of its Nyquist components, which keeps p(-m) = p(m) on the
    index grid (the inverse transform of p times a real grid's transform is
    then real)."""
    H = np.asarray(H, np.float64)
    Hinv = np.linalg.inv(H)
    V = abs(np.linalg.det(H))
    kk = np.arange(n)
    m = np.where(kk < n // 2, kk, kk - n).astype(np.float64)
    M = np.array(np.meshgrid(m, m, m, indexing="ij"))  # 3 x n x n x n
    nyq = np.abs(M) == n // 2
    acc = np.zeros((n, n, n))
    for signs in np.ndindex(2, 2, 2):
        Ms = np.where(nyq & (np.array(signs)[:, None, None, None] == 1), -M, M)
        k = 2 * math.pi * np.einsum("dj,d...->j...", Hinv, Ms)  # k_j = 2 pi sum_d Hinv[d, j] m_d
        kn = np.sqrt(np.einsum("j...,j...->...", k, k))
        kn[0, 0, 0] = 1.0
        acc += S_hat(split, kn)
    S = acc / 8
    p = S / V / (f[:, None, None] * f[None, :, None] * f[None, None, :]) ** 2
    p[0, 0, 0] = 0.0
    return p


def influence_cell(n, H, P, c, rc, c1):
    """ESP influence function on the index grid of a cell (eq. pk with V/n^3
    per grid point): PSWF splitting kernel, PSWF window."""
    kk = np.arange(n)
    m = np.where(kk < n // 2, kk, kk - n).astype(np.float64)
    f = phi_hat_1d(2 * math.pi * m / n, P, 1.0, c1)  # window transform in grid units
    return _influence_on_index_grid(n, H, PSWFSplit(c, rc), f)


def five_step_cell(pos, q, H, n, P, c, rc, c1):
    """All stages of the five-step method in a triclinic cell."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    H = np.asarray(H, np.float64)
    Hinv = np.linalg.inv(H)
    frac = np.mod(np.einsum("ik,jk->ij", pos, Hinv, optimize=False), 1.0)
    b = spread(frac, q, 1.0, n, P, c1)
    bhat = dft3(b, +1)
    p = influence_cell(n, H, P, c, rc, c1)
    cgrid = np.real(dft3(p * bhat, -1))
    ut, g_frac = interpolate(frac, 1.0, n, P, c1, cgrid)  # gradient in fractional coordinates
    grad = np.einsum("ij,jk->ik", g_frac, Hinv, optimize=False)   # d/dr = H^-T d/ds
    s0 = PSWFSplit(c, rc).S0()
    phi = ut - q * s0
    F = -q[:, None] * grad
    E = 0.5 * float(np.einsum("i,i->", q, phi, optimize=False))
    return dict(b=b, bhat=bhat, p=p, c=cgrid, phi=phi, F=F, E=E, s0=s0)


def five_step_cell_ik(pos, q, H, n, P, c, rc, c1):
    """Five-step method in a triclinic cell with forces by the "ik" route
    (Methods, force paragraph): the derivative of the potential along each
    fractional coordinate is the inverse transform of p b^ times -2 pi i m_d
    (0 at the Nyquist index), interpolated with the window itself; forces are
    F_i = -q_i H^-T grad_s. Potentials and energy are those of five_step_cell."""
    base = five_step_cell(pos, q, H, n, P, c, rc, c1)
    H = np.asarray(H, np.float64)
    Hinv = np.linalg.inv(H)
    frac = np.mod(np.einsum("ik,jk->ij", np.asarray(pos, np.float64), Hinv, optimize=False), 1.0)
    chat = base["p"] * base["bhat"]
    d = ik_factors(n, 1.0)  # derivative along a fractional coordinate
    gs = np.zeros((len(q), 3))
    for ax in range(3):
        shape = [1, 1, 1]
        shape[ax] = n
        g = np.real(dft3(chat * d.reshape(shape), -1))
        gs[:, ax], _ = interpolate(frac, 1.0, n, P, c1, g)
    out = dict(base)
    out["F"] = -np.asarray(q, np.float64)[:, None] * np.einsum("ij,jk->ik", gs, Hinv, optimize=False)
    return out


def five_step_classical_cell(pos, q, H, n, P, alpha, rc):
    """The classical method (Gaussian split, cardinal B-spline window of order
    P; Methods, classical fast Ewald methods) in a triclinic cell, on the same
    fractional grid as five_step_cell."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    H = np.asarray(H, np.float64)
    Hinv = np.linalg.inv(H)
    frac = np.mod(np.einsum("ik,jk->ij", pos, Hinv, optimize=False), 1.0)
    b = classical.spread(frac, q, 1.0, n, P)
    bhat = dft3(b, +1)
    kk = np.arange(n)
    m = np.where(kk < n // 2, kk, kk - n).astype(np.float64)
    f = classical.phi_hat_1d(2 * math.pi * m / n, P, 1.0)  # h sinc^P in grid units
    p = _influence_on_index_grid(n, H, GaussianSplit(alpha, rc), f)
    cgrid = np.real(dft3(p * bhat, -1))
    ut, g_frac = classical.interpolate(frac, 1.0, n, P, cgrid)
    s0 = GaussianSplit(alpha, rc).S0()
    phi = ut - q * s0
    F = -q[:, None] * np.einsum("ij,jk->ik", g_frac, Hinv, optimize=False)
    E = 0.5 * float(np.einsum("i,i->", q, phi, optimize=False))
    return dict(b=b, bhat=bhat, p=p, c=cgrid, phi=phi, F=F, E=E, s0=s0)
