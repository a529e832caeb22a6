"""Classical Ewald summation (Introduction, eq. ewalderf), kernel 1/(4 pi r).

u_i = sum_{j != i} q_j erfc(beta r_ij)/(4 pi r_ij)                    (real space,
                                                                     minimum image)
    + (1/L^3) sum_{m != 0} exp(-k^2/(4 beta^2))/k^2 Re[e^{-i k.r_i} rho(k)]
    - q_i beta / (2 pi^{3/2})                                         (self)

with k = 2 pi m / L, rho(k) = sum_j q_j e^{i k.r_j}, tin-foil boundary (the
m = 0 term dropped, charge-neutral input). F_i = -q_i grad u(r_i), E = (1/2) sum q_i u_i.

Defaults: beta = 11.8/L, so erfc(beta L/2) < 2e-17 and only the nearest image
contributes in real space; |m_d| <= ceil(12.2 beta L/(2 pi)), where the
Gaussian factor has fallen below 1e-16 relative. Cost O(N^2 + N M^3), so this
is for N up to ~10^4 (sampled evaluation covers larger N).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from .spectral import structure_factor, evaluate_modes


def _min_image(d, L):
    return d - L * np.round(d / L)


def ewald_real(pos, q, L, beta, targets=None, chunk=256):
    """Real-space part at the target particles (all by default)."""
    pos = np.asarray(pos, np.float64)
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    u = np.zeros(len(idx))
    g = np.zeros((len(idx), 3))
    c2 = 2 * beta / math.sqrt(math.pi)
    for s in range(0, len(idx), chunk):
        ii = idx[s:s + chunk]
        d = _min_image(pos[ii, None, :] - pos[None, :, :], L)
        r2 = np.einsum("abk,abk->ab", d, d)
        self_mask = ii[:, None] == np.arange(len(pos))[None, :]
        r2 = np.where(self_mask, 1.0, r2)
        r = np.sqrt(r2)
        e = erfc(beta * r) / (4 * math.pi * r)
        e = np.where(self_mask, 0.0, e)
        u[s:s + chunk] = np.einsum("ab,b->a", e, q, optimize=False)
        # d/dr [erfc(beta r)/(4 pi r)] = -(erfc/r^2 + c2 exp(-beta^2 r^2)/r)/(4 pi)
        dr = -(erfc(beta * r) / r2 + c2 * np.exp(-beta * beta * r2) / r) / (4 * math.pi)
        dr = np.where(self_mask, 0.0, dr) / r
        g[s:s + chunk] = np.einsum("ab,abk->ak", dr * q[None, :], d)
    return u, g


def ewald(pos, q, L, beta=None, mmax=None, targets=None):
    """Potentials u_i, forces F_i and total energy E by classical Ewald."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    beta = 11.8 / L if beta is None else beta
    mmax = int(math.ceil(12.2 * beta * L / (2 * math.pi))) if mmax is None else mmax
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    ur, gr = ewald_real(pos, q, L, beta, idx)
    m = np.arange(-mmax, mmax + 1)
    rho = structure_factor(pos, q, L, m)
    kx = 2 * math.pi * m / L
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kx[None, None, :] ** 2
    k2[mmax, mmax, mmax] = 1.0
    w = np.exp(-k2 / (4 * beta * beta)) / k2
    w[mmax, mmax, mmax] = 0.0
    uk, gk = evaluate_modes(pos[idx], L, m, w * rho / L ** 3)
    u = ur + uk - q[idx] * beta / (2 * math.pi ** 1.5)
    F = -q[idx, None] * (gr + gk)
    E = 0.5 * float(np.einsum("i,i->", q[idx], u, optimize=False)) if targets is None else None
    return u, F, E
