"""Direct (non-uniform) Fourier sums and the local sum.

  * structure_factor: rho(m) = sum_j q_j exp(2 pi i m.r_j / L)
  * evaluate_modes:   u(r) = Re sum_m W_m exp(-2 pi i m.r / L) and grad u
  * spectral_sum:     the truncated spectral part (eq. spectralpart with the
                      index set I, eq. truncationerror): W_m = S^(2 pi m/L)/L^3 rho(m)
  * local_sum:        the local part (eq. localpart) over pairs within the
                      kernel's support (minimum image)

All sums are plain O(N x modes) and O(N^2) loops, written as einsum contractions
evaluated by numpy's own loops (optimize=False, so no BLAS call);
exponentials factor per axis, exp(i k.r) = exp(i k_x x) exp(i k_y y) exp(i k_z z).

Reading for the Nyquist modes (listed in the design notes): I is the
asymmetric set {-n/2..n/2-1}^3; the sum here uses {-n/2..n/2}^3 with weight 1/2
on each |m_d| = n/2, which keeps u real and equals the average of the two
asymmetric choices.
"""
from __future__ import annotations

import math

import numpy as np

from .split import S_hat, L_and_dL


def _phase(x, m, L):
    return np.exp((2j * math.pi / L) * np.multiply.outer(x, m))


def structure_factor(pos, q, L, m, chunk=1024):
    pos = np.asarray(pos, np.float64)
    M = len(m)
    S = np.zeros((M, M * M), dtype=np.complex128)
    for s in range(0, len(pos), chunk):
        p = pos[s:s + chunk]
        ex = _phase(p[:, 0], m, L) * q[s:s + chunk, None]
        eyz = (_phase(p[:, 1], m, L)[:, :, None] * _phase(p[:, 2], m, L)[:, None, :]).reshape(len(p), M * M)
        S += np.einsum("ja,jb->ab", ex, eyz, optimize=False)
    return S.reshape(M, M, M)


def evaluate_modes(pos, L, m, W, chunk=512):
    """u_i = Re sum_m W_m e^{-i k.r_i}; grad_i = Re sum_m W_m (-i k) e^{-i k.r_i}."""
    pos = np.asarray(pos, np.float64)
    M = len(m)
    k = 2 * math.pi * np.asarray(m, np.float64) / L
    Wf = W.reshape(M, M * M)
    kyz_y = np.repeat(k, M)          # k_y for flattened (b, c)
    kyz_z = np.tile(k, M)            # k_z for flattened (b, c)
    u = np.zeros(len(pos))
    g = np.zeros((len(pos), 3))
    for s in range(0, len(pos), chunk):
        p = pos[s:s + chunk]
        exc = np.conj(_phase(p[:, 0], m, L))
        eyz = np.conj((_phase(p[:, 1], m, L)[:, :, None] * _phase(p[:, 2], m, L)[:, None, :]).reshape(len(p), M * M))
        A = np.einsum("ia,ab->ib", exc, Wf, optimize=False)
        Ax = np.einsum("ia,ab->ib", exc * (-1j * k)[None, :], Wf, optimize=False)
        u[s:s + chunk] = np.real(np.sum(A * eyz, axis=1))
        g[s:s + chunk, 0] = np.real(np.sum(Ax * eyz, axis=1))
        g[s:s + chunk, 1] = np.real(np.sum(A * eyz * (-1j * kyz_y)[None, :], axis=1))
        g[s:s + chunk, 2] = np.real(np.sum(A * eyz * (-1j * kyz_z)[None, :], axis=1))
    return u, g


def spectral_weights(split, n, L):
    """S^(2 pi m/L)/L^3 on m in {-n/2..n/2}^3 with the Nyquist halving, m=0 dropped."""
    m = np.arange(-(n // 2), n // 2 + 1)
    k = 2 * math.pi * m / L
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    zero = (len(m) // 2,) * 3
    k2[zero] = 1.0
    w = S_hat(split, np.sqrt(k2)) / L ** 3
    w[zero] = 0.0
    half = np.where(np.abs(m) == n // 2, 0.5, 1.0)
    w *= half[:, None, None] * half[None, :, None] * half[None, None, :]
    return m, w


def spectral_sum(pos, q, L, split, n, targets=None):
    """Truncated spectral potential u^s_i (self-image included) and grad u^s."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    m, w = spectral_weights(split, n, L)
    rho = structure_factor(pos, q, L, m)
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    return evaluate_modes(pos[idx], L, m, w * rho)


def local_sum(pos, q, L, split, targets=None, chunk=256):
    """u^l_i = sum_{j != i} q_j L(|r_ij|) over the nearest image within the
    kernel's support (which must not exceed L/2), and grad u^l."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    rcut = split.support
    if rcut > L / 2 + 1e-12:
        raise ValueError("local kernel support exceeds L/2; minimum image invalid")
    idx = np.arange(len(pos)) if targets is None else np.asarray(targets)
    u = np.zeros(len(idx))
    g = np.zeros((len(idx), 3))
    allj = np.arange(len(pos))
    for s in range(0, len(idx), chunk):
        ii = idx[s:s + chunk]
        d = pos[ii, None, :] - pos[None, :, :]
        d -= L * np.round(d / L)
        r = np.sqrt(np.einsum("abk,abk->ab", d, d))
        mask = (r < rcut) & (ii[:, None] != allj[None, :])
        a, b = np.nonzero(mask)
        Lr, dLr = L_and_dL(split, r[a, b])
        np.add.at(u, s + a, q[b] * Lr)
        np.add.at(g, s + a, (q[b] * dLr / r[a, b])[:, None] * d[a, b])
    return u, g
