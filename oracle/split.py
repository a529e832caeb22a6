"""The general radial split of the Coulomb kernel (Methods, eq. kernelsplitting):

    1/(4 pi r) = S(r) + L(r),   S(r) = G(r/rc)/(4 pi r),  L(r) = (1 - G(r/rc))/(4 pi r),

with G(t) = int_0^t chi and int_0^infty chi = 1.

Fourier transform of the smooth part (eq. hS): radial integration by parts
gives  S^(k) = chi^(rc |k|) / |k|^2  with  chi^(w) := int_0^infty chi(t) cos(w t) dt,
so chi^(0) = 1 and S^ -> 1/|k|^2 (the Coulomb transform) as k -> 0.

Readings of the paper (each listed in the design notes):
  * PSWF kernel (eq. pswf): chi(x) = psi_0^c(x) / int_0^1 psi_0^c on [0, 1]
    and chi = 0 beyond, so L(r) = 0 exactly for r >= rc. The normalisation is
    the one that makes S -> 1/(4 pi r) outside rc; eq. pswf's constant
    int_{-1}^{1} psi is the same choice written for the two-sided transform.
  * Self term (the (j,n) = (i,0) term of the spectral sum, eq. spectralpart):
    S(0) = chi(0)/(4 pi rc).
  * Gaussian kernel (eq. cem, with the missing sqrt(alpha) restored):
    chi(x) = 2 sqrt(alpha/pi) exp(-alpha x^2), G(t) = erf(sqrt(alpha) t),
    chi^(w) = exp(-w^2/(4 alpha)): classical Ewald with beta = sqrt(alpha)/rc.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .pswf import pswf


class PSWFSplit:
    def __init__(self, c: float, rc: float):
        self.c, self.rc = float(c), float(rc)
        self.psi = pswf(self.c)
        self.I1 = float(self.psi.integral(1.0))          # int_0^1 psi

    def chi(self, t):
        t = np.abs(np.asarray(t, dtype=np.float64))
        return np.where(t <= 1.0, self.psi(np.minimum(t, 1.0)) / self.I1, 0.0)

    def G(self, t):
        t = np.asarray(t, dtype=np.float64)
        return np.where(t >= 1.0, 1.0, self.psi.integral(np.clip(t, 0.0, 1.0)) / self.I1)

    def chihat(self, w):
        # int_0^1 psi cos = (1/2) int_{-1}^{1} psi cos  (psi even)
        return 0.5 * self.psi.ft(w) / self.I1

    @property
    def support(self):
        return self.rc

    def S0(self):
        return float(self.chi(0.0)) / (4 * math.pi * self.rc)


class GaussianSplit:
    def __init__(self, alpha: float, rc: float, support: float | None = None):
        self.alpha, self.rc = float(alpha), float(rc)
        # radius beyond which erfc(sqrt(alpha) r/rc) < 1e-16
        self._support = support if support is not None else rc * 5.9 / math.sqrt(alpha)

    def chi(self, t):
        t = np.asarray(t, dtype=np.float64)
        return 2 * math.sqrt(self.alpha / math.pi) * np.exp(-self.alpha * t * t)

    def G(self, t):
        return erf(math.sqrt(self.alpha) * np.asarray(t, dtype=np.float64))

    def chihat(self, w):
        w = np.asarray(w, dtype=np.float64)
        return np.exp(-w * w / (4 * self.alpha))

    @property
    def support(self):
        return self._support

    def S0(self):
        return float(self.chi(0.0)) / (4 * math.pi * self.rc)


def S_hat(split, k):
    """S^(k) = chi^(rc k)/k^2 for k > 0 (eq. hS)."""
    k = np.asarray(k, dtype=np.float64)
    return split.chihat(split.rc * k) / (k * k)


def L_and_dL(split, r):
    """Local kernel L(r) = (1 - G(r/rc))/(4 pi r) and its radial derivative."""
    r = np.asarray(r, dtype=np.float64)
    t = r / split.rc
    Gt = split.G(t)
    L = (1.0 - Gt) / (4 * math.pi * r)
    dL = -(1.0 - Gt) / (4 * math.pi * r * r) - split.chi(t) / (split.rc * 4 * math.pi * r)
    return L, dL
