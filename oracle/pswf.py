"""Prolate spheroidal wave function psi_0^c (Methods: "Optimizing the
evaluation of the spectral part using PSWFs").

psi_0^c is the eigenfunction with the largest eigenvalue of the finite Fourier
operator F_c[f](x) = int_{-1}^{1} f(t) exp(i c x t) dt on L^2[-1,1]; it is even.
Normalisation (a reading, pinned by Table 2): int_{-1}^{1} psi^2 = 1 and
psi(0) > 0. The shape parameter c for a tolerance eps solves psi_0^c(1) = eps.

Two independent routes:
  * PSWF (primary): psi_0^c also is the eigenfunction of the prolate
    differential operator -(d/dx)(1-x^2)(d/dx) + c^2 x^2 with the smallest
    eigenvalue (Slepian & Pollak 1961). In the orthonormal even Legendre basis
    that operator is a symmetric tridiagonal matrix whose low eigenvalues are
    well separated for every c, so the coefficients are accurate to rounding.
  * NystromPSWF (cross-check): the paper's definition taken literally, F_c
    discretised on Gauss-Legendre nodes and the top eigenvector of the cosine
    kernel. The top eigenvalues of that kernel cluster as c grows, so this
    route loses digits beyond c ~ 18; tests use it to pin the primary route in
    the range of Table 2.
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.optimize import brentq

_QT, _QW = npleg.leggauss(256)          # quadrature for transforms on [-1, 1]


class PSWF:
    """psi_0^c through its Legendre expansion (smallest eigenvalue of the
    prolate operator in the orthonormal even Legendre basis)."""

    def __init__(self, c: float, kmax: int | None = None):
        self.c = c = float(c)
        if kmax is None:
            kmax = 2 * int(c + 40)
        ks = np.arange(0, kmax, 2, dtype=np.float64)
        # x^2 P_k = (k+1)(k+2)/((2k+1)(2k+3)) P_{k+2}
        #         + [(k+1)^2/((2k+1)(2k+3)) + k^2/((2k+1)(2k-1))] P_k + (...) P_{k-2}
        diag = ks * (ks + 1) + c * c * (((ks + 1) ** 2) / ((2 * ks + 1) * (2 * ks + 3))
                                        + (ks ** 2) / ((2 * ks + 1) * (2 * ks - 1)))
        kk = ks[:-1]
        up = (kk + 1) * (kk + 2) / ((2 * kk + 1) * (2 * kk + 3))
        # change to the orthonormal basis sqrt(k+1/2) P_k
        off = c * c * up * np.sqrt((2 * kk + 1) / (2 * kk + 5))
        M = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
        vals, vecs = np.linalg.eigh(M)
        beta = vecs[:, 0]
        if beta[0] < 0:                 # int psi = sqrt(2) beta_0 > 0
            beta = -beta
        coef = np.zeros(kmax)
        coef[0::2] = beta * np.sqrt(ks + 0.5)
        self.chi0 = float(vals[0])      # prolate eigenvalue
        self.coef = coef                # psi = sum coef_k P_k, |psi|_2 = 1
        self._dcoef = npleg.legder(coef)
        self._icoef = npleg.legint(coef, lbnd=0.0)
        # eigenvalue of F_c from the eigen-relation at x = 0
        self.lam = float(self.ft(0.0) / self(0.0))

    def __call__(self, x):
        """psi(x), |x| <= 1."""
        return npleg.legval(np.asarray(x, dtype=np.float64), self.coef)

    def deriv(self, x):
        """psi'(x), |x| <= 1."""
        return npleg.legval(np.asarray(x, dtype=np.float64), self._dcoef)

    def integral(self, x):
        """int_0^x psi(s) ds, |x| <= 1."""
        return npleg.legval(np.asarray(x, dtype=np.float64), self._icoef)

    def ft(self, omega):
        """int_{-1}^{1} psi(t) cos(omega t) dt (256-node Gauss-Legendre)."""
        omega = np.asarray(omega, dtype=np.float64)
        return np.einsum("...t,t->...", np.cos(np.multiply.outer(omega, _QT)), _QW * self(_QT), optimize=False)


class NystromPSWF:
    """Cross-check only: top eigenvector of the Nystrom-discretised cosine
    kernel of F_c, evaluated through the eigen-relation."""

    def __init__(self, c: float, nodes: int = 192):
        self.c = float(c)
        t, w = npleg.leggauss(nodes)
        sw = np.sqrt(w)
        A = sw[:, None] * np.cos(self.c * np.outer(t, t)) * sw[None, :]
        vals, vecs = np.linalg.eigh(A)
        psi = vecs[:, -1] / sw
        if np.einsum("i,i->", w, psi, optimize=False) < 0:
            psi = -psi
        self.lam = float(vals[-1])
        self.t, self._wpsi = t, w * psi

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        return np.einsum("...t,t->...", np.cos(self.c * np.multiply.outer(x, self.t)), self._wpsi,
                         optimize=False) / self.lam


@functools.lru_cache(maxsize=128)
def pswf(c: float) -> PSWF:
    return PSWF(c)


def c_for_tolerance(eps: float) -> float:
    """Shape parameter c with psi_0^c(1) = eps (Methods, parameter choice)."""
    f = lambda c: np.log(PSWF(c)(1.0)) - np.log(eps)
    # c tends to log(1/eps) as eps -> 0; bracket around that value
    lo = max(0.5, np.log(1.0 / eps) - 3.0)
    hi = np.log(1.0 / eps) + 10.0
    return float(brentq(f, lo, hi, xtol=1e-13, rtol=1e-13))
