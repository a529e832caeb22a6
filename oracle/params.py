"""Parameter selection (Methods: parameter rules after eq. errorformula,
eq. pswfparameters, Table 2).

Rules followed, and readings where the paper leaves a choice open (each is
listed in the design notes):
  * c: psi_0^c(1) = eps, with eps = tol (the target force error).
  * P: P_esp of Table 2 for the largest tabulated eps not above tol (the more
    accurate side); above 1e-3 P = 5; below 1e-5 P grows by 3 per decade
    (reading: extrapolating the table's trend), capped at 16.
  * n: smallest even 2^a 3^b with h = L/n <= h_max (default 1.25 length
    units); the paper sets n from rc and leaves rc to a cost balance with the
    short-range code, which is not part of the long-range path.
  * rc = kappa c h / pi with kappa = 1.2, i.e. the truncation rule of eq.
    pswfparameters (n = c L/(pi rc)) with a 20% margin.
  * c1: argmin of the aliasing estimate E_A (eq. errorformula) over
    c1 in [0.9 c, 1.4 c] ("slightly larger than c"); the argmin does not
    depend on E_A's overall normalisation.
"""
from __future__ import annotations

import math

import numpy as np

from .pswf import c_for_tolerance, pswf
from .split import PSWFSplit

# Table 2: eps -> (alpha_G, c_pswf, P_esp, R_default)
TABLE2 = {
    1e-3: (6.9078, 9.5392, 5, 5.78),
    5e-4: (7.6009, 10.290, 5, 7.71),
    1e-4: (9.2103, 12.024, 6, 14.32),
    5e-5: (9.9035, 12.762, 7, 22.42),
    1e-5: (11.5129, 14.471, 8, 54.57),
}


def order_for_tol(tol: float) -> int:
    if tol >= 1e-3:
        return 5
    if tol < 1e-5:
        return int(min(16, 8 + math.ceil(3 * math.log10(1e-5 / tol) - 1e-9)))
    cols = sorted(TABLE2)                  # ascending eps
    best = max(e for e in cols if e <= tol * (1 + 1e-12))
    return TABLE2[best][2]


def is_smooth(n: int) -> bool:
    if n < 2 or n % 2:
        return False
    while n % 2 == 0:
        n //= 2
    while n % 3 == 0:
        n //= 3
    return n == 1


def grid_size(L: float, h_max: float = 1.25, n_min: int = 8) -> int:
    n = max(n_min, int(math.ceil(L / h_max - 1e-12)))
    while not is_smooth(n):
        n += 1
    return n


def cutoff_radius(c: float, h: float, kappa: float = 1.2) -> float:
    return kappa * c * h / math.pi


def _aliasing_weights(n, L, c, rc):
    """c1-independent factor of E_A: a(m_x) = sum_{m_y, m_z} |chi^(2 pi rc |m|/L)| / |m|^2."""
    split = PSWFSplit(c, rc)
    m = np.arange(-(n // 2), n // 2)
    m2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    vals = np.arange(3 * (n // 2) ** 2 + 1, dtype=np.float64)
    vals[0] = 1.0
    table = np.abs(split.chihat(2 * math.pi * rc * np.sqrt(vals) / L)) / vals
    table[0] = 0.0
    return m.astype(np.float64), table[m2].sum(axis=(1, 2))


def _aliasing_from_weights(m, a, n, L, c1, P):
    h = L / n
    psi1 = pswf(c1)
    ft = lambda xi: psi1.ft(xi * P * h / 2.0)
    ratio = np.abs(ft(2 * math.pi * (m + n) / L) / ft(2 * math.pi * m / L))
    return 6.0 * float(np.einsum("i,i->", a, ratio, optimize=False))


def aliasing_error(n, L, c, rc, c1, P):
    """E_A of eq. errorformula (up to its overall constant):
    6 sum_{m in I, m != 0} |chi^(2 pi rc|m|/L)/|m|^2 * phi^(k + 2 pi (n,0,0)/L)/phi^(k)|;
    phi^ factorises per axis, so only the x factor of the ratio survives."""
    m, a = _aliasing_weights(n, L, c, rc)
    return _aliasing_from_weights(m, a, n, L, c1, P)


def choose_c1(n, L, c, rc, P, lo=0.9, hi=1.4, num=51):
    m, a = _aliasing_weights(n, L, c, rc)
    grid = np.linspace(lo * c, hi * c, num)
    ea = [_aliasing_from_weights(m, a, n, L, float(x), P) for x in grid]
    return float(grid[int(np.argmin(ea))])


def esp_parameters(L, tol, n=None, P=None, h_max=1.25, kappa=1.2, c1=None, rc=None):
    c = c_for_tolerance(tol)
    P = order_for_tol(tol) if P is None else P
    n = grid_size(L, h_max) if n is None else n
    h = L / n
    rc = cutoff_radius(c, h, kappa) if rc is None else rc
    c1 = choose_c1(n, L, c, rc, P) if c1 is None else c1
    return dict(n=n, P=P, c=c, rc=rc, c1=c1, h=h, L=L, tol=tol)
