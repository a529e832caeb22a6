"""Pins of the oracle's Ewald sums and kernel split against textbook values,
brute-force lattice sums and exact special cases."""
import math

import numpy as np
import pytest

import workloads as W
from conftest import read_golden
from oracle.ewald import ewald
from oracle.pswf import c_for_tolerance
from oracle.split import PSWFSplit, GaussianSplit
from oracle.spectral import spectral_sum, local_sum


MADELUNG = float(read_golden("madelung.txt")[0][1])


def test_madelung_constant():
    pos, q, L = W.nacl_crystal()
    u, F, E = ewald(pos, q, L)
    r0 = 5.64 / 2
    # every ion sees u_i = -q_i M/(4 pi r0); E = -(N/2) M/(4 pi r0)
    M_i = -u * q * 4 * math.pi * r0
    assert np.max(np.abs(M_i - MADELUNG)) < 1e-6
    assert abs(-E * 4 * math.pi * r0 / (len(q) / 2) - MADELUNG) < 1e-6
    assert np.max(np.abs(F)) < 1e-12


def _brute_energy(pos, q, L, K):
    """Direct sum over whole image cells inside a sphere of K cells."""
    r = np.arange(-K, K + 1)
    nn = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    nn = nn[np.einsum("ij,ij->i", nn, nn) <= K * K] * L
    E = 0.0
    for i in range(len(q)):
        for j in range(len(q)):
            d = pos[i] - pos[j] + nn
            rr = np.sqrt(np.einsum("ij,ij->i", d, d))
            if i == j:
                rr = rr[rr > 0]
            E += 0.5 * q[i] * q[j] * np.sum(1.0 / (4 * math.pi * rr))
    return E


@pytest.mark.parametrize("seed,nq", [(0, 2), (1, 4)])
def test_brute_force_image_sum(seed, nq):
    # spherical summation in vacuum = tin-foil Ewald + |M|^2/(6V) (kernel 1/(4 pi r))
    rng = np.random.default_rng(seed)
    L = 3.0
    pos = rng.random((nq, 3)) * L
    q = rng.standard_normal(nq)
    q -= q.mean()
    _, _, E = ewald(pos, q, L)
    M = q @ pos
    Evac = E + M @ M / (6 * L ** 3)
    assert abs(_brute_energy(pos, q, L, 40) - Evac) < 1e-5 * abs(Evac)


def test_ewald_invariances():
    rng = np.random.default_rng(7)
    L = 9.0
    pos = rng.random((40, 3)) * L
    q = rng.standard_normal(40)
    q -= q.mean()
    u, F, E = ewald(pos, q, L)
    assert np.linalg.norm(F.sum(0)) < 1e-12 * np.linalg.norm(F)
    u2, F2, E2 = ewald(np.mod(pos + np.array([0.37, -1.9, 4.4]), L), q, L)
    assert np.max(np.abs(u2 - u)) < 1e-12 * np.max(np.abs(u))
    assert np.max(np.abs(F2 - F)) < 1e-11 * np.max(np.abs(F))
    # beta-independence (the split is exact)
    u3, F3, _ = ewald(pos, q, L, beta=10.0 / L, mmax=20)   # erfc(5) ~ 1.5e-12
    assert np.max(np.abs(u3 - u)) < 1e-10 * np.max(np.abs(u))
    # F = -grad E by central differences on one coordinate
    hh = 1e-6
    p1, p2 = pos.copy(), pos.copy()
    p1[3, 1] += hh
    p2[3, 1] -= hh
    fd = -(ewald(p1, q, L)[2] - ewald(p2, q, L)[2]) / (2 * hh)
    assert abs(fd - F[3, 1]) < 1e-6 * np.max(np.abs(F))


def test_gaussian_split_is_classical_ewald():
    # the general split with a Gaussian chi (eq. cem) is exactly the erfc split;
    # this pins S^ = chi^(rc k)/k^2, the local kernel and the self term
    pos, q, L = W.nacl_crystal(perturb=0.3, seed=3)
    u, F, E = ewald(pos, q, L)
    sp = GaussianSplit(alpha=9.0, rc=5.0)
    us, gs = spectral_sum(pos, q, L, sp, 48)
    ul, gl = local_sum(pos, q, L, sp)
    assert np.max(np.abs(us + ul - q * sp.S0() - u)) < 1e-12 * np.max(np.abs(u))
    Fe = -q[:, None] * (gs + gl)
    assert np.max(np.abs(Fe - F)) < 1e-11 * np.max(np.abs(F))


def test_pswf_split_reproduces_ewald_at_tight_eps():
    # with eps = 1e-10 the truncated spectral sum plus local sum minus self term
    # equals classical Ewald to ~eps (eqs. kernelsplitting, localpart, spectralpart)
    pos, q, L = W.nacl_crystal(perturb=0.3, seed=4)
    u, F, E = ewald(pos, q, L)
    sp = PSWFSplit(c_for_tolerance(1e-10), 5.0)
    us, gs = spectral_sum(pos, q, L, sp, 64)
    ul, gl = local_sum(pos, q, L, sp)
    assert np.max(np.abs(us + ul - q * sp.S0() - u)) < 1e-10 * np.max(np.abs(u))
    Fe = -q[:, None] * (gs + gl)
    assert np.sqrt(np.sum((Fe - F) ** 2) / np.sum(F ** 2)) < 1e-9


def test_local_part_vanishes_beyond_cutoff():
    sp = PSWFSplit(12.024, 4.0)
    from oracle.split import L_and_dL
    Lr, dLr = L_and_dL(sp, np.array([4.0, 4.5, 9.0]))
    assert np.all(np.abs(Lr) < 1e-15) and np.all(np.abs(dLr[1:]) < 1e-15)
    # continuity of the split at r -> 0: L(r) ~ 1/(4 pi r) - S(0)
    r = 1e-4
    assert abs(L_and_dL(sp, np.array([r]))[0][0] - (1 / (4 * math.pi * r) - sp.S0())) < 1e-6
