"""Pins of the triclinic-cell reference (oracle.cell): the orthorhombic special
case against oracle.box, Ewald's invariance under a change of cell that keeps
the lattice, the rock-salt Madelung constant in a sheared cell (Ewald and the
five-step method with the local part), and Delta against Ewald in a tilted
cell."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.box import ewald_box, five_step_box, local_sum_box
from oracle.cell import (cell_matrix, ewald_cell, five_step_cell, five_step_cell_ik, five_step_classical_cell,
                         influence_cell, local_sum_cell, plane_spacings)
from oracle.metrics import rel_rms
from oracle.params import esp_parameters
from oracle.split import PSWFSplit

MADELUNG = 1.747565


def _random_charges(H, N, seed):
    rng = np.random.default_rng(seed)
    s = rng.uniform(0, 1, (N, 3))
    return s @ np.asarray(H).T, np.tile([W.Q_O, W.Q_H, W.Q_H], N // 3)


def test_zero_tilt_is_the_orthorhombic_reference():
    box = (13.0, 15.0, 17.0)
    H = cell_matrix(*box)
    pos, q = _random_charges(H, 300, 1)
    u1, F1, E1 = ewald_box(pos, q, box)
    u2, F2, E2 = ewald_cell(pos, q, H)
    assert np.max(np.abs(u2 - u1)) < 1e-11 * np.max(np.abs(u1))
    assert np.max(np.abs(F2 - F1)) < 1e-10 * np.max(np.abs(F1))
    n, P, c, rc, c1 = 16, 6, 12.024, 4.5, 12.5
    a = five_step_box(pos, q, box, n, P, c, rc, c1)
    b = five_step_cell(pos, q, H, n, P, c, rc, c1)
    assert rel_rms(b["F"], a["F"]) < 1e-12 and abs(b["E"] - a["E"]) < 1e-12 * abs(a["E"])
    sp = PSWFSplit(c, rc)
    ua, ga = local_sum_box(pos, q, box, sp)
    ub, gb = local_sum_cell(pos, q, H, sp)
    assert np.max(np.abs(ub - ua)) < 1e-13 and np.max(np.abs(gb - ga)) < 1e-12


def test_ewald_is_invariant_under_a_change_of_cell():
    # H U with U unimodular spans the same lattice
    H = cell_matrix(14.0, 15.0, 16.0, xy=2.0, xz=-1.5, yz=3.0)
    U = np.array([[1, 1, 0], [0, 1, 0], [0, 0, 1]], np.float64)
    H2 = H @ U
    pos, q = _random_charges(H, 240, 2)
    u1, F1, E1 = ewald_cell(pos, q, H)
    u2, F2, E2 = ewald_cell(pos, q, H2)
    assert np.max(np.abs(u2 - u1)) < 1e-10 * np.max(np.abs(u1))
    assert np.max(np.abs(F2 - F1)) < 1e-9 * np.max(np.abs(F1))


def test_madelung_constant_in_a_sheared_cell():
    # 4 x 4 x 4 conventional rock-salt cells described by a sheared cell
    pos, q, L = W.nacl_crystal(cells=4)
    H = cell_matrix(L, L, L, xy=L)   # lattice vectors a, a + b, c
    u, F, E = ewald_cell(pos, q, H)
    r0 = 5.64 / 2
    assert np.max(np.abs(-u * q * 4 * math.pi * r0 - MADELUNG)) < 1e-6
    assert np.max(np.abs(F)) < 1e-10
    # the five-step method with the local part, on a grid along the sheared cell
    pr = esp_parameters(float(np.linalg.norm(H[:, 1])), 1e-4)
    n, P, c, rc, c1 = pr["n"], pr["P"], pr["c"], pr["rc"], pr["c1"]
    assert rc <= plane_spacings(H).min() / 2
    r = five_step_cell(pos, q, H, n, P, c, rc, c1)
    ul, gl = local_sum_cell(pos, q, H, PSWFSplit(c, rc))
    M = -(r["phi"] + ul) * q * 4 * math.pi * r0
    assert np.max(np.abs(M - MADELUNG)) < 1e-4 * MADELUNG


@pytest.mark.parametrize("tilts,tol", [((3.0, -2.0, 4.0), 1e-4), ((-5.0, 2.5, 0.0), 1e-3)])
def test_five_step_in_a_tilted_cell_reaches_the_tolerance(tilts, tol):
    H = cell_matrix(20.0, 19.0, 18.0, *tilts)
    N = 3 * int(0.03 * abs(np.linalg.det(H)) / 3)
    pos, q = _random_charges(H, N, 7)
    Lmax = float(np.linalg.norm(H, axis=0).max())
    pr = esp_parameters(Lmax, tol)
    n, P, c, rc, c1 = pr["n"], pr["P"], pr["c"], pr["rc"], pr["c1"]
    r = five_step_cell(pos, q, H, n, P, c, rc, c1)
    ul, gl = local_sum_cell(pos, q, H, PSWFSplit(c, rc))
    F = r["F"] - q[:, None] * gl
    _, F_e, E_e = ewald_cell(pos, q, H)
    assert rel_rms(F, F_e) < tol
    assert abs(0.5 * np.dot(q, r["phi"] + ul) - E_e) < tol * abs(E_e)


def test_influence_is_even_on_the_index_grid():
    # p(-m) = p(m), Nyquist indices included, so the convolution of a real grid is real
    H = cell_matrix(16.0, 15.0, 14.0, 4.0, -3.0, 2.0)
    n = 12
    p = influence_cell(n, H, 6, 12.024, 4.0, 12.5)
    neg = (-np.arange(n)) % n
    assert np.max(np.abs(p - p[np.ix_(neg, neg, neg)])) < 1e-14 * np.max(p)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((n, n, n))
    from oracle.fivestep import dft3
    c = dft3(p * dft3(b, +1), -1)
    assert np.max(np.abs(c.imag)) < 1e-13 * np.max(np.abs(c.real))
    # a zero-tilt cell matches the orthorhombic table
    from oracle.box import influence_box
    pb = influence_box(n, (16.0, 15.0, 14.0), 6, 12.024, 4.0, 12.5)
    pc = influence_cell(n, cell_matrix(16.0, 15.0, 14.0), 6, 12.024, 4.0, 12.5)
    assert np.max(np.abs(pc - pb)) < 1e-10 * np.max(np.abs(pb))



def test_ik_forces_in_a_cell():
    # a cubic cell reproduces the cubic ik route, which is built on Cartesian
    # derivatives instead of fractional ones
    from oracle.fivestep import five_step_ik
    L, n, P, c, rc, c1 = 14.0, 16, 6, 12.024, 4.5, 12.5
    pos, q = W.water_box(120, L, seed=4)
    a = five_step_ik(pos, q, L, n, P, c, rc, c1)
    b = five_step_cell_ik(pos, q, cell_matrix(L, L, L), n, P, c, rc, c1)
    assert rel_rms(b["F"], a["F"]) < 1e-12
    # a tilted cell: momentum conserved exactly, Delta against Ewald within
    # the tolerance, and agreement with the analytic-derivative forces
    H = cell_matrix(20.0, 19.0, 18.0, 3.0, -2.0, 4.0)
    N = 3 * int(0.03 * abs(np.linalg.det(H)) / 3)
    pos, q = _random_charges(H, N, 7)
    pr = esp_parameters(float(np.linalg.norm(H, axis=0).max()), 1e-4)
    n, P, c, rc, c1 = pr["n"], pr["P"], pr["c"], pr["rc"], pr["c1"]
    r = five_step_cell_ik(pos, q, H, n, P, c, rc, c1)
    ad = five_step_cell(pos, q, H, n, P, c, rc, c1)
    assert np.abs(r["F"].sum(0)).max() < 1e-12 * np.abs(r["F"]).max() * N
    ul, gl = local_sum_cell(pos, q, H, PSWFSplit(c, rc))
    _, F_e, _ = ewald_cell(pos, q, H)
    assert rel_rms(r["F"] - q[:, None] * gl, F_e) < 1e-4
    assert rel_rms(r["F"], ad["F"]) < 1e-3



def test_classical_method_in_a_cell():
    # a cubic cell reproduces the cubic classical reference
    from oracle.classical import five_step_classical
    from oracle.split import GaussianSplit
    L = 14.0
    pos, q = W.water_box(120, L, seed=4)
    alpha, rc, n, P = math.log(1e4), 4.5, 24, 6
    a = five_step_classical(pos, q, L, n, P, alpha, rc)
    b = five_step_classical_cell(pos, q, cell_matrix(L, L, L), n, P, alpha, rc)
    assert rel_rms(b["F"], a["F"]) < 1e-12 and abs(b["E"] - a["E"]) < 1e-12 * abs(a["E"])
    # a tilted cell: Delta against triclinic Ewald falls with the grid and
    # settles at the split's own error (alpha = log 1e4: about 1.2e-5)
    H = cell_matrix(20.0, 19.0, 18.0, 3.0, -2.0, 4.0)
    N = 3 * int(0.03 * abs(np.linalg.det(H)) / 3)
    pos, q = _random_charges(H, N, 7)
    _, F_e, _ = ewald_cell(pos, q, H)
    rc = 5.0
    ul, gl = local_sum_cell(pos, q, H, GaussianSplit(alpha, rc, support=rc))
    deltas = []
    for n, P in ((24, 5), (32, 5), (48, 8)):
        r = five_step_classical_cell(pos, q, H, n, P, alpha, rc)
        deltas.append(rel_rms(r["F"] - q[:, None] * gl, F_e))
    assert deltas[0] > deltas[1] > deltas[2] and deltas[2] < 3e-5
