"""Pins of the orthorhombic-box reference (oracle.box): cubic special cases
against the cubic functions, the Madelung constant of a non-cubic rock-salt
supercell, axis permutations, and the five-step method against Ewald."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.box import ewald_box, five_step_box, influence_box, local_sum_box
from oracle.ewald import ewald
from oracle.fivestep import five_step, influence
from oracle.metrics import rel_rms
from oracle.params import esp_parameters
from oracle.split import PSWFSplit
from oracle.spectral import local_sum

MADELUNG = 1.747565


def test_cubic_box_reduces_to_the_cubic_functions():
    pos, q = W.water_box(150, 14.0, seed=3)
    L = 14.0
    u1, F1, E1 = ewald(pos, q, L)
    u2, F2, E2 = ewald_box(pos, q, (L, L, L))
    assert np.max(np.abs(u2 - u1)) < 1e-12 * np.max(np.abs(u1))
    assert np.max(np.abs(F2 - F1)) < 1e-11 * np.max(np.abs(F1))
    pr = esp_parameters(L, 1e-4)
    pc = influence(pr["n"], L, pr["P"], pr["c"], pr["rc"], pr["c1"])
    pb = influence_box(pr["n"], (L, L, L), pr["P"], pr["c"], pr["rc"], pr["c1"])
    # equal up to the rounding of |k| (amplified where the transform's
    # quadrature cancels, at the corner modes)
    assert np.max(np.abs(pb - pc)) < 1e-10 * np.max(np.abs(pc))
    r1 = five_step(pos, q, L, pr["n"], pr["P"], pr["c"], pr["rc"], pr["c1"])
    r2 = five_step_box(pos, q, (L, L, L), pr["n"], pr["P"], pr["c"], pr["rc"], pr["c1"])
    assert rel_rms(r2["F"], r1["F"]) < 1e-13
    sp = PSWFSplit(pr["c"], pr["rc"])
    ul1, gl1 = local_sum(pos, q, L, sp)
    ul2, gl2 = local_sum_box(pos, q, (L, L, L), sp)
    assert np.max(np.abs(ul2 - ul1)) < 1e-13 and np.max(np.abs(gl2 - gl1)) < 1e-12


def test_madelung_constant_of_a_non_cubic_supercell():
    # 4 x 4 x 2 conventional cells: the same crystal in a 22.56 x 22.56 x 11.28 box
    pos, q, L = W.nacl_crystal(cells=4)
    keep = pos[:, 2] < L / 2 - 1e-9
    pos, q = pos[keep], q[keep]
    box = (L, L, L / 2)
    u, F, E = ewald_box(pos, q, box)
    r0 = 5.64 / 2
    M = -u * q * 4 * math.pi * r0
    assert np.max(np.abs(M - MADELUNG)) < 1e-6
    assert np.max(np.abs(F)) < 1e-12


def test_axis_permutation():
    rng = np.random.default_rng(7)
    box = np.array([13.0, 16.0, 19.0])
    pos = rng.uniform(0, 1, (300, 3)) * box
    q = np.tile([1.0, -1.0], 150)
    perm = [2, 0, 1]
    u, F, E = ewald_box(pos, q, box)
    u2, F2, E2 = ewald_box(pos[:, perm], q, box[perm])
    assert np.max(np.abs(u2 - u)) < 1e-11 * np.max(np.abs(u))
    assert np.max(np.abs(F2 - F[:, perm])) < 1e-10 * np.max(np.abs(F))
    n, P, c, rc, c1 = 24, 6, 12.024, 4.8, 12.5
    a = five_step_box(pos, q, box, n, P, c, rc, c1)
    b = five_step_box(pos[:, perm], q, box[perm], n, P, c, rc, c1)
    assert rel_rms(b["F"], a["F"][:, perm]) < 1e-12


@pytest.mark.parametrize("box,tol", [((18.0, 21.0, 24.0), 1e-4), ((24.0, 24.0, 16.0), 1e-3)])
def test_five_step_in_a_box_reaches_the_tolerance(box, tol):
    # random positions with the water charges (O, H, H repeated), neutral
    box = np.array(box)
    rng = np.random.default_rng(11)
    N = 3 * int(0.03 * np.prod(box))
    pos = rng.uniform(0, 1, (N, 3)) * box
    q = np.tile([W.Q_O, W.Q_H, W.Q_H], N // 3)
    pr = esp_parameters(float(box.max()), tol)
    n, P, c, c1 = pr["n"], pr["P"], pr["c"], pr["c1"]
    rc = pr["rc"]  # kappa c h_max / pi with h_max = max(L)/n
    r = five_step_box(pos, q, box, n, P, c, rc, c1)
    ul, gl = local_sum_box(pos, q, box, PSWFSplit(c, rc))
    F = r["F"] - q[:, None] * gl
    u_e, F_e, E_e = ewald_box(pos, q, box)
    assert rel_rms(F, F_e) < tol
    assert abs(0.5 * np.dot(q, r["phi"] + ul) - E_e) < tol * abs(E_e)
