"""Triclinic cells (tilts xy, xz, yz; the index grid over fractional
coordinates): the device path against the reference five-step method in a cell
(oracle.cell), with the local part against triclinic Ewald, positions outside
the cell, the rock-salt Madelung constant in a sheared cell, and a batch mixing
triclinic, orthorhombic and cubic systems.

Workloads: random positions with the water charges (O, H, H repeated) at
0.03 atoms/Å^3 in a 30 x 28 x 26 Å cell with tilts (6, -4, 5) and a
24 x 26 x 22 Å cell with tilts (-8, 5, -3), 4 x 4 x 4 rock-salt cells
described by the lattice vectors a, a + b, c, and 3000 rigid waters in a
rhombic dodecahedron of the 9000-atom box's volume (31^3 Å^3)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.cell import (cell_matrix, ewald_cell, five_step_cell, five_step_cell_ik, five_step_classical_cell,
                         local_sum_cell)
from oracle.metrics import rel_rms
from parity import elementwise
from oracle.split import PSWFSplit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_09727_amd.esp import Plan  # noqa: E402

DEV = torch.device("cuda:0")

CELLS = [(30.0, 28.0, 26.0, 6.0, -4.0, 5.0), (24.0, 26.0, 22.0, -8.0, 5.0, -3.0)]


def run(plan, pos, q):
    dt = torch.float64 if plan.precision == 64 else torch.float32
    tp = torch.tensor(np.ascontiguousarray(pos), dtype=dt, device=DEV)
    tq = torch.tensor(np.ascontiguousarray(q), dtype=dt, device=DEV)
    phi = torch.empty(len(q), dtype=dt, device=DEV)
    F = torch.empty((len(q), 3), dtype=dt, device=DEV)
    E = plan.longrange(tp, tq, phi, F)
    torch.cuda.synchronize()
    return phi.cpu().double().numpy(), F.cpu().double().numpy(), np.asarray(E)


def random_cell(cell, seed, density=0.03, outside=False):
    H = cell_matrix(*cell)
    rng = np.random.default_rng(seed)
    N = 3 * int(density * np.linalg.det(H) / 3)
    s = rng.uniform(0, 1, (N, 3))
    if outside:  # whole lattice vectors away from the cell
        s += rng.integers(-2, 3, (N, 3))
    return s @ H.T, np.tile([W.Q_O, W.Q_H, W.Q_H], N // 3)


def reference(pos, q, p, local):
    H = cell_matrix(p.L, p.Ly, p.Lz, p.xy, p.xz, p.yz)
    r = five_step_cell(pos, q, H, p.nf, p.P, p.c, p.rc, p.c1)
    phi, F = r["phi"], r["F"]
    if local:
        ul, gl = local_sum_cell(pos, q, H, PSWFSplit(p.c, p.rc))
        phi, F = phi + ul, F - q[:, None] * gl
    return phi, F, 0.5 * float(np.dot(q, phi))


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("prec,bar_F,bar_E", [(64, 1e-9, 1e-10), (32, 1e-5, 1e-6)])
@pytest.mark.parametrize("local", [0, 1])
def test_cell_against_reference(cell, prec, bar_F, bar_E, local):
    pos, q = random_cell(cell, seed=int(sum(cell)))
    plan = Plan(cell, len(q), 1e-4, precision=prec, local=local, degree=16 if prec == 64 else None)
    p = plan.params[0]
    assert (p.L, p.Ly, p.Lz, p.xy, p.xz, p.yz) == cell and p.nf == 24
    phi, F, E = run(plan, pos, q)
    plan.close()
    pr = pos if prec == 64 else pos.astype(np.float32).astype(np.float64)
    phi_r, F_r, E_r = reference(pr, q, p, local)
    # E = (1/2) sum q phi cancels between the charges of random positions: its
    # bar scales with (1/2) sum |q phi|, the size of the terms it sums
    eE = abs(E[0] - E_r) / (0.5 * float(np.abs(q * phi_r).sum()))
    eF, ephi = rel_rms(F, F_r), rel_rms(phi, phi_r)
    print(f"cell {cell} N={len(q)} prec={prec} local={local}: relF={eF:.2e} relphi={ephi:.2e} relE={eE:.2e}")
    assert eF < bar_F and ephi < bar_F and eE < bar_E, (eF, ephi, eE)
    elementwise(F, F_r, bar_F, "F")
    elementwise(phi, phi_r, bar_F, "phi")
    if local:
        _, F_e, E_e = ewald_cell(pr, q, cell_matrix(*cell))
        print(f"cell {cell} prec={prec}: Delta={rel_rms(F, F_e):.2e}")
        assert rel_rms(F, F_e) < 1e-4 and abs(E[0] - E_e) < 1e-4 * abs(E_e)


def test_positions_outside_the_cell():
    cell = CELLS[0]
    pos, q = random_cell(cell, seed=9, outside=True)
    plan = Plan(cell, len(q), 1e-4, precision=64, local=1, degree=16)
    phi, F, E = run(plan, pos, q)
    plan.close()
    phi_r, F_r, E_r = reference(pos, q, plan.params[0], 1)
    assert rel_rms(F, F_r) < 1e-9 and rel_rms(phi, phi_r) < 1e-9 and abs(E[0] - E_r) < 1e-10 * abs(E_r)


@pytest.mark.parametrize("prec", [64, 32])
def test_madelung_constant_in_a_sheared_cell(prec):
    pos, q, L = W.nacl_crystal(cells=4)
    cell = (L, L, L, L, 0.0, 0.0)  # lattice vectors a, a + b, c
    plan = Plan(cell, len(q), 1e-4, precision=prec, degree=16 if prec == 64 else None, local=1)
    phi, F, E = run(plan, pos, q)
    plan.close()
    r0 = 5.64 / 2
    M = -phi * q * 4 * math.pi * r0
    print(f"sheared rock salt prec={prec}: max |M - M_ref| = {np.max(np.abs(M - 1.747565)):.2e}, "
          f"max |F| / f_nn = {np.max(np.abs(F)) * 4 * math.pi * r0 ** 2:.2e}")
    assert np.max(np.abs(M - 1.747565)) < 1e-4 * 1.747565
    assert np.max(np.abs(F)) < 2e-4 / (4 * math.pi * r0 ** 2)


def test_batch_of_triclinic_orthorhombic_and_cubic_systems():
    cells = [CELLS[0], (20.0, 20.0, 20.0, 0.0, 0.0, 0.0), CELLS[1], (18.0, 21.0, 24.0, 0.0, 0.0, 0.0)]
    systems = [random_cell(c, seed=60 + i) for i, c in enumerate(cells)]
    Ns = [len(s[1]) for s in systems]
    off = np.cumsum([0] + Ns)
    per = [{"Ly": c[1], "Lz": c[2], "xy": c[3], "xz": c[4], "yz": c[5], "local": 1} for c in cells]
    batch = Plan([c[0] for c in cells], Ns, 1e-4, per_system=per)
    phi_b, F_b, E_b = run(batch, np.concatenate([s[0] for s in systems]), np.concatenate([s[1] for s in systems]))
    batch.close()
    for i, c in enumerate(cells):
        single = Plan(c, Ns[i], 1e-4, local=1)
        phi_s, F_s, E_s = run(single, systems[i][0], systems[i][1])
        single.close()
        sl = slice(off[i], off[i + 1])
        assert np.array_equal(F_s, F_b[sl]) and np.array_equal(phi_s, phi_b[sl]) and E_s[0] == E_b[i], i


def test_rhombic_dodecahedron_water9k_sampled():
    # the benchmark's triclinic workload: the long-range part whole, the local
    # part at 400 sampled atoms; FP32 as timed, and Delta against Ewald
    H = W.rhombic_dodecahedron(31.0 ** 3)
    cell = (H[0, 0], H[1, 1], H[2, 2], H[0, 1], H[0, 2], H[1, 2])
    pos, q = W.water_cell(3000, H, seed=3000)
    plan = Plan(cell, len(q), 1e-4, local=1)
    p = plan.params[0]
    phi, F, E = run(plan, pos, q)
    plan.close()
    x = pos.astype(np.float32).astype(np.float64)
    idx = np.random.default_rng(7).choice(len(q), 400, replace=False)
    r = five_step_cell(x, q, H, p.nf, p.P, p.c, p.rc, p.c1)
    ul, gl = local_sum_cell(x, q, H, PSWFSplit(p.c, p.rc), targets=idx)
    F_r = r["F"][idx] - q[idx, None] * gl
    phi_r = r["phi"][idx] + ul
    eF, ephi = rel_rms(F[idx], F_r), rel_rms(phi[idx], phi_r)
    u_e, F_e, _ = ewald_cell(x, q, H, targets=idx)
    delta = rel_rms(F[idx], F_e)
    print(f"rhombic dodecahedron N={len(q)} n={p.nf}: relF={eF:.2e} relphi={ephi:.2e} Delta(sampled)={delta:.2e}")
    assert eF < 1e-5 and ephi < 1e-5 and delta < 1e-4


def test_graph_replay_and_autotune_in_a_tilted_cell():
    # re-assembly (autotuned bin edges) keeps the per-system influence table;
    # graph replays equal the eager call
    cell = CELLS[1]
    pos, q = random_cell(cell, seed=21)
    plan = Plan(cell, len(q), 1e-4, local=1)
    eager = run(plan, pos, q)
    tp = torch.tensor(pos, dtype=torch.float32, device=DEV)
    tq = torch.tensor(q, dtype=torch.float32, device=DEV)
    phi = torch.empty(len(q), dtype=torch.float32, device=DEV)
    F = torch.empty((len(q), 3), dtype=torch.float32, device=DEV)
    plan.autotune(tp, tq, phi, F, reps=2)
    tuned = run(plan, pos, q)
    plan.set_graph(True)
    for _ in range(3):
        plan.longrange(tp, tq, phi, F)
        torch.cuda.synchronize()
        assert np.array_equal(F.cpu().double().numpy(), tuned[1])
        run(plan, pos, q)  # eager work between replays
    plan.close()
    assert rel_rms(tuned[1], eager[1]) < 1e-6 and rel_rms(tuned[0], eager[0]) < 1e-6


@pytest.mark.parametrize("cell,n_atoms", [((12.0, 13.0, 14.0, 9.0, -7.0, 8.0), 3), ((20.0, 18.0, 16.0, 14.0, 0.0, -11.0), 300)])
def test_small_and_non_reduced_cells(cell, n_atoms):
    # tilts beyond half a side (a non-reduced cell) and a three-atom system
    H = cell_matrix(*cell)
    rng = np.random.default_rng(17)
    pos = rng.uniform(0, 1, (n_atoms, 3)) @ H.T
    q = np.tile([W.Q_O, W.Q_H, W.Q_H], n_atoms // 3)
    # degree 16: the window polynomials exact to FP64 (the default degree fits
    # them to the tolerance, about 1e-5)
    plan = Plan(cell, len(q), 1e-4, precision=64, local=0, degree=16)
    phi, F, E = run(plan, pos, q)
    p = plan.params[0]
    plan.close()
    phi_r, F_r, E_r = reference(pos, q, p, 0)
    print(f"cell {cell} N={n_atoms} n={p.nf}: relF={rel_rms(F, F_r):.2e}")
    assert rel_rms(F, F_r) < 1e-9 and rel_rms(phi, phi_r) < 1e-9
    elementwise(F, F_r, 1e-9, "F")
    elementwise(phi, phi_r, 1e-9, "phi")



@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("prec,bar_F", [(64, 1e-9), (32, 1e-5)])
def test_ik_forces_in_a_tilted_cell(cell, prec, bar_F):
    # spectral derivatives along the fractional coordinates, mapped by H^-T,
    # against the reference ik route; with the local part against Ewald
    pos, q = random_cell(cell, seed=31)
    plan = Plan(cell, len(q), 1e-4, precision=prec, local=1, force_method=1, degree=16 if prec == 64 else None)
    p = plan.params[0]
    phi, F, E = run(plan, pos, q)
    plan.close()
    H = cell_matrix(*cell)
    pr = pos if prec == 64 else pos.astype(np.float32).astype(np.float64)
    r = five_step_cell_ik(pr, q, H, p.nf, p.P, p.c, p.rc, p.c1)
    ul, gl = local_sum_cell(pr, q, H, PSWFSplit(p.c, p.rc))
    F_r, phi_r = r["F"] - q[:, None] * gl, r["phi"] + ul
    eF, ephi = rel_rms(F, F_r), rel_rms(phi, phi_r)
    _, F_e, _ = ewald_cell(pr, q, H)
    print(f"ik cell {cell} prec={prec}: relF={eF:.2e} relphi={ephi:.2e} Delta={rel_rms(F, F_e):.2e}")
    assert eF < bar_F and ephi < bar_F and rel_rms(F, F_e) < 1e-4
    elementwise(F, F_r, bar_F, "ik F")
    elementwise(phi, phi_r, bar_F, "ik phi")
    # the long-range ik forces conserve momentum; the local part does by symmetry
    assert np.abs(F.sum(0)).max() < (1e-10 if prec == 64 else 1e-4) * np.abs(F).max() * len(q)


def test_ik_batch_of_tilted_and_box_systems_equals_each_alone():
    cells = [CELLS[0], (18.0, 21.0, 24.0, 0.0, 0.0, 0.0), CELLS[1]]
    systems = [random_cell(c, seed=70 + i) for i, c in enumerate(cells)]
    Ns = [len(s[1]) for s in systems]
    off = np.cumsum([0] + Ns)
    per = [{"Ly": c[1], "Lz": c[2], "xy": c[3], "xz": c[4], "yz": c[5], "force_method": 1} for c in cells]
    batch = Plan([c[0] for c in cells], Ns, 1e-4, per_system=per)
    phi_b, F_b, E_b = run(batch, np.concatenate([s[0] for s in systems]), np.concatenate([s[1] for s in systems]))
    batch.close()
    for i, c in enumerate(cells):
        single = Plan(c, Ns[i], 1e-4, force_method=1)
        phi_s, F_s, E_s = run(single, systems[i][0], systems[i][1])
        single.close()
        sl = slice(off[i], off[i + 1])
        assert np.array_equal(F_s, F_b[sl]) and np.array_equal(phi_s, phi_b[sl]) and E_s[0] == E_b[i], i



@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("prec,bar_F", [(64, 1e-10), (32, 1e-5)])
@pytest.mark.parametrize("local", [0, 1])
def test_classical_method_in_a_tilted_cell(cell, prec, bar_F, local):
    # Gaussian split and B-spline window on the fractional grid, at the
    # library's classical defaults (P = 5, alpha = log(1/tol), the ESP cutoff)
    from oracle.split import GaussianSplit
    pos, q = random_cell(cell, seed=41)
    plan = Plan(cell, len(q), 1e-4, precision=prec, local=local, method=1)
    p = plan.params[0]
    assert p.method == 1
    phi, F, E = run(plan, pos, q)
    plan.close()
    H = cell_matrix(*cell)
    pr = pos if prec == 64 else pos.astype(np.float32).astype(np.float64)
    r = five_step_classical_cell(pr, q, H, p.nf, p.P, p.c, p.rc)
    phi_r, F_r = r["phi"], r["F"]
    if local:
        ul, gl = local_sum_cell(pr, q, H, GaussianSplit(p.c, p.rc, support=p.rc))
        phi_r, F_r = phi_r + ul, F_r - q[:, None] * gl
    eF, ephi = rel_rms(F, F_r), rel_rms(phi, phi_r)
    msg = f"classical cell {cell} n={p.nf} P={p.P} prec={prec} local={local}: relF={eF:.2e} relphi={ephi:.2e}"
    if local:
        _, F_e, _ = ewald_cell(pr, q, H)
        msg += f" Delta={rel_rms(F, F_e):.2e}"
    print(msg)
    assert eF < bar_F and ephi < bar_F
    elementwise(F, F_r, bar_F, "F")
    elementwise(phi, phi_r, bar_F, "phi")
