"""Local part of the split on the device (local = 1): phi, F and E become the
full Coulomb values of the problem statement.

Checked against the reference five-step method plus the reference local sum
(brute force over nearest images with the exact kernel L(r) = (1 - G(r/rc))/
(4 pi r)) at the library's parameters, and against classical Ewald: the
full-Coulomb force error the paper reports (Delta) at the requested tolerance,
and the Madelung constant of rock salt. Workloads: the rock-salt crystal
(exact and perturbed, 512 ions), the 9000-atom water-like box (L = 31), a
700-atom box at three window widths and two bin edges, and small boxes whose
sub-cell grid wraps onto itself."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.ewald import ewald
from oracle.fivestep import five_step
from oracle.metrics import rel_rms
from parity import elementwise
from oracle.split import PSWFSplit
from oracle.spectral import local_sum

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_09727_amd.esp import Plan  # noqa: E402

DEV = torch.device("cuda:0")
MADELUNG = 1.747565
# FP64 checks use degree-16 window polynomials, so that the window fit (the
# reference uses the exact window) stays below the 1e-9 bars; FP32 runs at the
# library's degree for the tolerance
DEG = {64: 16, 32: None}


def _t(a, prec):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64 if prec == 64 else torch.float32, device=DEV)


def run(plan, pos, q, off=None):
    prec = plan.precision
    tp, tq = _t(pos, prec), _t(q, prec)
    phi = torch.empty(len(q), dtype=tp.dtype, device=DEV)
    F = torch.empty((len(q), 3), dtype=tp.dtype, device=DEV)
    E = plan.longrange(tp, tq, phi, F)
    torch.cuda.synchronize()
    return phi.cpu().double().numpy(), F.cpu().double().numpy(), np.asarray(E)


def full_reference(pos, q, p):
    """Five-step long-range part plus the local part: full Coulomb phi, F, E."""
    pos = np.asarray(pos, np.float64)
    r = five_step(pos, q, p.L, p.nf, p.P, p.c, p.rc, p.c1)
    ul, gl = local_sum(pos, q, p.L, PSWFSplit(p.c, p.rc))
    phi = r["phi"] + ul
    F = r["F"] - q[:, None] * gl
    return phi, F, 0.5 * float(np.dot(q, phi))


def _rounded(pos, prec):
    return pos if prec == 64 else pos.astype(np.float32).astype(np.float64)


def check(plan, pos, q, bar_F, bar_E, F_scale=None):
    phi, F, E = run(plan, pos, q)
    p = plan.params[0]
    assert p.local == 1
    phi_r, F_r, E_r = full_reference(_rounded(pos, plan.precision), q, p)
    eF = rel_rms(F, F_r) if F_scale is None else np.sqrt(np.mean((F - F_r) ** 2)) / F_scale
    ephi, eE = rel_rms(phi, phi_r), abs(E[0] - E_r) / abs(E_r)
    print(f"N={len(q)} n={p.nf} P={p.P} T={p.tile} prec={plan.precision}: relF={eF:.2e} "
          f"relphi={ephi:.2e} relE={eE:.2e}")
    assert eF < bar_F and ephi < bar_F and eE < bar_E, (eF, ephi, eE)
    if F_scale is None:
        elementwise(F, F_r, bar_F, "full F")
    elementwise(phi, phi_r, bar_F, "full phi")
    # the energy is (1/2) sum q phi of the returned potentials
    assert abs(E[0] - 0.5 * np.dot(q, phi)) < 10 * bar_E * abs(E[0])
    return phi, F, E


def test_madelung_constant_on_the_device():
    pos, q, L = W.nacl_crystal()
    plan = Plan(L, len(q), 1e-4, nf=16, P=6, precision=64, degree=16, local=1)
    # forces vanish by symmetry: measure them against the force between two
    # unit charges at the nearest-neighbour distance
    r0 = 5.64 / 2
    phi, F, E = check(plan, pos, q, 1e-9, 1e-10, F_scale=1.0 / (4 * math.pi * r0 ** 2))
    M = -phi * q * 4 * math.pi * r0
    assert np.max(np.abs(M - MADELUNG)) < 1e-4 * MADELUNG
    assert abs(-E[0] * 4 * math.pi * r0 / (len(q) / 2) - MADELUNG) < 1e-4 * MADELUNG
    assert np.max(np.abs(F)) < 1e-4 / (4 * math.pi * r0 ** 2)
    plan.close()


@pytest.mark.parametrize("prec,bar_F,bar_E", [(64, 1e-9, 1e-10), (32, 1e-5, 1e-6)])
def test_perturbed_nacl_against_ewald(prec, bar_F, bar_E):
    pos, q, L = W.nacl_crystal(perturb=0.1, seed=1)
    plan = Plan(L, len(q), 1e-4, nf=16, P=6, precision=prec, degree=DEG[prec], local=1)
    phi, F, E = check(plan, pos, q, bar_F, bar_E)
    u_e, F_e, E_e = ewald(_rounded(pos, prec), q, L)
    delta = rel_rms(F, F_e)
    print(f"perturbed NaCl prec={prec}: Delta={delta:.2e} relE={abs(E[0] - E_e) / abs(E_e):.2e}")
    # the crystal's forces are small restoring forces left after near
    # cancellation, so their relative error is about twice the tolerance
    # (the reference method itself gives 2.0e-4 here)
    assert delta < 3e-4 and abs(E[0] - E_e) < 1e-4 * abs(E_e)
    plan.close()


@pytest.fixture(scope="module")
def water9k():
    pos, q = W.water_box(3000, 31.0, seed=2)
    u, F, E = ewald(pos, q, 31.0)
    return pos, q, 31.0, F, E


@pytest.mark.parametrize("prec,bar_F,bar_E", [(64, 1e-9, 1e-10), (32, 1e-5, 1e-6)])
def test_water9k_full_coulomb(water9k, prec, bar_F, bar_E):
    pos, q, L, F_ewald, E_ewald = water9k
    plan = Plan(L, len(q), 1e-4, precision=prec, degree=DEG[prec], local=1)
    phi, F, E = check(plan, pos, q, bar_F, bar_E)
    # the paper's error measure on the full forces, against Ewald
    delta = rel_rms(F, F_ewald)
    print(f"water9k prec={prec}: Delta={delta:.2e} relE={abs(E[0] - E_ewald) / abs(E_ewald):.2e}")
    assert delta < 1e-4
    assert abs(E[0] - E_ewald) < 1e-4 * abs(E_ewald)
    plan.close()


@pytest.mark.parametrize("tol,P,n,tile", [(1e-3, 5, 24, 8), (1e-5, 8, 24, 12), (1e-4, 7, 36, 12),
                                          (1e-4, 6, 24, 8)])
def test_other_orders_bins_and_sizes(tol, P, n, tile):
    pos, q = W.water_box(700, 20.0, seed=P)
    for prec, bar in ((64, 1e-9), (32, max(1e-5, tol / 10))):
        plan = Plan(20.0, len(q), tol, nf=n, P=P, precision=prec, tile=tile, degree=DEG[prec], local=1)
        assert plan.params[0].tile == tile
        check(plan, pos, q, bar, bar / 10)
        plan.close()


@pytest.mark.parametrize("L,n_mol", [(13.0, 120), (17.1, 166)])
def test_small_boxes_with_wrapped_stencils(L, n_mol):
    # few bins per side: the stencil around a sub-cell reaches the same
    # sub-cells through more than one periodic image
    pos, q = W.water_box(n_mol, L, seed=9)
    plan = Plan(L, len(q), 1e-4, precision=64, degree=16, local=1)
    p = plan.params[0]
    assert p.nf // p.tile <= 2 and p.rc <= L / 2
    check(plan, pos, q, 1e-9, 1e-10)
    plan.close()


def test_ragged_positions_and_edges():
    # positions far outside the box, exactly on bin and box boundaries, and
    # close pairs
    pos, q = W.water_box(400, 16.0, seed=4)
    pos = pos.copy()
    pos[:20] += 16.0 * np.arange(-10, 10)[:, None]
    pos[20:26, 0] = [0.0, 8.0, 16.0 - 1e-12, 4.0, 12.0, 15.999]
    pos[26] = pos[27] + np.array([0.05, 0.0, 0.0])
    plan = Plan(16.0, len(q), 1e-4, precision=64, degree=16, local=1)
    check(plan, pos, q, 1e-9, 1e-10)
    plan.close()


def test_dense_cluster_takes_the_global_paths():
    # 4500 of 6000 atoms packed into one bin: that bin's sub-cell sort runs
    # beyond its LDS staging and the halos around it exceed the pair pass's
    # LDS staging, so both take their global-memory paths; the rest of the box
    # stays on the staged paths
    pos, q = W.water_box(2000, 24.0, seed=11)
    rng = np.random.default_rng(11)
    pos = pos.copy()
    pos[:4500] = rng.uniform(0.5, 7.5, size=(4500, 3))
    plan = Plan(24.0, len(q), 1e-4, precision=64, degree=16, local=1)
    p = plan.params[0]
    assert p.tile * p.h >= 7.5
    check(plan, pos, q, 1e-9, 1e-10)
    plan.close()


def test_batch_alone_and_binning_paths_bitwise():
    # 70 small systems take the one-block binning in a batch and the chunked
    # kernels alone; the local sums run in the canonical sub-cell order either
    # way, so every output is bitwise identical. The batch also mixes in
    # systems without the local part.
    systems = [W.water_box_at_density(3 * (200 + 37 * i % 400), seed=100 + i) for i in range(70)]
    Ls = [s[2] for s in systems]
    Ns = [len(s[1]) for s in systems]
    off = np.cumsum([0] + Ns)
    locals_ = [0 if i % 7 == 3 else 1 for i in range(70)]
    pos = np.concatenate([s[0] for s in systems])
    q = np.concatenate([s[1] for s in systems])
    batch = Plan(Ls, Ns, 1e-4, per_system=[{"local": l} for l in locals_])
    phi_b, F_b, E_b = run(batch, pos, q)
    phi_b2, F_b2, E_b2 = run(batch, pos, q)
    batch.close()
    assert np.array_equal(F_b, F_b2) and np.array_equal(phi_b, phi_b2) and np.array_equal(E_b, E_b2)
    for i in (0, 3, 17, 41, 69):
        sl = slice(off[i], off[i + 1])
        single = Plan(Ls[i], Ns[i], 1e-4, local=locals_[i])
        phi_s, F_s, E_s = run(single, systems[i][0], systems[i][1])
        single.close()
        assert np.array_equal(F_s, F_b[sl]) and np.array_equal(phi_s, phi_b[sl]), i
        assert E_s[0] == E_b[i], i
    # one system against the full reference
    p = Plan(Ls[0], Ns[0], 1e-4, local=1)
    phi_r, F_r, E_r = full_reference(systems[0][0].astype(np.float32).astype(np.float64), systems[0][1],
                                     p.params[0])
    p.close()
    assert rel_rms(F_b[off[0]:off[1]], F_r) < 1e-5


def test_translation_invariance_of_the_local_part():
    # a shift by whole grid spacings leaves every output unchanged up to
    # rounding (bins and sub-cells move, pairs do not)
    pos, q = W.water_box(500, 18.0, seed=6)
    plan = Plan(18.0, len(q), 1e-4, precision=64, local=1)
    phi, F, E = run(plan, pos, q)
    h = plan.params[0].h
    phi2, F2, E2 = run(plan, pos + h * np.array([3, -5, 11]), q)
    plan.close()
    assert rel_rms(F2, F) < 1e-11 and abs(E2[0] - E[0]) < 1e-12 * abs(E[0])


def test_graph_replay_with_the_local_part():
    # a batch with the local part captured as one HIP graph: every replay,
    # with eager work and synchronisations between replays, equals the eager
    # result bitwise
    systems = [W.water_box_at_density(3 * (900 + 200 * i), seed=500 + i) for i in range(4)]
    Ls = [s[2] for s in systems]
    Ns = [len(s[1]) for s in systems]
    pos = torch.tensor(np.concatenate([s[0] for s in systems]), dtype=torch.float32, device=DEV)
    q = torch.tensor(np.concatenate([s[1] for s in systems]), dtype=torch.float32, device=DEV)
    plan = Plan(Ls, Ns, 1e-4, local=1)
    phi = torch.empty(sum(Ns), dtype=torch.float32, device=DEV)
    F = torch.empty((sum(Ns), 3), dtype=torch.float32, device=DEV)
    E0 = np.asarray(plan.longrange(pos, q, phi, F))
    F0, phi0 = F.clone(), phi.clone()
    plan.set_graph(True)
    for rep in range(4):
        F.zero_()
        phi.zero_()
        torch.cuda.synchronize()
        E = np.asarray(plan.longrange(pos, q, phi, F))
        torch.cuda.synchronize()
        assert torch.equal(F, F0) and torch.equal(phi, phi0) and np.array_equal(E, E0), rep
    plan.close()


def test_autotune_keeps_the_local_part():
    # the autotuner rebuilds the plan (new bin edges, new local-part scratch):
    # results before and after agree with each other and with the reference
    pos, q = W.water_box(1500, 24.0, seed=8)
    plan = Plan(24.0, len(q), 1e-4, local=1)
    tp = torch.tensor(pos, dtype=torch.float32, device=DEV)
    tq = torch.tensor(q, dtype=torch.float32, device=DEV)
    phi = torch.empty(len(q), dtype=torch.float32, device=DEV)
    F = torch.empty((len(q), 3), dtype=torch.float32, device=DEV)
    E0 = plan.longrange(tp, tq, phi, F)[0]
    F0 = F.cpu().double().numpy()
    tiles = plan.autotune(tp, tq, phi, F, reps=2)
    E1 = plan.longrange(tp, tq, phi, F)[0]
    F1 = F.cpu().double().numpy()
    p = plan.params[0]
    plan.close()
    assert p.tile == tiles[0] and p.local == 1
    assert rel_rms(F1, F0) < 1e-5 and abs(E1 - E0) < 1e-6 * abs(E0)
    _, F_r, E_r = full_reference(pos.astype(np.float32).astype(np.float64), q, p)
    assert rel_rms(F1, F_r) < 1e-5 and abs(E1 - E_r) < 1e-6 * abs(E_r)


def test_large_water_full_coulomb_sampled():
    # the 300,000-atom box (L = 100, tol 1e-5, n = 96, P = 8) with the local
    # part: forces and potentials at 2000 sampled particles against the
    # reference five-step method plus the local sum at those particles
    cfg = W.WATER_300K
    pos, q = W.water_box(cfg["n_mol"], cfg["L"], cfg["seed"])
    L, tol = cfg["L"], cfg["tol"]
    plan = Plan(L, len(q), tol, local=1)
    p = plan.params[0]
    assert (p.nf, p.P) == (96, 8)
    phi, F, E = run(plan, pos, q)
    plan.close()
    bad = np.flatnonzero(~(np.isfinite(phi) & np.isfinite(F).all(1)))
    assert len(bad) == 0 and np.isfinite(E[0]), f"device output not finite at {len(bad)} particles: {bad[:8]}, E={E}"
    pr = pos.astype(np.float32).astype(np.float64)
    r = five_step(pr, q, L, p.nf, p.P, p.c, p.rc, p.c1)
    idx = np.random.default_rng(3).choice(len(q), 2000, replace=False)
    ul, gl = local_sum(pr, q, L, PSWFSplit(p.c, p.rc), targets=idx)
    F_r = r["F"][idx] - q[idx, None] * gl
    phi_r = r["phi"][idx] + ul
    parts = {"spread b": r["b"], "b^": r["bhat"], "p": r["p"], "c^": r["chat"], "c": r["c"],
             "five_step F": r["F"], "five_step phi": r["phi"], "local u": ul, "local grad": gl}
    assert np.isfinite(F_r).all() and np.isfinite(phi_r).all(), \
        "reference not finite: " + ", ".join(f"{k} {int((~np.isfinite(v)).sum())}" for k, v in parts.items())
    eF, ephi = rel_rms(F[idx], F_r), rel_rms(phi[idx], phi_r)
    # molecules placed at random at three times liquid density leave some
    # atoms of different molecules a few hundredths of an angstrom apart;
    # those pairs take their displacement in FP64, so the sampled atoms with
    # such a contact meet the tolerance like the others
    from scipy.spatial import cKDTree
    d_nn = cKDTree(np.mod(pr, L), boxsize=L).query(np.mod(pr[idx], L), k=2)[0][:, 1]
    far = d_nn >= 0.5
    print(f"300k full Coulomb, 2000 samples: relF={eF:.2e} relphi={ephi:.2e}; "
          f"{far.sum()} without a contact < 0.5 A: relF={rel_rms(F[idx][far], F_r[far]):.2e}; "
          f"{(~far).sum()} with one: relF={rel_rms(F[idx][~far], F_r[~far]):.2e}")
    assert eF < 1e-5 and ephi < 1e-5
    elementwise(F[idx], F_r, 1e-5, "full F (sampled)")
    elementwise(phi[idx], phi_r, 1e-5, "full phi (sampled)")
