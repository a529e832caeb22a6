"""Pins of the default-parameter rules by the force error they produce.

The paper leaves c1 ("slightly larger than c") and the cutoff rc (a cost
balance with the short-range code) open. The reference picks c1 as the
argmin of the aliasing estimate E_A (eq. errorformula) and rc = kappa c h/pi
with kappa = 1.2 (eq. pswfparameters with a margin). Here those choices are
checked against the measured error Delta (eq. Deltadef: five-step forces
against classical Ewald minus the local part, over the total Coulomb force),
not against E_A again."""
import numpy as np
import pytest

import workloads as W
from oracle.ewald import ewald
from oracle.fivestep import five_step
from oracle.metrics import rel_rms
from oracle.params import esp_parameters
from oracle.split import PSWFSplit
from oracle.spectral import local_sum


class _Box:
    def __init__(self, pos, q, L):
        self.pos, self.q, self.L = pos, q, L
        _, self.F, _ = ewald(pos, q, L)
        self._local = {}

    def delta(self, prm, c1=None):
        key = (prm["c"], prm["rc"])
        if key not in self._local:
            self._local[key] = local_sum(self.pos, self.q, self.L, PSWFSplit(*key))[1]
        Fs = self.F + self.q[:, None] * self._local[key]          # F^Ewald - F^local
        r = five_step(self.pos, self.q, self.L, prm["n"], prm["P"], prm["c"], prm["rc"],
                      prm["c1"] if c1 is None else c1)
        return rel_rms(r["F"], Fs, self.F)


@pytest.fixture(scope="module")
def water_9000():
    # the 9000-atom water box: L = 31, grid 32, P = 6 at tol 1e-4
    pos, q = W.water_box(3000, 31.0, 2)
    return _Box(pos, q, 31.0)


@pytest.fixture(scope="module")
def nacl_perturbed():
    # the 512-ion rock-salt crystal with +-0.1 displacements, grid 16, P = 6
    pos, q, L = W.nacl_crystal(perturb=0.1, seed=1)
    return _Box(pos, q, L)


def _c1_scan(box, prm):
    xs = np.linspace(0.9, 1.4, 11)
    deltas = np.array([box.delta(prm, x * prm["c"]) for x in xs])
    return xs, deltas


@pytest.mark.slow
@pytest.mark.parametrize("which", ["water_9000", "nacl_perturbed"])
def test_c1_rule_lands_at_the_force_error_minimum(which, request):
    box = request.getfixturevalue(which)
    prm = esp_parameters(box.L, 1e-4, n=16 if which == "nacl_perturbed" else None, P=6)
    xs, deltas = _c1_scan(box, prm)
    chosen = box.delta(prm)
    # the error has an interior minimum over [0.9 c, 1.4 c] ...
    i = int(np.argmin(deltas))
    assert 0 < i < len(xs) - 1 and deltas[0] > 3 * deltas[i] and deltas[-1] > 3 * deltas[i]
    # ... and the E_A argmin sits within 10% of it (measured 2-3%), while a
    # c1 at or just above c (c1/c = 1.0-1.1) costs 1.2x or more
    assert chosen <= 1.10 * deltas.min(), (prm["c1"] / prm["c"], chosen, xs[i], deltas[i])
    assert min(box.delta(prm, x * prm["c"]) for x in (1.0, 1.05, 1.1)) > 1.2 * chosen


@pytest.mark.parametrize("tol", [1e-3, 1e-5])
def test_c1_rule_at_other_orders(tol):
    # P = 5 and P = 8: the same rule, a smaller water box at the ensemble's
    # grid spacing
    pos, q = W.water_box(500, 17.0, 21)
    box = _Box(pos, q, 17.0)
    prm = esp_parameters(17.0, tol)
    _, deltas = _c1_scan(box, prm)
    assert box.delta(prm) <= 1.10 * deltas.min()


@pytest.mark.slow
def test_cutoff_rule(water_9000):
    # At a fixed grid the error falls as rc grows (a wider local part leaves
    # a narrower spectrum to resolve), so kappa has no interior optimum; it
    # trades the local part's cost (~rc^3) against error. kappa = 1, the rule
    # of eq. pswfparameters without margin, already meets the tolerance;
    # the default 1.2 keeps a margin of 4x or more.
    box = water_9000
    ds = []
    for kappa in (1.0, 1.1, 1.2, 1.3):
        prm = esp_parameters(box.L, 1e-4, kappa=kappa)
        assert prm["n"] == 32 and prm["P"] == 6
        ds.append(box.delta(prm))
    assert all(a > b for a, b in zip(ds, ds[1:])), ds
    assert ds[0] <= 1e-4 and ds[2] <= 0.25e-4, ds
