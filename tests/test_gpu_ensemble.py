"""Batched ensemble of uneven systems through one plan (one launch per phase
for all systems) against the CPU reference, before and after autotuning.

Workload: 256 water-like boxes at 1 g/cm^3, atom counts log-uniform in
[500, 20000] (seeded), tol 1e-4, FP32 (grids 16^3 .. 48^3, six distinct
sizes). Every system is compared with the reference five-step method (exact
window, matrix DFT) at the library's parameters: relative RMS force error
below 1e-4 and relative energy error below 1e-5, the bars of the single
system tests, and no particle's force or potential off by more than
10 x 1e-4 of the system's RMS value."""
import numpy as np
import pytest

import workloads as W
from oracle.fivestep import five_step
from oracle.metrics import rel_rms
from parity import elementwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_09727_amd.esp import Plan  # noqa: E402

DEV = torch.device("cuda:0")
NSYS = 256
CHUNKS = 8


@pytest.fixture(scope="module")
def ensemble_results():
    systems = W.ensemble(n_sys=NSYS)
    Ls = [s[2] for s in systems]
    Ns = [len(s[1]) for s in systems]
    off = np.cumsum([0] + Ns)
    pos = torch.tensor(np.concatenate([s[0] for s in systems]), dtype=torch.float32, device=DEV)
    q = torch.tensor(np.concatenate([s[1] for s in systems]), dtype=torch.float32, device=DEV)
    plan = Plan(Ls, Ns, 1e-4)
    phi = torch.empty(off[-1], dtype=torch.float32, device=DEV)
    F = torch.empty((off[-1], 3), dtype=torch.float32, device=DEV)
    E = plan.longrange(pos, q, phi, F)
    torch.cuda.synchronize()
    res = dict(systems=systems, off=off, params=list(plan.params), E=E,
               F=F.cpu().double().numpy(), phi=phi.cpu().double().numpy())
    tiles = plan.autotune(pos, q, phi, F, reps=2)
    E2 = plan.longrange(pos, q, phi, F)
    torch.cuda.synchronize()
    res.update(tiles=tiles, E_tuned=E2, F_tuned=F.cpu().double().numpy(), phi_tuned=phi.cpu().double().numpy(),
               params_tuned=list(plan.params))
    plan.close()
    return res


def test_ensemble_shapes(ensemble_results):
    r = ensemble_results
    ns = sorted({p.nf for p in r["params"]})
    assert len(r["systems"]) == NSYS
    assert ns[0] == 16 and ns[-1] == 48 and len(ns) >= 4
    assert all(p.P == 6 for p in r["params"])
    # the autotuner only changes bin edges, to admissible divisors of n
    for p0, p1, T in zip(r["params"], r["params_tuned"], r["tiles"]):
        assert (p1.nf, p1.P, p1.c1, p1.rc) == (p0.nf, p0.P, p0.c1, p0.rc)
        assert p1.tile == T and p0.nf % T == 0 and 8 <= T <= 16


@pytest.mark.parametrize("chunk", range(CHUNKS))
def test_ensemble_vs_reference(ensemble_results, chunk):
    r = ensemble_results
    off = r["off"]
    for s in range(chunk, NSYS, CHUNKS):
        pos, q, L = r["systems"][s]
        p = r["params"][s]
        ref = five_step(pos, q, L, p.nf, p.P, p.c, p.rc, p.c1)
        sl = slice(off[s], off[s + 1])
        for F, phi, E in ((r["F"], r["phi"], r["E"]), (r["F_tuned"], r["phi_tuned"], r["E_tuned"])):
            assert rel_rms(F[sl], ref["F"]) < 1e-4, (s, p.nf, len(q))
            assert rel_rms(phi[sl], ref["phi"]) < 1e-4, (s, p.nf, len(q))
            elementwise(F[sl], ref["F"], 1e-4, f"F system {s}")
            elementwise(phi[sl], ref["phi"], 1e-4, f"phi system {s}")
            assert abs(E[s] - ref["E"]) < 1e-5 * abs(ref["E"]), (s, E[s], ref["E"])


def test_autotuned_matches_default_tiles(ensemble_results):
    # the fixed-point spread is exact; only the halo fold's float sums and
    # nothing else depend on the bin edge
    r = ensemble_results
    assert rel_rms(r["F_tuned"], r["F"]) < 1e-5
    assert np.max(np.abs(r["E_tuned"] - r["E"]) / np.abs(r["E"])) < 1e-6
