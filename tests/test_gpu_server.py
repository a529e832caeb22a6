"""Serving: continuous batching of independent long-range solves (esp_server_*)
through the C ABI. Results are checked against the CPU reference on the
host-reproduced drifted positions, alone vs in a mix, and under an HBM
budget that forces queueing."""
import time

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

from paper_2505_09727_amd.esp import EspError, Server, esp_plan_query  # noqa: E402


def _system(kind, n, seed):
    if kind == "water":
        return W.water_box_at_density(n - n % 3, seed)
    return W.ionic_melt(n, seed)


def _final_positions(pos, L, nsteps, seed, drift):
    p = pos.astype(np.float32)
    for k in range(1, nsteps):
        p = W.serving_drift(p, L, k, seed, drift)
    return p


def test_served_results_match_reference():
    srv = Server(hbm_budget_bytes=256 << 20, keep_outputs=True)
    cases = [("water", 3000, 1e-4, 11), ("melt", 2000, 1e-3, 12), ("water", 6000, 1e-5, 13)]
    ids = {}
    for kind, n, tol, seed in cases:
        pos, q, L = _system(kind, n, seed)
        rid = srv.submit(pos, q, L, tol, nsteps=3, drift=0.01, seed=seed, tag=seed)
        ids[rid] = (pos, q, L, tol, seed)
    srv.wait(120)
    res = {r["id"]: r for r in srv.poll()}
    assert set(res) == set(ids)
    for rid, (pos, q, L, tol, seed) in ids.items():
        r = res[rid]
        assert r["status"] == 0 and r["nsteps"] == 3
        phi, F = srv.fetch(rid, len(q))
        pfin = _final_positions(pos, L, 3, seed, 0.01)
        p = esp_plan_query(L, len(q), tol)
        ref = five_step(pfin.astype(np.float64), q, L, p.nf, p.P, p.c, p.rc, p.c1)
        eF = rel_rms(F.astype(np.float64), ref["F"])
        print(f"served N={len(q)} tol={tol}: relF={eF:.2e} E={r['E_last']:.6g} ref={ref['E']:.6g}")
        assert eF < tol
        elementwise(F, ref["F"], tol, "served F")
        elementwise(phi, ref["phi"], tol, "served phi")
        assert abs(r["E_last"] - ref["E"]) < 1e-5 * abs(ref["E"])
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
    srv.close()


def test_alone_equals_in_the_mix():
    pos, q, L = _system("water", 4500, 21)
    alone = Server(keep_outputs=True, hbm_budget_bytes=256 << 20)
    rid = alone.submit(pos, q, L, 1e-4, nsteps=4, drift=0.02, seed=5)
    alone.wait(60)
    r_alone = alone.poll()[0]
    phi_a, F_a = alone.fetch(rid, len(q))
    alone.close()
    mix = Server(keep_outputs=True, hbm_budget_bytes=512 << 20)
    others = [_system(k, n, s) for k, n, s in [("melt", 8000, 1), ("water", 12000, 2), ("water", 1500, 3),
                                                 ("melt", 3000, 4)]]
    for i, (p2, q2, L2) in enumerate(others[:2]):
        mix.submit(p2, q2, L2, [1e-3, 1e-5][i], nsteps=6, drift=0.01, seed=100 + i)
    rid2 = mix.submit(pos, q, L, 1e-4, nsteps=4, drift=0.02, seed=5)
    for i, (p2, q2, L2) in enumerate(others[2:]):
        mix.submit(p2, q2, L2, 1e-4, nsteps=2, drift=0.01, seed=200 + i)
    mix.wait(120)
    res = {r["id"]: r for r in mix.poll()}
    phi_m, F_m = mix.fetch(rid2, len(q))
    mix.close()
    # fixed-point spread and fixed reduction orders: bitwise identical
    assert np.array_equal(F_m, F_a) and np.array_equal(phi_m, phi_a)
    assert res[rid2]["E_last"] == r_alone["E_last"]


def test_admission_by_budget_queues_and_completes():
    # each 9000-atom request needs about 1.2 MB of device state, so a 3 MB
    # budget admits two at a time and the rest wait for memory
    systems = [_system("water", 9000, 40 + i) for i in range(8)]
    budget = 3 << 20
    srv = Server(hbm_budget_bytes=budget, max_active=64)
    for i, (pos, q, L) in enumerate(systems):
        srv.submit(pos, q, L, 1e-4, nsteps=5, drift=0.01, seed=i, tag=i)
    srv.wait(120)
    res = sorted(srv.poll(), key=lambda r: r["tag"])
    st = srv.stats()
    srv.close()
    assert len(res) == 8 and all(r["status"] == 0 for r in res)
    assert st["bytes_peak"] <= budget and st["bytes_in_use"] == 0
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)            # FIFO admission
    # at most two resident at any time: the third waited for a completion
    assert res[2]["t_admit"] >= min(res[0]["t_done"], res[1]["t_done"])
    for i in range(len(res)):
        live = sum(1 for r in res if r["t_admit"] <= res[i]["t_admit"] < r["t_done"])
        assert live <= 2
    assert st["completed"] == 8 and st["p99_latency_s"] >= st["p50_latency_s"] > 0


def test_continuous_batching_overlaps_requests():
    long_pos, long_q, long_L = _system("water", 30000, 7)
    shorts = [_system("melt", 2000, 10 + i) for i in range(4)]
    srv = Server(hbm_budget_bytes=512 << 20)
    # warm the parameter caches so submission itself is quick
    for p2, q2, L2 in shorts[:1]:
        srv.submit(p2, q2, L2, 1e-3, nsteps=1)
    srv.submit(long_pos, long_q, long_L, 1e-4, nsteps=1)
    srv.wait(60)
    srv.poll()
    rid_long = srv.submit(long_pos, long_q, long_L, 1e-4, nsteps=3000, drift=0.01, seed=1)
    time.sleep(0.02)
    short = [srv.submit(p2, q2, L2, 1e-3, nsteps=3, seed=i) for i, (p2, q2, L2) in enumerate(shorts)]
    srv.wait(120)
    res = {r["id"]: r for r in srv.poll()}
    srv.close()
    # the short requests were admitted and finished while the long one ran
    for rid in short:
        assert res[rid]["t_submit"] < res[rid_long]["t_done"]
        assert res[rid]["t_admit"] < res[rid_long]["t_done"]
        assert res[rid]["t_done"] < res[rid_long]["t_done"]


def test_request_larger_than_budget_is_refused():
    srv = Server(hbm_budget_bytes=4 << 20)
    pos, q, L = _system("water", 60000, 3)
    with pytest.raises(EspError) as ei:
        srv.submit(pos, q, L, 1e-4)
    assert ei.value.status == -6
    srv.close()
