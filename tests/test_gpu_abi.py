"""The boundary's stream, batch and short-range entry points on the GPU.

A plan given the caller's stream enqueues on it: calls made while that stream
is torch's current stream need no event ordering, and the results are bitwise
those of a plan on its own stream (every sum has a fixed order).
esp_batch_longrange gives every system of a batch its single-system result
bitwise. esp_plan_shortrange_coeffs returns the local kernel of the plan's
split (eq. kernelsplitting), checked against the reference's L(r)."""
import ctypes as C
import math

import numpy as np
import pytest

import workloads as W
from oracle.split import PSWFSplit, L_and_dL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_09727_amd.esp import Plan, esp_local_coeffs, lib  # noqa: E402

DEV = torch.device("cuda:0")


def _buffers(pos, q, dtype=torch.float32):
    tp = torch.tensor(pos, dtype=dtype, device=DEV)
    tq = torch.tensor(q, dtype=dtype, device=DEV)
    phi = torch.empty(len(q), dtype=dtype, device=DEV)
    F = torch.empty((len(q), 3), dtype=dtype, device=DEV)
    return tp, tq, phi, F


@pytest.mark.parametrize("graph", [False, True])
def test_plan_on_the_callers_stream(graph):
    pos, q = W.water_box(3000, 31.0, seed=2)
    print(f"caller stream, graph={graph}", flush=True)
    own = Plan(31.0, len(q), 1e-4)
    tp, tq, phi0, F0 = _buffers(pos, q)
    E0 = own.longrange(tp, tq, phi0, F0)
    torch.cuda.synchronize()
    own.close()
    s = torch.cuda.Stream()
    plan = Plan(31.0, len(q), 1e-4, stream=s)
    assert plan.stream == s.cuda_stream and plan.params[0].stream == s.cuda_stream
    assert plan.params[0].deterministic == 1
    plan.set_graph(graph)
    with torch.cuda.stream(s):
        assert plan._order_after_torch() is None      # same stream: no fences
        tp2, tq2, phi, F = _buffers(pos, q)
        for _ in range(3):
            E = plan.longrange(tp2, tq2, phi, F)
            phi_h, F_h = phi.cpu(), F.cpu()
        assert np.array_equal(E, E0)
        assert torch.equal(phi_h, phi0.cpu()) and torch.equal(F_h, F0.cpu())
    # switching streams: back to the default one, with ordering
    plan.set_stream(torch.cuda.current_stream())
    assert plan.stream in (None, 0, torch.cuda.current_stream().cuda_stream)
    if not graph:   # no graph capture on the null stream
        E2 = plan.longrange(tp2, tq2, phi, F)
        torch.cuda.synchronize()
        assert np.array_equal(E2, E0) and torch.equal(F.cpu(), F0.cpu())
    plan.close()


def test_batch_longrange_matches_single_systems():
    sizes = [(300, 14.4, 31), (1000, 20.0, 32), (2000, 26.0, 33)]
    systems = [W.water_box(n, L, s) for n, L, s in sizes]
    Ls = [L for _, L, _ in sizes]
    Ns = [len(q) for _, q in systems]
    print("batch of 3 systems against each alone", flush=True)
    batch = Plan(Ls, Ns, 1e-4)
    pos = np.concatenate([p for p, _ in systems])
    q = np.concatenate([q for _, q in systems])
    tp, tq, phi, F = _buffers(pos, q)
    E = batch.batch_longrange(tp, tq, phi, F)
    torch.cuda.synchronize()
    off = np.cumsum([0] + Ns)
    for s, ((p, qs), L) in enumerate(zip(systems, Ls)):
        one = Plan(L, len(qs), 1e-4, tile=batch.params[s].tile)
        tp1, tq1, phi1, F1 = _buffers(p, qs)
        E1 = one.longrange(tp1, tq1, phi1, F1)
        torch.cuda.synchronize()
        one.close()
        assert E1[0] == E[s]
        assert torch.equal(F1, F[off[s]:off[s + 1]]) and torch.equal(phi1, phi[off[s]:off[s + 1]])
    batch.close()


def test_profile_launches_cover_the_phase():
    """esp_plan_profile_launches: on a batch of three grid sizes (three
    pipeline lanes) the spread and the gather launch once per lane; the
    launches' particles and grid points add up to the batch's, every launch
    takes a positive time, and their sum is within the phase's time plus
    slack (the per-phase profile runs the same launches back to back)."""
    sizes = [(300, 14.4, 41), (1000, 20.0, 42), (3000, 31.0, 43)]
    systems = [W.water_box(n, L, s) for n, L, s in sizes]
    Ls = [L for _, L, _ in sizes]
    Ns = [len(q) for _, q in systems]
    plan = Plan(Ls, Ns, 1e-4)
    grids = {p.nf for p in plan.params}
    pos = np.concatenate([p for p, _ in systems])
    q = np.concatenate([q for _, q in systems])
    tp, tq, phi, F = _buffers(pos, q)
    print(f"profile launches: grids {sorted(grids)}", flush=True)
    for phase in ("spread", "gather"):
        ls = plan.profile_launches(tp, tq, phi, F, 3, phase)
        assert len(ls) == min(3, len(grids)), ls
        assert sum(L["particles"] for L in ls) == sum(Ns)
        assert sum(L["points"] for L in ls) == sum(p.nf ** 3 for p in plan.params)
        assert all(L["ms"] > 0 for L in ls)
        assert all(L["blocks"] > 0 and L["blocks"] % 8 == 0 for L in ls)  # runs of the 8 XCDs
    with pytest.raises(Exception):
        plan.profile_launches(tp, tq, phi, F, 1, "fft_x_scale")
    plan.close()


def test_shortrange_coeffs_are_the_split_kernel():
    plan = Plan(31.0, 9000, 1e-4)
    p = plan.params[0]
    A, B = plan.shortrange_coeffs()
    A2, B2 = esp_local_coeffs(p)
    assert np.array_equal(A, A2) and np.array_equal(B, B2)
    plan.close()
    # evaluate the documented form against the reference's L(r), L'(r)
    K, d = A.shape[0], A.shape[1] - 1
    rho = p.rc / p.h
    r = np.linspace(0.05, 0.999, 400) * rho             # grid units
    x = r * r / (rho * rho)
    k = np.minimum(np.floor(K * x).astype(int), K - 1)
    y = K * x - k - 0.5
    powers = y[:, None] ** np.arange(d + 1)[None, :]
    hL = 1 / (4 * math.pi * r) - np.sum(A[k] * powers, axis=1)
    h2dL_r = -1 / (4 * math.pi * r ** 3) - np.sum(B[k] * powers, axis=1)
    Lr, dLr = L_and_dL(PSWFSplit(p.c, p.rc), r * p.h)
    scale = np.max(np.abs(p.h * Lr))
    assert np.max(np.abs(hL - p.h * Lr)) < 1e-9 * scale
    assert np.max(np.abs(h2dL_r - p.h ** 2 * dLr / r)) < 1e-9 * np.max(np.abs(p.h ** 2 * dLr / r))
