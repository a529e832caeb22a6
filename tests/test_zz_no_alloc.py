"""The entry point that allocates nothing (esp_longrange_noalloc), through
the C ABI, against the plan-based esp_longrange on the same parameters: two
calls in a row, the second with a smaller system, each bitwise equal to the
plan's result; a system beyond the fixed block is refused before any work."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from oracle.metrics import rel_rms
from parity import elementwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_09727_amd.esp import EspError, Plan, esp_longrange_noalloc, lib  # noqa: E402

DEV = torch.device("cuda:0")


def _buffers(pos, q, dt):
    return (torch.tensor(pos, dtype=dt, device=DEV), torch.tensor(q, dtype=dt, device=DEV),
            torch.empty(len(q), dtype=dt, device=DEV), torch.empty((len(q), 3), dtype=dt, device=DEV))


def _with_plan(L, pos, q, dt, **req):
    plan = Plan(L, len(q), 1e-4, **req)
    tp, tq, phi, F = _buffers(pos, q, dt)
    E = plan.longrange(tp, tq, phi, F)[0]
    torch.cuda.synchronize()
    plan.close()
    return E, phi.cpu(), F.cpu()


@pytest.mark.parametrize("prec", [32, 64])
def test_noalloc_equals_plan_twice_second_smaller(prec):
    dt = torch.float32 if prec == 32 else torch.float64
    cases = [W.water_box(3000, 31.0, seed=2) + (31.0,), W.water_box(400, 16.0, seed=6) + (16.0,)]
    for pos, q, L in cases:
        print(f"no-alloc call: N={len(q)} L={L} prec={prec}", flush=True)
        E_ref, phi_ref, F_ref = _with_plan(L, pos, q, dt, precision=prec)
        tp, tq, phi, F = _buffers(pos, q, dt)
        phi.fill_(np.nan)
        F.fill_(np.nan)
        E = esp_longrange_noalloc(L, tp, tq, phi, F, tol=1e-4, precision=prec)
        if prec == 32:
            # deterministic: bitwise the plan's result
            assert E == E_ref
            assert torch.equal(phi.cpu(), phi_ref) and torch.equal(F.cpu(), F_ref)
        else:
            # the FP64 spread adds with floating-point atomics: equal to rounding
            assert abs(E - E_ref) <= 1e-12 * abs(E_ref)
            assert rel_rms(F.cpu().numpy(), F_ref.numpy()) < 1e-12
            assert rel_rms(phi.cpu().numpy(), phi_ref.numpy()) < 1e-12
            elementwise(F.cpu().numpy(), F_ref.numpy(), 1e-12, "FP64 F")


def test_noalloc_on_a_side_stream_and_raw_abi():
    pos, q, L = W.water_box(1000, 20.0, seed=9) + (20.0,)
    E_ref, phi_ref, F_ref = _with_plan(L, pos, q, torch.float32)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tp, tq, phi, F = _buffers(pos, q, torch.float32)
        box = (C.c_double * 3)(L, L, L)
        E = C.c_double(0.0)
        st = lib().esp_longrange_noalloc(box, len(q), 1e-4, None, C.c_void_p(tp.data_ptr()),
                                         C.c_void_p(tq.data_ptr()), C.c_void_p(phi.data_ptr()),
                                         C.c_void_p(F.data_ptr()), C.byref(E), C.c_void_p(s.cuda_stream))
        assert st == 0, lib().esp_last_error()
        assert E.value == E_ref
        assert torch.equal(F.cpu(), F_ref) and torch.equal(phi.cpu(), phi_ref)


def test_noalloc_refuses_systems_beyond_the_block():
    # a 600,000-atom box at grid 144 needs more than the fixed block; the
    # size is checked before anything is enqueued, so the buffers stay untouched
    N = 600000
    tp = torch.zeros((N, 3), dtype=torch.float32, device=DEV)
    tq = torch.zeros(N, dtype=torch.float32, device=DEV)
    with pytest.raises(EspError) as ei:
        esp_longrange_noalloc(180.0, tp, tq, None, None, tol=1e-4)
    assert ei.value.status == -2 and "bytes" in str(ei.value)
