"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol esp.h declares, and its parameter rules and tables agree with the
independent CPU reference."""
import math
import os
import re

import numpy as np
import pytest

from conftest import ROOT

esp = pytest.importorskip("paper_2505_09727_amd.esp")

from oracle.fivestep import influence, phi_hat_1d          # noqa: E402
from oracle.params import aliasing_error, esp_parameters    # noqa: E402
from oracle.pswf import c_for_tolerance, pswf              # noqa: E402
from oracle.split import PSWFSplit, L_and_dL               # noqa: E402


def _lib_or_skip():
    try:
        return esp.lib()
    except RuntimeError as e:
        pytest.skip(str(e))


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "esp.h")).read()
    names = set(re.findall(r"\b(esp_[a-z_0-9]+)\s*\(", hdr))
    assert len(names) >= 18
    for n in sorted(names):
        assert hasattr(L, n), n
    assert "gfx950" in esp.esp_version()


@pytest.mark.parametrize("L,N,tol,n,P", [(31.0, 9000, 1e-4, 32, 6), (100.0, 300000, 1e-5, 96, 8),
                                         (22.56, 512, 1e-3, 24, 5)])
def test_default_parameters_match_reference_rules(L, N, tol, n, P):
    _lib_or_skip()
    p = esp.esp_plan_query(L, N, tol)
    ref = esp_parameters(L, tol)
    assert (p.nf, p.P) == (n, P) == (ref["n"], ref["P"])
    assert abs(p.c - c_for_tolerance(tol)) < 1e-9
    assert abs(p.rc - ref["rc"]) < 1e-9
    assert p.precision == 32 and p.tile == 0
    # c1: the library's choice is (near-)optimal for the reference's E_A
    ea = aliasing_error(p.nf, L, p.c, p.rc, p.c1, p.P)
    ea_ref = aliasing_error(p.nf, L, p.c, p.rc, ref["c1"], p.P)
    assert ea <= 1.01 * ea_ref
    s0 = PSWFSplit(p.c, p.rc).S0()
    assert abs(p.s0 - s0) < 1e-12 * s0


@pytest.mark.parametrize("tol,P", [(1e-3, 5), (1e-4, 6), (1e-5, 8)])
def test_window_polynomials_fit_pswf(tol, P):
    _lib_or_skip()
    p = esp.esp_plan_query(31.0, 9000, tol)
    coef = esp.esp_window_coeffs(p)
    assert coef.shape == (P, p.degree + 1)
    psi = pswf(p.c1)
    y = np.linspace(-0.5, 0.5, 101)
    err = 0.0
    for j in range(P):
        fit = np.polynomial.polynomial.polyval(y, coef[j])
        exact = psi(2 * (y + 0.5 + P / 2 - 1 - j) / P)
        err = max(err, np.max(np.abs(fit - exact)))
    assert err <= 0.05 * tol * psi(0.0)
    # high-degree fit reproduces the window to rounding
    p16 = esp.esp_plan_query(31.0, 9000, tol, degree=16)
    c16 = esp.esp_window_coeffs(p16)
    for j in range(P):
        fit = np.polynomial.polynomial.polyval(y, c16[j])
        assert np.max(np.abs(fit - psi(2 * (y + 0.5 + P / 2 - 1 - j) / P))) < 1e-10


def test_influence_tables_match_reference():
    _lib_or_skip()
    p = esp.esp_plan_query(17.0, 1500, 1e-4, nf=18)
    TS, Tphi = esp.esp_influence_tables(p)
    pref = influence(p.nf, p.L, p.P, p.c, p.rc, p.c1)
    n = p.nf
    k = np.arange(n)
    m = np.abs(np.where(k < n // 2, k, k - n))
    m2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    plib = TS[m2] * Tphi[m][:, None, None] * Tphi[m][None, :, None] * Tphi[m][None, None, :]
    assert plib[0, 0, 0] == 0.0
    assert np.max(np.abs(plib - pref)) < 1e-10 * np.max(np.abs(pref))
    ph = phi_hat_1d(2 * math.pi * np.arange(n // 2 + 1) / p.L, p.P, p.h, p.c1)
    assert np.max(np.abs(Tphi * ph ** 2 - 1)) < 1e-10


def test_local_kernel_matches_reference():
    _lib_or_skip()
    p = esp.esp_plan_query(31.0, 9000, 1e-4)
    r = np.linspace(0.3, p.rc * 1.2, 50)
    Lr, dLr = esp.esp_local_kernel(p, r)
    Lo, dLo = L_and_dL(PSWFSplit(p.c, p.rc), r)
    assert np.max(np.abs(Lr - Lo)) < 1e-11 * np.max(np.abs(Lo))
    assert np.max(np.abs(dLr - dLo)) < 1e-11 * np.max(np.abs(dLo))
    assert np.all(Lr[r >= p.rc] == 0)


@pytest.mark.parametrize("tol,L", [(1e-3, 31.0), (1e-4, 31.0), (1e-5, 100.0), (1e-4, 22.56)])
def test_local_polynomials_match_reference_kernel(tol, L):
    # the device's piecewise polynomials in grid units against the reference
    # L(r) = (1 - G(r/rc))/(4 pi r) and L'(r) of an independent PSWF evaluation
    _lib_or_skip()
    p = esp.esp_plan_query(L, 9000, tol)
    A, B = esp.esp_local_coeffs(p)
    K, d1 = A.shape
    assert K == 1 and 9 <= d1 <= 17
    h, rho = p.h, p.rc / p.h
    r = np.linspace(1e-3, 1.0 - 1e-9, 4001) * p.rc
    rg = r / h
    x = (rg / rho) ** 2
    k = np.minimum((x * K).astype(int), K - 1)
    y = x * K - k - 0.5
    Av = np.zeros_like(y)
    Bv = np.zeros_like(y)
    for m in range(d1 - 1, -1, -1):
        Av = Av * y + A[k, m]
        Bv = Bv * y + B[k, m]
    L_dev = (1.0 / (4 * math.pi * rg) - Av) / h
    dL_dev = (-1.0 / (4 * math.pi * rg ** 3) - Bv) * rg / h ** 2
    L_ref, dL_ref = L_and_dL(PSWFSplit(p.c, p.rc), r)
    # pointwise, against the larger of the value and the Coulomb magnitude at
    # the cutoff (1/(4 pi rc), 1/(4 pi rc^2))
    assert np.all(np.abs(L_dev - L_ref) < 1e-10 * np.maximum(np.abs(L_ref), 1 / (4 * math.pi * p.rc)))
    assert np.all(np.abs(dL_dev - dL_ref) < 1e-10 * np.maximum(np.abs(dL_ref), 1 / (4 * math.pi * p.rc ** 2)))
    # L vanishes at the cutoff
    assert abs(L_dev[-1]) < 1e-10 / (4 * math.pi * p.rc)


def test_local_part_needs_half_box_cutoff():
    _lib_or_skip()
    with pytest.raises(esp.EspError) as ei:
        esp.esp_plan_query(8.0, 100, 1e-4, local=1)
    assert ei.value.status == -2
    assert esp.esp_plan_query(22.56, 512, 1e-4, local=1).local == 1


def test_orthorhombic_parameters():
    # the longest side sets the grid, the coarsest spacing the cutoff
    _lib_or_skip()
    p = esp.esp_plan_query((18.0, 21.0, 24.0), 1000, 1e-4)
    c = esp.esp_plan_query(24.0, 1000, 1e-4)
    assert (p.L, p.Ly, p.Lz) == (18.0, 21.0, 24.0)
    assert p.nf == c.nf and abs(p.rc - c.rc) < 1e-12 and p.c1 == c.c1 and p.P == c.P
    assert abs(p.h - 18.0 / p.nf) < 1e-15
    with pytest.raises(esp.EspError):
        esp.esp_plan_query((24.0, 24.0, 8.0), 1000, 1e-4, local=1)  # rc > 8/2


def test_triclinic_parameters():
    # the longest lattice vector sets the grid and the cutoff; the local part
    # needs rc at most half the smallest distance between lattice planes
    _lib_or_skip()
    p = esp.esp_plan_query((16.0, 15.0, 14.0), 1000, 1e-4, xy=10.0, xz=-2.0, yz=3.0)
    c = esp.esp_plan_query(math.hypot(10.0, 15.0), 1000, 1e-4)
    assert (p.xy, p.xz, p.yz) == (10.0, -2.0, 3.0)
    assert p.nf == c.nf and abs(p.rc - c.rc) < 1e-12 and p.c1 == c.c1 and p.P == c.P
    assert esp.esp_plan_query((14.0, 14.0, 14.0), 1000, 1e-4, local=1).local == 1
    with pytest.raises(esp.EspError) as ei:  # plane spacing 14/sqrt(1 + (13/14)^2) = 10.3 < 2 rc
        esp.esp_plan_query((14.0, 14.0, 14.0), 1000, 1e-4, xy=13.0, local=1)
    assert ei.value.status == -2 and "plane" in esp.lib().esp_last_error().decode()
    c = esp.esp_plan_query((16.0, 15.0, 14.0), 1000, 1e-4, xy=1.0, method=1)
    assert c.method == 1 and c.nf == esp.esp_plan_query(16.0, 1000, 1e-4, method=1).nf  # longest vector: a
    assert esp.esp_plan_query((16.0, 15.0, 14.0), 1000, 1e-4, xy=1.0, force_method=1).force_method == 1
    with pytest.raises(esp.EspError) as ei:
        esp.esp_plan_query((16.0, 15.0, 14.0), 1000, 1e-4, yz=math.inf)
    assert ei.value.status == -1


def test_table2_through_the_library():
    _lib_or_skip()
    for eps, c_tab, P_tab in [(1e-3, 9.5392, 5), (5e-4, 10.290, 5), (1e-4, 12.024, 6), (5e-5, 12.762, 7),
                              (1e-5, 14.471, 8)]:
        p = esp.esp_plan_query(31.0, 9000, eps)
        assert abs(p.c - c_tab) < 3e-3 and p.P == P_tab


@pytest.mark.parametrize("kw,box,tol,status", [
    ({}, (10.0, 10.0, -1.0), 1e-4, -1),        # negative side
    ({}, 10.0, 0.5, -1),                        # tolerance out of range
    ({"nf": 10}, 10.0, 1e-4, -2),               # 10 is not 2^a 3^b
    ({"nf": 192}, 10.0, 1e-4, -2),              # beyond the built FFT range
    ({"P": 13}, 10.0, 1e-4, -2),
    ({"precision": 16}, 10.0, 1e-4, -1),
])
def test_invalid_arguments_return_status(kw, box, tol, status):
    _lib_or_skip()
    with pytest.raises(esp.EspError) as ei:
        esp.esp_plan_query(box, 100, tol, **kw)
    assert ei.value.status == status
    assert esp.lib().esp_last_error().decode() != ""


def test_warm_tables_covers_every_grid_and_rejects_bad_tolerances():
    """Warm-up resolves every smooth grid of a tolerance (host only); a later
    query of any box with that grid and tolerance then agrees with the oracle's
    rules, and tolerances outside Table 2's orders are refused."""
    _lib_or_skip()
    from paper_2505_09727_amd import EspError, esp_warm_tables
    esp_warm_tables([1e-3], nf_max=48, threads=2)
    prm = esp.esp_plan_query(40.0, 4000, 1e-3)
    ref = esp_parameters(40.0, 1e-3)
    assert (prm.nf, prm.P) == (ref["n"], ref["P"])
    ea = aliasing_error(prm.nf, 40.0, prm.c, prm.rc, prm.c1, prm.P)
    assert ea <= 1.01 * aliasing_error(prm.nf, 40.0, prm.c, prm.rc, ref["c1"], prm.P)
    for bad in ([0.0], [1e-14]):
        with pytest.raises(EspError):
            esp_warm_tables(bad, nf_max=16)


def test_stream_and_determinism_fields():
    """esp_params carries the caller's stream (passed through unchanged by
    the host query) and the determinism flag (1 for FP32 plans, 0 for FP64
    ones; requiring it of an FP64 plan or passing other values is refused)."""
    _lib_or_skip()
    p = esp.esp_plan_query(31.0, 9000, 1e-4)
    assert p.deterministic == 1 and not p.stream
    p = esp.esp_plan_query(31.0, 9000, 1e-4, deterministic=1, stream=0x1234)
    assert p.deterministic == 1 and p.stream == 0x1234
    assert esp.esp_plan_query(31.0, 9000, 1e-4, precision=64).deterministic == 0
    with pytest.raises(esp.EspError) as ei:
        esp.esp_plan_query(31.0, 9000, 1e-4, deterministic=2)
    assert ei.value.status == -1
    with pytest.raises(esp.EspError) as ei:
        esp.esp_plan_query(31.0, 9000, 1e-4, deterministic=1, precision=64)
    assert ei.value.status == -2


def test_plan_entry_points_reject_null_plans():
    """The plan-level calls added for the boundary (stream selection, batched
    evaluation, short-range coefficients) return ESP_E_INVALID on a NULL plan
    without touching a device."""
    L = _lib_or_skip()
    import ctypes as C
    coef = (C.c_double * (2 * esp.ESP_LOCAL_COEF_MAX))()
    K, d = C.c_int(0), C.c_int(0)
    assert L.esp_plan_shortrange_coeffs(None, coef, C.byref(K), C.byref(d)) == -1
    assert L.esp_plan_set_stream(None, None) == -1
    assert L.esp_batch_longrange(None, None, None, None, None, None) == -1
    assert L.esp_last_error().decode() != ""
