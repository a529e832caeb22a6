"""Pins of the oracle's five-step pipeline: exact special cases (library FFT),
the Parseval identity, invariances, convergence to the truncated spectral sum,
and the paper's error claim eps = Delta against classical Ewald."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.ewald import ewald
from oracle.fivestep import five_step, dft3, influence, spread
from oracle.metrics import rel_rms
from oracle.params import esp_parameters, aliasing_error, choose_c1
from oracle.split import PSWFSplit
from oracle.spectral import spectral_sum, local_sum


def _small_water(seed=11, n_mol=300, L=14.4):
    pos, q = W.water_box(n_mol, L, seed)
    return pos, q, L


def test_dft_is_library_fft():
    rng = np.random.default_rng(0)
    for n in (6, 16, 18):
        b = rng.standard_normal((n, n, n))
        # sum_l e^{+2 pi i k.l/n} b_l = n^3 ifftn(b)
        assert np.max(np.abs(dft3(b, +1) - n ** 3 * np.fft.ifftn(b))) < 1e-10
        assert np.max(np.abs(dft3(b, -1) - np.fft.fftn(b))) < 1e-10


def test_parseval_energy_identity():
    pos, q, L = _small_water()
    prm = esp_parameters(L, 1e-4, n=16)
    r = five_step(pos, q, L, prm["n"], prm["P"], prm["c"], prm["rc"], prm["c1"])
    # sum_i q_i u~_i = sum_k p_k |b^_k|^2  (spread and interpolation are adjoint)
    assert abs(r["E"] - (r["Ek"] - 0.5 * r["s0"] * np.sum(q * q))) < 1e-12 * abs(r["E"])
    assert np.max(np.abs(np.imag(np.fft.fftn(r["c"])[0, 0, 0]))) < 1e-9


def test_influence_is_even_and_drops_zero_mode():
    p = influence(18, 12.0, 6, 12.024, 3.5, 13.5)
    assert p[0, 0, 0] == 0.0
    assert np.max(np.abs(p - p[::-1, ::-1, ::-1][np.ix_(*(np.roll(np.arange(18), 1),) * 3)])) < 1e-13 * p.max()


def test_invariances():
    pos, q, L = _small_water(seed=12)
    prm = esp_parameters(L, 1e-4, n=16)
    a = (prm["n"], prm["P"], prm["c"], prm["rc"], prm["c1"])
    r = five_step(pos, q, L, *a)
    h = L / prm["n"]
    # shift by an integer number of grid spacings: identical up to rounding
    r2 = five_step(np.mod(pos + h * np.array([3, -5, 7]), L), q, L, *a)
    assert np.max(np.abs(r2["F"] - r["F"])) < 1e-11 * np.max(np.abs(r["F"]))
    # q -> -q: forces and energy unchanged, potentials negate
    r3 = five_step(pos, -q, L, *a)
    assert np.max(np.abs(r3["F"] - r["F"])) < 1e-12 * np.max(np.abs(r["F"]))
    assert np.max(np.abs(r3["phi"] + r["phi"])) < 1e-12 * np.max(np.abs(r["phi"]))
    # linearity of the potential in q
    qa = q * np.linspace(0.5, 1.5, len(q))
    qa -= qa.mean()
    ra = five_step(pos, qa, L, *a)
    rb = five_step(pos, q - qa, L, *a)
    assert np.max(np.abs(ra["phi"] + rb["phi"] - r["phi"])) < 1e-11 * np.max(np.abs(r["phi"]))
    # arbitrary shift: equal within the method's error
    r4 = five_step(np.mod(pos + np.array([0.31, 0.77, -0.4]), L), q, L, *a)
    assert rel_rms(r4["F"], r["F"]) < 2e-3


def test_spread_total_charge_weight():
    # sum_l b_l = sum_j q_j (sum_l phi~(r_j - h l)); for a single unit charge the
    # grid sum equals the separable sum of the 1D window samples
    from oracle.pswf import pswf
    L, n, P, c1 = 10.0, 12, 6, 13.0
    b = spread(np.array([[1.234, 5.5, 9.99]]), np.array([1.0]), L, n, P, c1)
    psi = pswf(c1)
    tot = 1.0
    for x in (1.234, 5.5, 9.99):
        u = x * n / L
        l = np.floor(u - P / 2) + 1 + np.arange(P)
        tot *= np.sum(psi(2 * (u - l) / P))
    assert abs(b.sum() - tot) < 1e-13 * abs(tot)
    assert np.count_nonzero(b) == P ** 3


def test_converges_to_truncated_spectral_sum():
    # with a wide window the aliasing error vanishes and the five-step result
    # approaches the direct truncated spectral sum (eq. spectralpart on I).
    # A tight splitting kernel (eps = 1e-9) keeps the Nyquist plane and the
    # slowly decaying transform tail of the compact kernel below the floor.
    from oracle.pswf import c_for_tolerance
    pos, q, L = _small_water(seed=13, n_mol=100, L=10.0)
    n, c, rc = 16, c_for_tolerance(1e-9), 6.0
    sp = PSWFSplit(c, rc)
    us, gs = spectral_sum(pos, q, L, sp, n)
    Fs = -q[:, None] * gs
    errs = []
    for P in (6, 10, 14):
        c1 = choose_c1(n, L, c, rc, P, lo=0.3, hi=2.0, num=35)
        r = five_step(pos, q, L, n, P, c, rc, c1)
        errs.append(rel_rms(r["F"], Fs))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[2] < 1e-8


def test_aliasing_estimate_prefers_c1_near_c():
    n, L, c, rc, P = 32, 31.0, 12.024, 4.45, 6
    c1 = choose_c1(n, L, c, rc, P)
    assert 1.0 * c <= c1 <= 1.3 * c
    assert aliasing_error(n, L, c, rc, c1, P) < aliasing_error(n, L, c, rc, 0.9 * c, P)


def _delta_vs_ewald(pos, q, L, tol, **kw):
    u, F, E = ewald(pos, q, L)
    prm = esp_parameters(L, tol, **kw)
    sp = PSWFSplit(prm["c"], prm["rc"])
    ul, gl = local_sum(pos, q, L, sp)
    Fs_exact = F + q[:, None] * gl          # F^Ewald - F^local
    r = five_step(pos, q, L, prm["n"], prm["P"], prm["c"], prm["rc"], prm["c1"])
    return rel_rms(r["F"], Fs_exact, F), r, prm, (u, F, E), ul


@pytest.mark.parametrize("tol", [1e-3, 1e-4, 1e-5])
def test_error_meets_tolerance_water(tol):
    # eps = Delta (Methods: parameter selection; eq. Deltadef)
    pos, q, L = _small_water(seed=21, n_mol=500, L=17.0)
    delta, *_ = _delta_vs_ewald(pos, q, L, tol)
    assert delta <= tol


def test_nacl_energy_and_madelung():
    pos, q, L = W.nacl_crystal()
    delta, r, prm, (u, F, E), ul = _delta_vs_ewald(pos, q, L, 1e-4, n=16, P=6)
    E_esp = r["E"] + 0.5 * float(np.dot(q, ul))
    assert abs(E_esp - E) < 1e-4 * abs(E)
    phi_tot = r["phi"] + ul
    assert np.max(np.abs(phi_tot - u)) < 1e-4 * np.max(np.abs(u))


# ---------------------------------------------------------------- ik forces

def test_ik_factors_differentiate_a_single_mode():
    # c^ with one pair of modes +-m0 along y: c(x) = 2 cos(2 pi m0 y/L) on the
    # grid (inverse transform c_l = sum exp(-2 pi i k.l/n) c^_k); its derivative
    # is -(4 pi m0/L) sin(2 pi m0 y/L)
    from oracle.fivestep import ik_factors
    n, L, m0 = 12, 7.5, 3
    chat = np.zeros((n, n, n), complex)
    chat[0, m0, 0] = 1.0
    chat[0, n - m0, 0] = 1.0
    y = np.arange(n) * L / n
    c = np.real(dft3(chat, -1))
    assert np.allclose(c[0, :, 0], 2 * np.cos(2 * np.pi * m0 * y / L), atol=1e-12)
    dy = np.real(dft3(chat * ik_factors(n, L).reshape(1, n, 1), -1))
    assert np.allclose(dy[0, :, 0], -(4 * np.pi * m0 / L) * np.sin(2 * np.pi * m0 * y / L), atol=1e-12)
    # the mode is constant along x and z, and so is its y-derivative
    assert np.allclose(dy, np.broadcast_to(dy[:1, :, :1], dy.shape), atol=1e-12)
    for ax in (0, 2):
        shape = [1, 1, 1]
        shape[ax] = n
        assert np.allclose(np.real(dft3(chat * ik_factors(n, L).reshape(shape), -1)), 0.0, atol=1e-12)


def test_ik_forces_conserve_momentum_and_match_ad():
    # the ik route with one window for spreading and interpolation makes the
    # net force vanish exactly (odd derivative factors against the even,
    # real p |b^|^2); both routes approximate the same spectral force
    from oracle.fivestep import five_step_ik
    pos, q = W.water_box(200, 12.0, seed=21)
    L, n, P, tol = 12.0, 16, 6, 1e-4
    prm = esp_parameters(L, tol)
    ik = five_step_ik(pos, q, L, n, P, prm["c"], prm["rc"], prm["c1"])
    ad = five_step(pos, q, L, n, P, prm["c"], prm["rc"], prm["c1"])
    fscale = np.sqrt(np.mean(ik["F"] ** 2))
    assert np.max(np.abs(ik["F"].sum(axis=0))) < 1e-12 * fscale * len(q)
    assert np.max(np.abs(ad["F"].sum(axis=0))) > 1e3 * np.max(np.abs(ik["F"].sum(axis=0)))
    assert rel_rms(ik["F"], ad["F"]) < 1e-3
    assert np.allclose(ik["phi"], ad["phi"]) and ik["E"] == ad["E"]


def test_ik_error_meets_tolerance_against_ewald():
    from oracle.fivestep import five_step_ik
    pos, q = W.water_box(200, 12.0, seed=22)
    L, tol = 12.0, 1e-4
    prm = esp_parameters(L, tol)
    ik = five_step_ik(pos, q, L, prm["n"], prm["P"], prm["c"], prm["rc"], prm["c1"])
    _, F_ewald, _ = ewald(pos, q, L)
    ul, gl = local_sum(pos, q, L, PSWFSplit(prm["c"], prm["rc"]))
    Fs_exact = F_ewald + q[:, None] * gl
    assert rel_rms(ik["F"], Fs_exact, F_ewald) < tol
