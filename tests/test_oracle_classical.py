"""Pins of the classical-method reference (oracle.classical): B-spline closed
forms and identities, the window transform, and the whole method against
classical Ewald at fine resolution and at the default parameters."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.classical import bspline, dbspline, five_step_classical, parameters, phi_hat_1d
from oracle.ewald import ewald
from oracle.metrics import rel_rms
from oracle.split import GaussianSplit
from oracle.spectral import local_sum


def test_bspline_textbook_values():
    # cubic (P = 4): 2/3 at the centre, 1/6 one grid point away; quadratic
    # (P = 3): 3/4, 1/2 at +-1/2, 1/8 at +-1; linear (P = 2): the hat
    assert np.allclose(bspline([0.0, 1.0, -1.0, 2.0, 2.5], 4), [2 / 3, 1 / 6, 1 / 6, 0.0, 0.0], atol=1e-15)
    assert np.allclose(bspline([0.0, 0.5, -0.5, 1.0, 1.5], 3), [3 / 4, 1 / 2, 1 / 2, 1 / 8, 0.0], atol=1e-15)
    assert np.allclose(bspline([0.0, 0.25, -0.75, 1.0], 2), [1.0, 0.75, 0.25, 0.0], atol=1e-15)


@pytest.mark.parametrize("P", [3, 4, 5, 6, 7, 8])
def test_bspline_partition_of_unity_integral_and_derivative(P):
    rng = np.random.default_rng(P)
    x = rng.uniform(-0.5, 0.5, 200)
    shifts = np.arange(-P, P + 1)
    assert np.allclose(bspline(x[:, None] - shifts[None, :], P).sum(1), 1.0, atol=1e-13)
    t = np.linspace(-P / 2, P / 2, 20001)
    assert abs(np.trapezoid(bspline(t, P), t) - 1.0) < 1e-7
    eps = 1e-6
    xs = rng.uniform(-P / 2 + 0.01, P / 2 - 0.01, 100)
    fd = (bspline(xs + eps, P) - bspline(xs - eps, P)) / (2 * eps)
    assert np.max(np.abs(fd - dbspline(xs, P))) < 1e-6


@pytest.mark.parametrize("P", [4, 5, 8])
def test_window_transform_is_sinc_power(P):
    # int B_P(x/h) cos(xi x) dx = h (sin(xi h/2)/(xi h/2))^P
    h = 0.9
    x = np.linspace(-P * h / 2, P * h / 2, 40001)
    w = bspline(x / h, P)
    for xi in (0.0, 0.7, 2.1, 3.3):
        num = np.trapezoid(w * np.cos(xi * x), x)
        assert abs(num - phi_hat_1d(xi, P, h)) < 1e-8 * h


def _full(pos, q, L, n, P, alpha, rc):
    r = five_step_classical(pos, q, L, n, P, alpha, rc)
    ul, gl = local_sum(pos, q, L, GaussianSplit(alpha, rc, support=rc))
    return r["phi"] + ul, r["F"] - q[:, None] * gl


def test_fine_classical_method_is_ewald():
    # alpha = log(1e8) truncates the local part at the 1e-8 level; n = 48
    # with P = 8 leaves the aliasing below that
    pos, q, L = W.nacl_crystal(perturb=0.1, seed=1)
    alpha, rc = math.log(1e8), 10.0
    phi, F = _full(pos, q, L, 48, 8, alpha, rc)
    u_e, F_e, E_e = ewald(pos, q, L)
    assert rel_rms(F, F_e) < 1e-5
    assert abs(0.5 * np.dot(q, phi) - E_e) < 1e-7 * abs(E_e)


def test_default_parameters_reach_their_tolerance_with_a_wide_window():
    # eq. cemparameters at eps = 1e-4 with the ESP cutoff: the truncation
    # error is then ~eps once aliasing is small (P = 8)
    pos, q = W.water_box(300, 15.0, seed=5)
    L, tol, rc = 15.0, 1e-4, 4.4
    alpha, n = parameters(L, tol, rc)
    assert n == 2 * math.ceil(alpha * L / (math.pi * rc))
    n = 24 if n <= 24 else n
    phi, F = _full(pos, q, L, n, 8, alpha, rc)
    _, F_e, _ = ewald(pos, q, L)
    assert rel_rms(F, F_e) < 3 * tol
