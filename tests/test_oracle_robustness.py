"""The reference's sums do not depend on memory they never write.

On the GPU host the 300,000-atom reference once came back with every force
NaN while the device output was finite. Its matrix DFT then ran through
BLAS complex GEMM (numpy allocates the product with np.empty). These tests
pin the two properties that rule out uninitialised memory in the reference:
its sums call no BLAS routine, and its results are bit-identical whether the
heap it allocates from was left full of NaN or not."""
import ast
import glob
import math
import os

import numpy as np

import workloads as W
from oracle.ewald import ewald
from oracle.fivestep import dft3, five_step
from oracle.params import esp_parameters
from oracle.spectral import evaluate_modes, structure_factor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_reference_sums_call_no_blas():
    # no matrix products (@, dot, tensordot, matmul, inner, vdot) and no
    # optimised einsum, which would route through tensordot
    banned = {"dot", "tensordot", "matmul", "inner", "vdot"}
    found = []
    for path in sorted(glob.glob(os.path.join(ROOT, "oracle", "*.py"))):
        tree = ast.parse(open(path).read(), path)
        for node in ast.walk(tree):
            if isinstance(node, ast.BinOp) and isinstance(node.op, ast.MatMult):
                found.append(f"{os.path.basename(path)}:{node.lineno} @")
            if isinstance(node, ast.Call) and isinstance(node.func, ast.Attribute):
                if node.func.attr in banned:
                    found.append(f"{os.path.basename(path)}:{node.lineno} {node.func.attr}")
                if node.func.attr == "einsum":
                    # numpy's default is optimize=False (its own loops)
                    opt = [k for k in node.keywords if k.arg == "optimize"]
                    if opt and not (isinstance(opt[0].value, ast.Constant) and opt[0].value.value is False):
                        found.append(f"{os.path.basename(path)}:{node.lineno} optimised einsum")
    assert not found, found


def _prime_heap_with_nan(nbytes):
    # fill, free and refill blocks of the sizes the reference allocates, so
    # that np.empty of those sizes hands back NaN-filled memory
    for _ in range(2):
        junk = [np.full(nbytes // 8, np.nan) for _ in range(4)]
        del junk
    probe = np.empty(nbytes // 8)
    primed = int(np.isnan(probe).sum())
    del probe
    return primed


def test_results_do_not_depend_on_heap_contents():
    pos, q = W.water_box(300, 14.4, seed=11)
    L = 14.4
    prm = esp_parameters(L, 1e-4, n=24)
    args = (prm["n"], prm["P"], prm["c"], prm["rc"], prm["c1"])
    m = np.arange(-8, 9)
    clean = five_step(pos, q, L, *args)
    rho = structure_factor(pos, q, L, m)
    u_m, g_m = evaluate_modes(pos, L, m, rho)
    u_e, F_e, E_e = ewald(pos, q, L)
    b = np.random.default_rng(1).standard_normal((48, 48, 48))
    d_clean = dft3(b, +1)
    for size in (48 ** 3 * 16, 24 ** 3 * 16, len(m) ** 3 * 16):
        assert _prime_heap_with_nan(size) > 0
        d = dft3(b, +1)
        assert np.array_equal(d, d_clean)
    assert _prime_heap_with_nan(24 ** 3 * 16) > 0
    again = five_step(pos, q, L, *args)
    for k in ("b", "bhat", "c", "phi", "F"):
        assert np.array_equal(again[k], clean[k]), k
    assert again["E"] == clean["E"]
    assert _prime_heap_with_nan(len(m) ** 3 * 16) > 0
    assert np.array_equal(structure_factor(pos, q, L, m), rho)
    u2, g2 = evaluate_modes(pos, L, m, rho)
    assert np.array_equal(u2, u_m) and np.array_equal(g2, g_m)
    u3, F3, E3 = ewald(pos, q, L)
    assert np.array_equal(u3, u_e) and np.array_equal(F3, F_e) and E3 == E_e


def test_structure_factor_is_the_definition():
    # rho(m) = sum_j q_j exp(2 pi i m.r_j/L), term by term on a tiny input
    rng = np.random.default_rng(5)
    pos = rng.uniform(0, 3.0, (5, 3))
    q = rng.standard_normal(5)
    m = np.arange(-2, 3)
    rho = structure_factor(pos, q, 3.0, m, chunk=2)
    for a, mx in enumerate(m):
        for b_, my in enumerate(m):
            for c, mz in enumerate(m):
                ref = sum(q[j] * complex(math.cos(2 * math.pi * (mx * pos[j, 0] + my * pos[j, 1] + mz * pos[j, 2]) / 3.0),
                                         math.sin(2 * math.pi * (mx * pos[j, 0] + my * pos[j, 1] + mz * pos[j, 2]) / 3.0))
                          for j in range(5))
                assert abs(rho[a, b_, c] - ref) < 1e-12
