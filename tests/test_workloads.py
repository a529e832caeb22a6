"""Seeded generators: SplitMix64 drift stream pinned to the generator's
published first outputs; workloads are neutral and reproducible."""
import numpy as np

import workloads as W
from conftest import read_golden


def test_splitmix64_published_outputs():
    ref = [int(r[0], 16) for r in read_golden("splitmix64.txt")]
    got = [int(v) for v in W.splitmix64_sequence(0, len(ref))]
    assert got == ref


def test_serving_drift_is_bounded_uniform_and_wraps():
    rng = np.random.default_rng(0)
    L = 20.0
    pos = (rng.random((5000, 3)) * L).astype(np.float32)
    pos[0] = [0.0, L - 1e-6, 10.0]
    p1 = W.serving_drift(pos, L, step=1, seed=42, drift=0.5)
    d = (p1 - pos + L / 2) % L - L / 2
    assert np.all(np.abs(d) <= 0.5 + 1e-5)
    assert abs(d.mean()) < 0.02 and abs(d.std() - 0.5 / np.sqrt(3)) < 0.01
    assert np.all((p1 >= 0) & (p1 < L))
    assert not np.array_equal(W.serving_drift(pos, L, 2, 42, 0.5), p1)
    assert np.array_equal(W.serving_drift(pos, L, 1, 42, 0.5), p1)


def test_workloads_neutral_and_seeded():
    for pos, q, L in [W.nacl_crystal(), W.water_box_at_density(3000, 1), W.ionic_melt(1000, 2)]:
        assert abs(q.sum()) < 1e-9 and np.all((pos >= 0) & (pos < L))
    a = W.water_box(100, 10.0, 7)
    b = W.water_box(100, 10.0, 7)
    assert np.array_equal(a[0], b[0])
    # rigid geometry: O-H 1.0, H-O-H 109.47 degrees (up to wrapping)
    p, _ = W.water_box(50, 100.0, 3)
    m = p.reshape(-1, 3, 3)
    d1 = (m[:, 1] - m[:, 0] + 50) % 100 - 50
    d2 = (m[:, 2] - m[:, 0] + 50) % 100 - 50
    assert np.allclose(np.linalg.norm(d1, axis=1), 1.0)
    cosang = np.sum(d1 * d2, 1) / (np.linalg.norm(d1, axis=1) * np.linalg.norm(d2, axis=1))
    assert np.allclose(np.degrees(np.arccos(cosang)), 109.47)
    sizes = W.ensemble_sizes()
    assert len(sizes) == 256 and sizes.min() >= 498 and sizes.max() <= 20001 and np.all(sizes % 3 == 0)
    reqs = W.request_stream(duration_s=1.0)
    gaps = np.diff([r.t_arrival for r in reqs])
    assert 1500 < len(reqs) < 2500 and abs(gaps.mean() - 1 / 2000) < 1e-4
