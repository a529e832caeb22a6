"""Seeded synthetic inputs: charges and positions only.

This module is shared by the tests, the benchmark and the CPU reference; it
holds none of the electrostatics arithmetic. Every generator is a pure
function of its seed (numpy PCG64), returns float64 arrays, and wraps
positions into the periodic box [0, L)^3.

Workloads (all cubic, periodic, charge neutral):
  * rock-salt NaCl crystal (ions of charge +-1, conventional cell a);
  * water-like boxes of rigid three-site molecules (O -0.8476, H +0.4238,
    O-H 1.0, H-O-H 109.47 degrees), uniform centres, uniform random
    orientations;
  * an ensemble of water boxes at liquid density with log-uniform sizes;
  * a Poisson request stream for the serving workload;
  * ionic melts (equal numbers of +1 and -1 charges at uniform positions).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

Q_O = -0.8476
Q_H = +0.4238
R_OH = 1.0
THETA_HOH_DEG = 109.47
WATER_MOLECULES_PER_A3 = 0.033427   # 1 g/cm^3
IONIC_MELT_IONS_PER_A3 = 0.0446     # rock-salt number density


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def wrap(pos: np.ndarray, L: float) -> np.ndarray:
    """Map positions into [0, L)."""
    out = np.mod(pos, L)
    out[out >= L] = 0.0
    return out


def nacl_crystal(cells: int = 4, a: float = 5.64, perturb: float = 0.0, seed: int = 1):
    """Rock-salt crystal of cells^3 conventional cells (8 ions per cell).

    Na+ on the fcc sites (0,0,0)+fcc, Cl- on (1/2,0,0)+fcc. With perturb > 0
    each coordinate is displaced by U(-perturb, perturb).
    Returns (pos[N,3], q[N], L).
    """
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    na = fcc
    cl = fcc + np.array([.5, 0, 0])
    basis = np.concatenate([na, cl])
    qb = np.concatenate([np.ones(4), -np.ones(4)])
    g = np.arange(cells)
    shifts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = (shifts[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    q = np.tile(qb, len(shifts))
    L = cells * a
    if perturb > 0:
        pos = pos + _rng(seed).uniform(-perturb, perturb, size=pos.shape)
    return wrap(pos, L), q, L


def _random_rotations(rng: np.random.Generator, m: int) -> np.ndarray:
    """Uniform random rotation matrices from uniform unit quaternions
    (Shoemake, Graphics Gems III, 1992)."""
    u1, u2, u3 = rng.random((3, m))
    a = np.sqrt(1 - u1)
    b = np.sqrt(u1)
    w = a * np.sin(2 * np.pi * u2)
    x = a * np.cos(2 * np.pi * u2)
    y = b * np.sin(2 * np.pi * u3)
    z = b * np.cos(2 * np.pi * u3)
    R = np.empty((m, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def water_box(n_mol: int, L, seed: int):
    """n_mol rigid three-site waters with uniform O positions in [0,L)^3 and
    uniform random orientations. Atom order per molecule: O, H, H. L may also
    be the three sides of an orthorhombic box.
    Returns (pos[3*n_mol,3], q[3*n_mol])."""
    rng = _rng(seed)
    o = rng.random((n_mol, 3)) * L
    half = math.radians(THETA_HOH_DEG) / 2
    body = np.array([[0.0, 0.0, 0.0],
                     [math.sin(half), math.cos(half), 0.0],
                     [-math.sin(half), math.cos(half), 0.0]]) * R_OH
    R = _random_rotations(rng, n_mol)
    pos = o[:, None, :] + np.einsum("mij,aj->mai", R, body)
    q = np.tile(np.array([Q_O, Q_H, Q_H]), n_mol)
    return wrap(pos.reshape(-1, 3), L), q


def water_cell(n_mol: int, H, seed: int):
    """n_mol rigid three-site waters in the triclinic cell whose lattice vectors
    are the columns of H: O positions H s with s uniform in [0,1)^3, uniform
    random orientations, atoms left unwrapped (a hydrogen may sit just
    outside the cell). Atom order per molecule: O, H, H.
    Returns (pos[3*n_mol,3], q[3*n_mol])."""
    rng = _rng(seed)
    o = rng.random((n_mol, 3)) @ np.asarray(H, np.float64).T
    half = math.radians(THETA_HOH_DEG) / 2
    body = np.array([[0.0, 0.0, 0.0],
                     [math.sin(half), math.cos(half), 0.0],
                     [-math.sin(half), math.cos(half), 0.0]]) * R_OH
    R = _random_rotations(rng, n_mol)
    pos = o[:, None, :] + np.einsum("mij,aj->mai", R, body)
    return pos.reshape(-1, 3), np.tile(np.array([Q_O, Q_H, Q_H]), n_mol)


def rhombic_dodecahedron(volume: float):
    """Cell matrix (lattice vectors as columns) of the rhombic dodecahedron with
    a square xy face, a = (d, 0, 0), b = (0, d, 0), c = (d/2, d/2, d/sqrt 2),
    of the given volume (d^3 / sqrt 2)."""
    d = (volume * math.sqrt(2.0)) ** (1.0 / 3.0)
    return np.array([[d, 0.0, d / 2], [0.0, d, d / 2], [0.0, 0.0, d / math.sqrt(2.0)]])


def water_box_at_density(n_atoms: int, seed: int, density=WATER_MOLECULES_PER_A3):
    """Water box of n_atoms (a multiple of 3) at the given molecule density."""
    n_mol = n_atoms // 3
    L = (n_mol / density) ** (1.0 / 3.0)
    pos, q = water_box(n_mol, L, seed)
    return pos, q, L


def ionic_melt(n_ions: int, seed: int, density=IONIC_MELT_IONS_PER_A3):
    """Equal numbers of +1/-1 charges at uniform random positions."""
    n_ions -= n_ions % 2
    L = (n_ions / density) ** (1.0 / 3.0)
    rng = _rng(seed)
    pos = rng.random((n_ions, 3)) * L
    q = np.where(np.arange(n_ions) % 2 == 0, 1.0, -1.0)
    return wrap(pos, L), q, L


def drift(pos: np.ndarray, L: float, step: int, seed: int, amplitude: float = 0.01):
    """Seeded per-step random drift: each coordinate += U(-a, a)."""
    rng = _rng((seed << 20) ^ (step + 1))
    return wrap(pos + rng.uniform(-amplitude, amplitude, size=pos.shape), L)


def ensemble_sizes(n_sys: int = 256, lo: int = 500, hi: int = 20000, seed: int = 4):
    """Atom counts log-uniform in [lo, hi], rounded to whole molecules."""
    rng = _rng(seed)
    x = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_sys))
    return (3 * np.maximum(1, np.round(x / 3))).astype(np.int64)


def ensemble(n_sys: int = 256, lo: int = 500, hi: int = 20000, seed: int = 4):
    """List of (pos, q, L) water boxes at 1 g/cm^3 with log-uniform sizes."""
    sizes = ensemble_sizes(n_sys, lo, hi, seed)
    return [water_box_at_density(int(n), seed * 100003 + i) for i, n in enumerate(sizes)]


@dataclass
class Request:
    rid: int
    t_arrival: float
    kind: str          # "water" or "melt"
    n_atoms: int
    tol: float
    seed: int
    steps: int = 10

    def system(self):
        if self.kind == "water":
            return water_box_at_density(self.n_atoms - self.n_atoms % 3, self.seed)
        return ionic_melt(self.n_atoms, self.seed)


def request_stream(duration_s: float = 10.0, rate_hz: float = 2000.0, lo: int = 1000,
                   hi: int = 200000, tols=(1e-3, 1e-4, 1e-5), seed: int = 5,
                   max_requests: int | None = None):
    """Poisson arrivals (exponential gaps) with log-uniform sizes, random
    kind (water or ionic melt, p = 1/2) and a tolerance drawn uniformly."""
    rng = _rng(seed)
    out, t, i = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s or (max_requests is not None and i >= max_requests):
            break
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        kind = "water" if rng.random() < 0.5 else "melt"
        tol = float(tols[rng.integers(len(tols))])
        out.append(Request(i, t, kind, n, tol, int(seed * 1000003 + i)))
        i += 1
    return out


# Named workload configurations (sizes as stated for the paper's water-like and
# ionic test boxes).
NACL = dict(cells=4, a=5.64, n=16, P=6, tol=1e-4)
WATER_9K = dict(n_mol=3000, L=31.0, n=32, tol=1e-4, seed=2)
WATER_300K = dict(n_mol=100000, L=100.0, n=96, tol=1e-5, seed=3, steps=100)


# ---------------------------------------------------------------------------
# Serving drift stream: counter-based SplitMix64 (Steele, Lea & Flood,
# "Fast splittable pseudorandom number generators", OOPSLA 2014; constants of
# Vigna's reference splitmix64.c). The variate of (step k, particle i,
# component c) is mix(seed + (k * 2^40 + 3 i + c + 1) * GAMMA) / 2^64, and a
# coordinate moves by drift * (2u - 1) in FP32 with wrapping into [0, L).

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_sequence(seed: int, count: int):
    """The classic sequential generator: state += GAMMA, output mix(state)."""
    k = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return splitmix64_mix(np.uint64(seed) + k * _GAMMA)


def serving_drift(pos32: np.ndarray, L: float, step: int, seed: int, drift: float) -> np.ndarray:
    """Positions (float32, N x 3) after the drift of `step` (>= 1)."""
    N = pos32.shape[0]
    ctr = (np.uint64(step) << np.uint64(40)) + np.arange(3 * N, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        z = splitmix64_mix(np.uint64(seed) + ctr * _GAMMA)
    u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    d = (drift * (2.0 * u - 1.0)).astype(np.float32).reshape(N, 3)
    x = (pos32.astype(np.float32) + d).astype(np.float32)
    Lf = np.float32(L)
    x = np.where(x >= Lf, (x - Lf).astype(np.float32), x)
    x = np.where(x < np.float32(0), (x + Lf).astype(np.float32), x)
    return x.astype(np.float32)
