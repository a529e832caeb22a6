"""Host-side helpers for the sampled serving check: the drifted positions a
served request reaches, and a reference evaluation that returns only what the
check compares (forces, potentials, energy and the magnitude of its terms).
Imported by pool workers, so it touches no GPU."""
import numpy as np

import workloads as W


def positions_at_step(pos, L, step, seed, drift):
    """Positions of a served request at step `step` (0: as submitted)."""
    p = np.asarray(pos, np.float32)
    for k in range(1, step + 1):
        p = W.serving_drift(p, L, k, seed, drift)
    return p


def limit_threads():
    from threadpoolctl import threadpool_limits
    threadpool_limits(2)


def reference(pos32, q, L, nf, P, c, rc, c1):
    from oracle.fivestep import five_step
    r = five_step(np.asarray(pos32, np.float64), q, L, nf, P, c, rc, c1)
    return r["F"], r["phi"], r["E"], 0.5 * float(np.sum(np.abs(q * r["phi"])))
