"""Element-wise parity bar shared by the device tests.

Next to the relative RMS error of eq. Deltadef, every comparison of device
results with the CPU reference also bounds the worst particle:

    max_i |x_i - x_i^ref| / rms_j |x_j^ref|  <=  K tol,   K = 10,

with |.| the Euclidean norm of a force vector. An RMS bar alone would let
one particle in N carry an error sqrt(N) times the bar; this one holds every
particle to ten times the tolerance, in units of the typical magnitude."""
import numpy as np

K_ELEMENTWISE = 10.0


def worst(got, ref):
    """max_i |got_i - ref_i| / rms |ref| (rows are vectors when 2-D)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if got.ndim == 2:
        d = np.sqrt(np.sum((got - ref) ** 2, axis=1))
        s = np.sqrt(np.mean(np.sum(ref ** 2, axis=1)))
    else:
        d = np.abs(got - ref)
        s = np.sqrt(np.mean(ref ** 2))
    return float(d.max() / s)


def elementwise(got, ref, tol, what="", k=K_ELEMENTWISE):
    """Assert the worst particle is within k * tol; returns the measured ratio."""
    w = worst(got, ref)
    print(f"  worst particle {what}: {w:.2e} (bar {k * tol:.1e})", flush=True)
    assert w <= k * tol, f"{what}: worst particle {w:.3e} > {k} x {tol:.1e}"
    return w
