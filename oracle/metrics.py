"""Relative RMS force error (eq. Deltadef)."""
from __future__ import annotations

import numpy as np


def rel_rms(F_test, F_ref, F_norm=None) -> float:
    """sqrt(sum |F_test - F_ref|^2 / sum |F_norm|^2), F_norm defaulting to F_ref."""
    F_test = np.asarray(F_test, np.float64)
    F_ref = np.asarray(F_ref, np.float64)
    F_norm = F_ref if F_norm is None else np.asarray(F_norm, np.float64)
    return float(np.sqrt(np.sum((F_test - F_ref) ** 2) / np.sum(F_norm ** 2)))
