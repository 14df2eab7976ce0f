"""Test helpers (no method arithmetic)."""
import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def zero_sources(prob):
    for s in prob.sources:
        s.incr = np.zeros_like(s.incr)
    return prob
