"""Comparison helpers of the GPU parity tests.

rel(a, b) is the larger of two relative differences of a result a from its reference b:
the L2 one, ||a - b||_2 / ||b||_2, and the element-wise one, max|a - b| / max|b|.  A bound on
it therefore also bounds every single cell: an error confined to a few cells (one boundary
face of a 512^3 grid holds 1/512 of them) is not diluted by the norm.  Arguments may be arrays
or sequences of arrays (the patches of a refined mesh), compared pairwise."""
import math

import numpy as np


def _pairs(a, b):
    if isinstance(a, np.ndarray) or np.isscalar(a):
        return [(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))]
    return [(np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)) for x, y in zip(a, b)]


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2 (over all pairs)."""
    pairs = _pairs(a, b)
    num = math.sqrt(sum(float(np.sum((x - y) ** 2)) for x, y in pairs))
    den = math.sqrt(sum(float(np.sum(y ** 2)) for _, y in pairs))
    return num / den


def rel_max(a, b):
    """max|a - b| / max|b| (over all pairs)."""
    pairs = _pairs(a, b)
    num = max(float(np.max(np.abs(x - y))) if x.size else 0.0 for x, y in pairs)
    den = max(float(np.max(np.abs(y))) if y.size else 0.0 for _, y in pairs)
    return num / den


def rel(a, b):
    """The larger of rel_l2 and rel_max."""
    return max(rel_l2(a, b), rel_max(a, b))
