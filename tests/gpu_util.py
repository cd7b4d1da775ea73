"""Helpers shared by the GPU tests (no solver arithmetic here)."""
import numpy as np


def zyx_nodes_from_xyz(a):
    """(3, N1, N2, N3) oracle layout -> (3, N3, N2, N1) library layout."""
    return np.ascontiguousarray(a.transpose(0, 3, 2, 1))


def xyz_nodes_from_zyx(a):
    return np.ascontiguousarray(a.transpose(0, 3, 2, 1))


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / den)
