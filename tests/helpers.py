"""Shared helpers of the test suite: build matching GPU and oracle tubes from
one parameter dict and compare results normwise per field."""
import numpy as np


def oracle_tube(params):
    from oracle import oracle as O
    return O.Tube(**params)


def gpu_tube(params):
    from paper_1608_03004_amd import Tube
    return Tube(**params)


def normwise(a, b):
    """max|a - b| / max|b| per row (rows are fields or quadrature points)."""
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / scale


def field_errors(gpu_fields, ref_fields):
    """Dict of normwise max and L2 errors per field name."""
    names = ("N0", "Nz", "T00", "T0z", "Tzz", "e", "n", "v", "T", "Nabs")
    out = {}
    for k, name in enumerate(names):
        d = gpu_fields[k] - ref_fields[k]
        s = max(np.abs(ref_fields[k]).max(), 1e-300)
        out[name] = (np.abs(d).max() / s, np.sqrt(np.mean(d * d)) / s)
    return out
