"""Oracle: rounding to the storage precisions of the inner V-cycle (test infrastructure only).

Plain IEEE round-to-nearest-even: float32 by NumPy's cast, bfloat16 (8 exponent bits, 7 stored
mantissa bits) by rounding the float32 bit pattern to its upper 16 bits, ties to even.
"""
import copy

import numpy as np


def bf16(x):
    """Round to bfloat16 (round to nearest even), via float32."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def rounded(x, kind):
    """x rounded to kind in {"f64", "f32", "bf16"} (values returned as float64)."""
    if kind in (None, "f64"):
        return np.asarray(x, dtype=np.float64)
    if kind == "f32":
        return f32(x)
    if kind == "bf16":
        return bf16(x)
    raise ValueError(f"unknown storage precision {kind!r}")


def with_stored_factors(mesh, kind):
    """Shallow copy of a mesh whose geometric factors (not its coordinates, mass or faces) are
    rounded to the storage precision kind: the operator a V-cycle level applies when its factors
    are held in that precision and everything else is exact."""
    if kind in (None, "f64"):
        return mesh
    m = copy.copy(mesh)
    names = ("Grr", "Grs", "Gss") if mesh.dim == 2 else ("Grr", "Gtt", "Grs", "Gts", "Gss")
    for nm in names:
        setattr(m, nm, rounded(getattr(mesh, nm), kind))
    return m
