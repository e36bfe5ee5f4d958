"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and rejects bad
descriptors before touching the GPU.  No GPU compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import gll

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2411_14977_amd", "libsem.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")


def declared_symbols():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_symbols()
    assert "sem_poisson_solve" in names and "sem_mesh_setup" in names
    for n in names:
        assert hasattr(lib, n), n


def test_bad_descriptors_are_rejected_before_gpu_use():
    from paper_2411_14977_amd import binding as B
    cases = []
    d = B.sem_mesh_desc_default()
    d.order = 0
    cases.append(d)
    d = B.sem_mesh_desc_default()
    d.order = 13
    cases.append(d)
    d = B.sem_mesh_desc_default()   # no h / eta
    cases.append(d)
    h = np.ones(9)
    for mutate in (lambda d: setattr(d, "inner_prec", 7), lambda d: setattr(d, "outer", 3),
                   lambda d: setattr(d, "smoother", 9), lambda d: setattr(d, "cheb_lo", -1.0),
                   lambda d: setattr(d, "schwarz_overlap", 9),
                   lambda d: setattr(d, "schwarz_overlap", -1)):
        d = B.sem_mesh_desc_default()
        d.order, d.ne[0], d.ne[2] = 4, 2, 2
        d.h = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.eta = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        mutate(d)
        cases.append(d)
    for d in cases:
        with pytest.raises(B.SemError) as e:
            B.sem_mesh_setup(d)
        assert e.value.status == 1


@pytest.mark.parametrize("P", [1, 2, 5, 8, 12])
def test_library_gll_rule_matches_oracle(P):
    from paper_2411_14977_amd import binding as B
    r, w = B.sem_gll(P)
    assert np.abs(r - gll.gll_nodes(P)).max() < 1e-15
    assert np.abs(w - gll.gll_weights(P)).max() < 1e-14


def test_bad_semi_coarsened_descriptors_are_rejected_before_gpu_use():
    """Orders along x and sigma that the hierarchy cannot take: out of range, 3D with two
    orders, level lists where an order grows, nothing drops, both drop between levels of
    different orders, a first or last level that does not match, the Schwarz smoother on
    such levels, and columns too tall for one workgroup."""
    from paper_2411_14977_amd import binding as B
    h = np.ones(4096)
    dp = ctypes.POINTER(ctypes.c_double)

    def desc(order, order_z, levels=None, dim=2, ne=(4, 1, 2), smoother=None):
        d = B.sem_mesh_desc_default()
        d.dim, d.order, d.order_z = dim, order, order_z
        for k in range(3):
            d.ne[k] = ne[k]
        d.h = h.ctypes.data_as(dp)
        d.eta = h.ctypes.data_as(dp)
        if smoother is not None:
            d.smoother = smoother
        if levels:
            d.nlevels = len(levels)
            for k, (px, pz) in enumerate(levels):
                d.level_order[k], d.level_order_z[k] = px, pz
        return d

    bad = [
        desc(4, 13),
        desc(4, -1),
        desc(4, 2, dim=3, ne=(2, 2, 2)),
        desc(6, 3, [(6, 3), (6, 4), (3, 3), (1, 1)]),          # sigma order grows
        desc(6, 3, [(6, 3), (6, 3), (1, 1)]),                  # nothing drops
        desc(6, 3, [(6, 3), (3, 2), (1, 1)]),                  # both drop, orders differ
        desc(6, 3, [(6, 2), (3, 2), (1, 1)]),                  # first level is not (6, 3)
        desc(6, 3, [(6, 3), (3, 3), (2, 2)]),                  # last level is not (1, 1)
        desc(6, 3, smoother=2),                                # Schwarz on unequal orders
        desc(12, 8, ne=(4, 1, 20)),                            # 13 * 9 * 20 threads > 1024
    ]
    for d in bad:
        with pytest.raises(B.SemError) as e:
            B.sem_mesh_setup(d)
        assert e.value.status == 1



def test_lserk_coefficients_match_the_oracle():
    """The library's stage-loop coefficients are the five-stage fourth-order scheme the oracle's
    order pins hold (host call, no GPU)."""
    from oracle import lserk
    from paper_2411_14977_amd import binding as B
    a, b, c = B.sem_lserk_coefficients()
    ao, bo, co = lserk.coefficients()
    assert np.array_equal(a, ao) and np.array_equal(b, bo) and np.array_equal(c, co)
