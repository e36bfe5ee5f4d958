"""Pins of the oracle's overlapping and 3D additive Schwarz smoother (Sec. 5.3).

The subdomain of element e is its own nodes widened by a number of node layers across every
face; the pins do not retype that box rule:

* subdomains equal a breadth-first search of king moves (8 neighbours in 2D, 26 in 3D) over the
  node grid, `overlap` steps out from the element's nodes taken from the mesh connectivity;
  with no overlap they are the element's own nodes;
* when every subdomain covers the whole domain, W = 1/E and S^{-1} = A^{-1}: one sweep from
  zero is the exact solve (2D and 3D);
* the unweighted sum is symmetric, the weights are one over the number of subdomains holding a
  node (brute-force count), and the sum equals the dense construction with 0/1 restrictions;
* as a smoother it converges to the direct solution, and overlap lowers the iteration count.
"""
import itertools

import numpy as np

import workloads as W
from oracle import assemble, pmg
from tests import oracle_cases as oc


def _tank2d(Nx=3, Nz=2, P=3, **kw):
    wl = W.tank(Nx, Nz, P, Lx=25.6 * Nx / 256)
    return wl, oc.hierarchy(wl, smoother="asm", **kw)


def _tank3d(Nx=2, Ny=2, Nz=2, P=2, **kw):
    wl = W.tank3d(Nx, Ny, Nz, P, L=0.8)
    return wl, oc.hierarchy(wl, smoother="asm", **kw)


def _grid_shape(m):
    return (m.nx_nodes, m.nz_nodes) if m.dim == 2 else (m.nx_nodes, m.ny_nodes, m.nz_nodes)


def _bfs_nodes(m, e, overlap):
    """Nodes within `overlap` king moves of element e's nodes (from the connectivity l2g)."""
    shape = _grid_shape(m)
    seen = {tuple(int(v) for v in np.unravel_index(g, shape)) for g in m.l2g[e]}
    front = set(seen)
    steps = list(itertools.product((-1, 0, 1), repeat=len(shape)))
    for _ in range(overlap):
        nxt = set()
        for p in front:
            for s in steps:
                q = tuple(a + b for a, b in zip(p, s))
                if all(0 <= q[k] < shape[k] for k in range(len(shape))) and q not in seen:
                    nxt.add(q)
        seen |= nxt
        front = nxt
    return sorted(int(np.ravel_multi_index(p, shape)) for p in seen)


def test_subdomains_are_king_move_neighbourhoods_2d():
    for (Nx, Nz, P) in ((3, 3, 3), (4, 2, 2)):
        _, H = _tank2d(Nx, Nz, P)
        L = H.levels[0]
        for ov in (0, 1, 2, 4):
            nodes = L.block_nodes(ov)
            assert len(nodes) == L.mesh.E
            for e in range(L.mesh.E):
                assert list(nodes[e]) == _bfs_nodes(L.mesh, e, ov), (Nx, Nz, P, ov, e)
        # no overlap: exactly the element's nodes, in its local order
        for e in range(L.mesh.E):
            assert np.array_equal(L.block_nodes(0)[e], L.mesh.l2g[e])


def test_subdomains_are_king_move_neighbourhoods_3d():
    _, H = _tank3d(Nx=3, Ny=2, Nz=2, P=2)
    L = H.levels[0]
    for ov in (0, 1, 3):
        nodes = L.block_nodes(ov)
        for e in range(L.mesh.E):
            assert list(nodes[e]) == _bfs_nodes(L.mesh, e, ov), (ov, e)
    for e in range(L.mesh.E):
        assert np.array_equal(L.block_nodes(0)[e], L.mesh.l2g[e])


def _exact_one_sweep(H, ov):
    L = H.levels[0]
    b = W.random_vector(L.N, 11)
    b[L.dn] = 0.0
    H.schwarz_overlap = ov
    x = H.schwarz_sweeps(0, b, np.zeros(L.N), 1)
    xd = np.linalg.solve(L.A.toarray(), b)
    return np.abs(x - xd).max() / np.abs(xd).max()


def test_whole_domain_subdomains_solve_exactly():
    _, H = _tank2d(Nx=3, Nz=2, P=2)
    m = H.levels[0].mesh
    ov = max(m.nx_nodes, m.nz_nodes)
    w = H.levels[0].schwarz_blocks(ov)[1]
    assert np.allclose(w, 1.0 / m.E, rtol=0, atol=0)
    assert _exact_one_sweep(H, ov) < 1e-11
    # a smaller overlap is not exact
    assert _exact_one_sweep(H, 1) > 1e-6
    _, H3 = _tank3d(Nx=2, Ny=2, Nz=1, P=2)
    m3 = H3.levels[0].mesh
    assert _exact_one_sweep(H3, max(m3.nx_nodes, m3.ny_nodes, m3.nz_nodes)) < 1e-11


def _dense_S(L, ov, weighted=True):
    n = L.N
    S = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        S[:, k] = L.schwarz(e, weighted=weighted, overlap=ov)
    return S


def test_overlap_symmetry_weights_and_dense_construction():
    for make, ov in ((lambda: _tank2d(Nx=3, Nz=2, P=2), 1), (lambda: _tank2d(Nx=3, Nz=3, P=3), 2),
                     (lambda: _tank3d(Nx=2, Ny=2, Nz=1, P=2), 0),
                     (lambda: _tank3d(Nx=2, Ny=2, Nz=2, P=1), 1)):
        _, H = make()
        L = H.levels[0]
        n = L.N
        S0 = _dense_S(L, ov, weighted=False)
        assert np.abs(S0 - S0.T).max() < 1e-11 * np.abs(S0).max()
        sets = [_bfs_nodes(L.mesh, e, ov) for e in range(L.mesh.E)]
        counts = np.zeros(n)
        for s in sets:
            counts[s] += 1.0
        w = L.schwarz_blocks(ov)[1]
        assert np.allclose(w * counts, 1.0, rtol=1e-15, atol=0)
        A = L.A.toarray()
        Rs = []
        for s in sets:
            R = np.zeros((len(s), n))
            R[np.arange(len(s)), s] = 1.0
            Rs.append(R)
        S = np.diag(1.0 / counts) @ sum(R.T @ np.linalg.inv(R @ A @ R.T) @ R for R in Rs)
        Sw = _dense_S(L, ov)
        assert np.abs(Sw - S).max() < 1e-11 * np.abs(S).max()


def _pcg_iters(H, b):
    L = H.levels[0]
    x, it, _ = pmg.fpcg(L.A, b, np.zeros(L.N), H.vcycle, 1e-10)
    xd = assemble.solve_direct(L.A, b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    return it


def test_overlapping_smoother_converges_and_overlap_helps_2d():
    its = []
    for ov in (0, 1, 2):
        _, H = _tank2d(Nx=8, Nz=2, P=4, nu_pre=1, nu_post=1, schwarz_overlap=ov)
        L = H.levels[0]
        b = W.random_vector(L.N, 7)
        b[L.dn] = 0.0
        its.append(_pcg_iters(H, b))
    assert its[1] <= its[0] and its[2] <= its[1], its
    assert its[2] < its[0], its


def test_3d_smoother_converges():
    its = []
    for ov in (0, 1):
        _, H = _tank3d(Nx=2, Ny=2, Nz=2, P=3, nu_pre=1, nu_post=1, schwarz_overlap=ov)
        L = H.levels[0]
        b = W.random_vector(L.N, 9)
        b[L.dn] = 0.0
        its.append(_pcg_iters(H, b))
    assert its[1] <= its[0] <= 25, its
