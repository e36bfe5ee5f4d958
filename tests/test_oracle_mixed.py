"""Pins of the oracle's mixed-stage sigma-Laplacian (Sec. 3.1, eq. poissonp; eq. weak4 read as
int_{Omega^k} nabla^(k) v . nabla^(k-1) f).

* with equal surfaces it is the same-stage operator;
* brute force: the bilinear form evaluated node by node from the two meshes' isoparametric
  Jacobians (the gradient of each stage from its own nodal coordinates, not from the sigma
  formulas), test function with stage k's, trial function with stage k-1's, stage k's measure;
* constants in the kernel of the unmasked matrix (nabla^(k-1) 1 = 0), and the matrix is not
  symmetric once the surfaces differ.
"""
import math

import numpy as np

from oracle import assemble, mesh, mixed
from tests import oracle_cases as oc


def meshes(Nx=3, Nz=2, P=4, Lx=1.5):
    x = oc.fine_x_nodes(Nx, P, Lx)
    h = 0.5 - 0.1 * np.sin(math.pi * x / Lx)
    ek = 0.05 * np.sin(2 * math.pi * x / Lx + 0.3)
    ekm1 = 0.04 * np.cos(2 * math.pi * x / Lx - 0.2)
    return (mesh.Mesh2D(Nx, Nz, P, Lx, h, ek), mesh.Mesh2D(Nx, Nz, P, Lx, h, ekm1))


def test_equal_surfaces_give_the_same_stage_operator():
    mk, _ = meshes()
    A = mixed.assemble_operator(mk, mk).toarray()
    B = assemble.assemble_operator(mk).toarray()
    assert np.abs(A - B).max() < 1e-14 * np.abs(B).max()


def test_bruteforce_two_geometries():
    mk, mkm1 = meshes(Nx=2, Nz=2, P=3)
    NP, D, w = mk.NP, mk.D, mk.w
    Xk, Zk = mk.X.reshape(mk.E, NP, NP), mk.Z.reshape(mk.E, NP, NP)
    Zp = mkm1.Z.reshape(mk.E, NP, NP)   # same x nodes, the previous stage's z

    def jac(X, Z, e, qi, qj):
        xr = sum(D[qi, k] * X[e, k, qj] for k in range(NP))
        xs = sum(D[qj, k] * X[e, qi, k] for k in range(NP))
        zr = sum(D[qi, k] * Z[e, k, qj] for k in range(NP))
        zs = sum(D[qj, k] * Z[e, qi, k] for k in range(NP))
        return np.array([[xr, xs], [zr, zs]])

    K = np.zeros((mk.N, mk.N))
    for e in range(mk.E):
        g = mk.l2g[e].reshape(NP, NP)
        for qi in range(NP):
            for qj in range(NP):
                Jk, Jp = jac(Xk, Zk, e, qi, qj), jac(Xk, Zp, e, qi, qj)
                Gk, Gp = np.linalg.inv(Jk).T, np.linalg.inv(Jp).T
                wq = w[qi] * w[qj] * abs(np.linalg.det(Jk))
                grads = []
                for a in range(NP):
                    for b in range(NP):
                        dr = D[qi, a] if b == qj else 0.0
                        ds = D[qj, b] if a == qi else 0.0
                        if dr or ds:
                            grads.append((g[a, b], np.array([dr, ds])))
                for gv, rv in grads:
                    for gf, rf in grads:
                        K[gv, gf] += wq * (Gk @ rv) @ (Gp @ rf)
    A = mixed.assemble_stiffness(mk, mkm1).toarray()
    assert np.abs(K - A).max() < 1e-12 * np.abs(A).max()


def test_constant_kernel_and_asymmetry():
    mk, mkm1 = meshes()
    A = mixed.assemble_stiffness(mk, mkm1)
    sc = abs(A).max()
    assert np.abs(A @ np.ones(mk.N)).max() < 1e-13 * sc
    assert abs(A - A.T).max() > 1e-6 * sc
