"""Oracle: the mixed-stage sigma-Laplacian of two stage geometries (test infrastructure only).

Inside a Runge-Kutta stage the paper's pressure operator is the divergence at stage k of a
gradient taken with the previous stage's sigma transform (Sec. 3.1, eq. poissonp; weak form
eq. weak4), nabla^(k) . nabla^(k-1) p.  Reading (the printed weak form pairs the stage labels of
the two cross terms the other way round and leaves the measure open): with
nabla^(m) f = (f_x + sigma_x^(m) f_sigma, sigma_z^(m) f_sigma) (x-derivative at fixed sigma),
integration by parts against v over the stage-k domain gives the bilinear form
    a(v, f) = int_{Omega^k} nabla^(k) v . nabla^(k-1) f dOmega^k
            = int v_x f_x + sigma_x^(k-1) v_x f_sigma + sigma_x^(k) v_sigma f_x
                  + (sigma_x^(k) sigma_x^(k-1) + sigma_z^(k) sigma_z^(k-1)) v_sigma f_sigma,
not symmetric unless the two surfaces agree (then it is the same-stage form of assemble.py).
With GLL collocation and |J| = (dx/2)(d^(k) dsig/2) the per-node factors of
A_e = sum_ab D_a^T diag(G_ab) D_b (a: test derivative, b: trial derivative) are
    G_rr = w d^(k) dsig/dx,  G_rs = w d^(k) sigma_x^(k-1),  G_sr = w d^(k) sigma_x^(k),
    G_ss = w (dx/dsig) d^(k) (sigma_x^(k) sigma_x^(k-1) + 1/(d^(k) d^(k-1))).
The Dirichlet surface is masked as in the same-stage operator.
"""
import numpy as np
import scipy.sparse as sp

from . import assemble


def _node_depth(m):
    """d = h + eta at every element-local node, shape (E, NP, NPz)."""
    d = np.repeat(m.d[:, None, :], m.Nz, axis=1)              # (Nx, Nz, NP)
    return np.repeat(d[..., None], m.NPz, axis=-1).reshape(m.E, m.NP, m.NPz)


def factors(mk, mkm1):
    """(G_rr, G_rs, G_sr, G_ss) of the mixed-stage form, stage k mesh mk, stage k-1 mesh mkm1
    (same tank: elements, orders, length and depth; different surfaces)."""
    ww = np.outer(mk.w, mk.wz)[None]
    dk, dkm1 = _node_depth(mk), _node_depth(mkm1)
    sk, skm1 = mk.sigx, mkm1.sigx
    Grr = ww * dk * mk.dsig / mk.dx
    Grs = ww * dk * skm1
    Gsr = ww * dk * sk
    Gss = ww * (mk.dx / mk.dsig) * dk * (sk * skm1 + 1.0 / (dk * dkm1))
    return Grr, Grs, Gsr, Gss


def element_matrices(mk, mkm1):
    ops = assemble._kron_ops(mk)
    E = mk.E
    Grr, Grs, Gsr, Gss = (g.reshape(E, -1) for g in factors(mk, mkm1))
    A = np.zeros((E, mk.NL, mk.NL))
    for a, b, G in (("r", "r", Grr), ("r", "s", Grs), ("s", "r", Gsr), ("s", "s", Gss)):
        A += np.einsum("ka,ek,kb->eab", ops[a], G, ops[b])
    return A


def assemble_stiffness(mk, mkm1):
    Ae = element_matrices(mk, mkm1)
    NL = Ae.shape[1]
    rows = np.repeat(mk.l2g, NL, axis=1).ravel()
    cols = np.tile(mk.l2g, (1, NL)).ravel()
    return sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(mk.N, mk.N)).tocsr()


def assemble_operator(mk, mkm1, dirichlet=True):
    A = assemble_stiffness(mk, mkm1)
    return assemble.masked(A, mk.dirichlet_nodes()) if dirichlet else A
