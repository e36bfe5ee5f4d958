"""Oracle: 1D spectral building blocks (test infrastructure only; see oracle/__init__).

Follows Sec. 4.3 ("Element construction in 2D") of the paper:
* orthonormal Legendre polynomials from the three-term recurrence with
  a_k = sqrt(k^2 / ((2k+1)(2k-1))), P~0 = 1/sqrt(2), P~1 = sqrt(3/2) x;
* Legendre-Gauss-Lobatto (GLL) nodes;
* generalized Vandermonde V_ij = psi_j(r_i), V_r = d psi_j / dr (r_i);
* differentiation matrix D_r = V_r V^{-1};
and Sec. 5.2 ("Transfer operators"): I_{Pp} = Phi^p V^{-1}.
"""
import numpy as np
import numpy.polynomial.legendre as npleg


def _a(k):
    # recurrence coefficient a_k of Sec. 4.3
    return np.sqrt(k * k / ((2.0 * k + 1.0) * (2.0 * k - 1.0)))


def legendre_orthonormal(N, x):
    """Rows k=0..N of the orthonormal Legendre polynomials at points x.

    Returns array (N+1, len(x)).  Built only from the paper's recurrence
    a_k P~_k = x P~_{k-1} - a_{k-1} P~_{k-2} and its two starting values.
    """
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((N + 1, x.size))
    out[0] = 1.0 / np.sqrt(2.0)
    if N >= 1:
        out[1] = np.sqrt(1.5) * x
    for k in range(2, N + 1):
        out[k] = (x * out[k - 1] - _a(k - 1) * out[k - 2]) / _a(k)
    return out


def legendre_orthonormal_deriv(N, x):
    """d/dx of the rows of legendre_orthonormal, from differentiating the recurrence:
    a_k P~'_k = P~_{k-1} + x P~'_{k-1} - a_{k-1} P~'_{k-2}."""
    x = np.asarray(x, dtype=np.float64)
    p = legendre_orthonormal(N, x)
    d = np.zeros_like(p)
    if N >= 1:
        d[1] = np.sqrt(1.5)
    for k in range(2, N + 1):
        d[k] = (p[k - 1] + x * d[k - 1] - _a(k - 1) * d[k - 2]) / _a(k)
    return d


def legendre_standard(N, x):
    """Classical (non-normalised) Legendre P_N(x) = P~_N(x) / sqrt((2N+1)/2)."""
    return legendre_orthonormal(N, x)[N] / np.sqrt((2.0 * N + 1.0) / 2.0)


def gll_nodes(P):
    """GLL nodes on [-1,1]: the end points and the P-1 roots of P_P'(x), ascending.

    The roots are located with NumPy's Legendre-series root finder (a library
    primitive) and polished with Newton steps on P~_P' using the recurrence.
    """
    if P < 1:
        raise ValueError("order must be >= 1")
    if P == 1:
        return np.array([-1.0, 1.0])
    inner = np.sort(np.real(npleg.Legendre.basis(P).deriv().roots()))
    for _ in range(6):
        # Newton on f = P~_P'(x); f' = P~_P''(x) from the ODE (1-x^2)P'' = 2xP' - P(P+1)P
        p = legendre_orthonormal(P, inner)[P]
        dp = legendre_orthonormal_deriv(P, inner)[P]
        d2p = (2.0 * inner * dp - P * (P + 1) * p) / (1.0 - inner * inner)
        inner = inner - dp / d2p
    r = np.concatenate(([-1.0], inner, [1.0]))
    if P % 2 == 0:
        r[P // 2] = 0.0          # symmetric rule: the middle node is exactly 0
    # enforce exact antisymmetry of the node set
    r = 0.5 * (r - r[::-1])
    return r


def gll_weights(P, r=None):
    """GLL weights w_i = 2 / (P (P+1) P_P(r_i)^2)."""
    if r is None:
        r = gll_nodes(P)
    return 2.0 / (P * (P + 1) * legendre_standard(P, r) ** 2)


def vandermonde(N, r):
    """V_ij = P~_j(r_i), j = 0..N."""
    return legendre_orthonormal(N, r).T.copy()


def vandermonde_deriv(N, r):
    """(V_r)_ij = P~_j'(r_i)."""
    return legendre_orthonormal_deriv(N, r).T.copy()


def diff_matrix(P):
    """D_r = V_r V^{-1} at the GLL nodes of order P (Sec. 4.3)."""
    r = gll_nodes(P)
    V = vandermonde(P, r)
    Vr = vandermonde_deriv(P, r)
    return np.linalg.solve(V.T, Vr.T).T


def diff_matrix_closed_form(P):
    """Textbook GLL Lagrange-derivative matrix (used only as an independent pin):
    D_ij = P_P(r_i) / (P_P(r_j) (r_i - r_j)) for i != j,
    D_00 = -P(P+1)/4, D_PP = P(P+1)/4, otherwise 0 on the diagonal."""
    r = gll_nodes(P)
    L = legendre_standard(P, r)
    n = P + 1
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = L[i] / (L[j] * (r[i] - r[j]))
    D[0, 0] = -P * (P + 1) / 4.0
    D[P, P] = P * (P + 1) / 4.0
    return D


def transfer_matrix(P_from, P_to):
    """I_{P_from -> P_to} = Phi^{to} V^{-1} (Sec. 5.2).

    V is the Vandermonde of the source nodes (order P_from, modes 0..P_from);
    Phi^{to}_ij = psi_j(r^{to}_i) evaluates the same modes at the target nodes.
    With P_to > P_from this is the prolongation (coarse Lagrange basis sampled at
    fine nodes); shape (P_to+1, P_from+1).
    """
    rs = gll_nodes(P_from)
    rt = gll_nodes(P_to)
    V = vandermonde(P_from, rs)
    Phi = vandermonde(P_from, rt)
    return np.linalg.solve(V.T, Phi.T).T
