"""Oracle: geometric p-multigrid V-cycle and outer iterations (test infrastructure only).

Sec. 5 of the paper:
* grid hierarchy by reducing the polynomial order with the mesh kept (Sec. 5.1).  Eq. gridcoars
  as printed, P_{n-1} = ceil((P_n + 1)/2), stalls at 2 and never reaches the P = 1 coarsest
  grid the section names; it is read as P_{n-1} = ceil(P_n / 2) (8 -> 4 -> 2 -> 1);
* semi-coarsening (Sec. 5.1) where the x and sigma orders differ: each coarser level lowers only
  the larger of the two orders, by the same rule, but not below the smaller one, until they
  match; from there both drop together (16x8 -> 8x8 -> 4x4 -> ..., 2x8 -> 2x4 -> 2x2 -> 1x1;
  the clamp at the smaller order is this reading of "until both directions have matching
  orders").  The prolongation is then the interpolation along the changed direction and the
  identity along the other;
* prolongation from interpolation, I_{Pp} = Phi^p V^{-1}, applied per element and per
  direction (tensor product), and restriction R = P^T (Sec. 5.2);
* a fixed number of smoothing steps on every level before and after the coarse correction
  (Sec. 5.3, V-cycle of Sec. 5); the smoothers here are damped Jacobi, Chebyshev acceleration
  of Jacobi (polynomials in D^{-1} A) and the paper's additive Schwarz smoother (Sec. 5.3):
  x <- x + S^{-1}(b - A x), S^{-1} = W sum_i R_i^T (R_i A R_i^T)^{-1} R_i,
  W = (sum_i R_i R_i^T)^{-1}.  Its subdomains are read as the element blocks (each element's
  (P+1)^d nodes; blocks of neighbouring elements share their face nodes), widened by a chosen
  number of overlap node layers across every face (the paper leaves the overlap to the user);
  2D and 3D;
* the coarsest (P = 1) problem solved exactly (sparse direct).  In 3D the paper's P = 1 grid is
  too large for an exact solve at the benchmark size; the hierarchy is continued below it by
  coarsening the mesh by 2 in x and y (P = 1, linear interpolation in x and y, identity in
  sigma, coarse operators re-discretised from h and eta at the coarse vertices) until a level
  has at most ``coarse_dense_max`` nodes, which is solved exactly.  (The paper is silent on the
  coarse solver; this reading is stated where it is used.)
* coarse operators re-discretised with the same formula at the coarse order;
* outer iterations: preconditioned defect correction x += B(b - A x) (Sec. 5.4), flexible
  conjugate gradients (one-term Polak-Ribiere beta) with B as preconditioner, and GMRES with B
  as right preconditioner (Sec. 5.4 names GMRES, Saad and Schultz 1986): restarted every m
  steps, the k-th iterate of a cycle minimises ||b - A x|| over x0 + span{B v_1 .. B v_k} with
  v_1 .. v_k the Arnoldi basis (the flexible form, Saad 1993, which equals right-preconditioned
  GMRES for the fixed linear B of a V-cycle).

Chebyshev smoothing follows the classical three-term recurrence on the interval
[lo, hi] = [a, b] lambda_hat of D^{-1} A (Saad, "Iterative Methods for Sparse Linear Systems",
Alg. 12.1):  theta = (b+a)/2, delta = (b-a)/2, sigma1 = theta/delta, rho_0 = 1/sigma1,
d_0 = D^{-1} r_0 / theta; then rho_j = 1/(2 sigma1 - rho_{j-1}),
d_j = rho_j rho_{j-1} d_{j-1} + (2 rho_j / delta) D^{-1} r_j, and x_{j+1} = x_j + d_j.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import gll
from .assemble import assemble_operator
from .mesh import Mesh2D, Mesh3D
from .precision import with_stored_factors


def coarsen_orders(P):
    """P, ceil(P/2), ..., 1."""
    out = [int(P)]
    while out[-1] > 1:
        out.append((out[-1] + 1) // 2)
    return out


def coarsen_orders_2d(Px, Pz):
    """Level orders (P_x, P_sigma) from (Px, Pz) down to (1, 1): while the orders differ the
    larger drops to max(ceil(P/2), the smaller); equal orders drop together."""
    out = [(int(Px), int(Pz))]
    while out[-1] != (1, 1):
        px, pz = out[-1]
        if px == pz:
            out.append(((px + 1) // 2, (pz + 1) // 2))
        elif px > pz:
            out.append((max((px + 1) // 2, pz), pz))
        else:
            out.append((px, max((pz + 1) // 2, px)))
    return out


def level_orders_2d(orders):
    """Level orders as (P_x, P_sigma) pairs: an int P stands for (P, P)."""
    return [(int(o), int(o)) if np.isscalar(o) else (int(o[0]), int(o[1])) for o in orders]


def prolongation_1d_linear(Nc):
    """Linear interpolation from Nc to 2 Nc intervals: even fine nodes coincide with coarse
    nodes, odd ones take the mean of their two neighbours."""
    M = sp.lil_matrix((2 * Nc + 1, Nc + 1))
    for f in range(2 * Nc + 1):
        if f % 2 == 0:
            M[f, f // 2] = 1.0
        else:
            M[f, (f - 1) // 2] = 0.5
            M[f, (f + 1) // 2] = 0.5
    return M.tocsr()


def prolongation_1d(Ne, Pc, Pf):
    """Global 1D interpolation matrix from order Pc to order Pf on Ne elements.

    Row of fine node exPf + i, column of coarse node exPc + k holds I_{Pc->Pf}[i, k]; a node
    shared by two elements takes the row of the element on its left (both agree: the
    coarse Lagrange basis is continuous).
    """
    if Pc == Pf:
        return sp.identity(Ne * Pf + 1, format="csr")
    J = gll.transfer_matrix(Pc, Pf)
    nf, nc = Ne * Pf + 1, Ne * Pc + 1
    M = np.zeros((nf, nc))
    for ex in range(Ne - 1, -1, -1):
        M[ex * Pf: ex * Pf + Pf + 1, ex * Pc: ex * Pc + Pc + 1] = J
    return sp.csr_matrix(M)


class Level:
    """One level: its mesh (exact geometry) and the masked operator.  gstore: precision in which
    the level's geometric factors are held ("f64", "f32" or "bf16"); the operator and its
    diagonal are built from the rounded factors, everything else stays exact FP64."""

    def __init__(self, mesh, gstore=None):
        self.mesh = mesh
        self.gstore = gstore
        self.A = assemble_operator(with_stored_factors(mesh, gstore), dirichlet=True)
        self.diag = self.A.diagonal().copy()
        self.dinv = 1.0 / self.diag
        self.dn = mesh.dirichlet_nodes()
        self.N = mesh.N
        self.lam = None          # largest eigenvalue estimate of D^{-1} A
        self.lu = None
        self._blocks = None

    def block_nodes(self, overlap=0):
        """Global nodes of every subdomain: element e's nodes, widened by `overlap` node layers
        across each of its faces into the neighbouring elements (clipped at the domain)."""
        m = self.mesh
        out = []
        if m.dim == 2:
            Px, Pz = m.P, m.Pz
            for e in range(m.E):
                ex, ez = divmod(e, m.Nz)
                ix = np.arange(max(0, ex * Px - overlap), min(m.nx_nodes, ex * Px + Px + overlap + 1))
                iz = np.arange(max(0, ez * Pz - overlap), min(m.nz_nodes, ez * Pz + Pz + overlap + 1))
                out.append((ix[:, None] * m.nz_nodes + iz[None, :]).ravel())
            return out
        P = m.P
        for e in range(m.E):
            ez = e % m.Nz
            ey = (e // m.Nz) % m.Ny
            ex = e // (m.Nz * m.Ny)
            ix = np.arange(max(0, ex * P - overlap), min(m.nx_nodes, ex * P + P + overlap + 1))
            iy = np.arange(max(0, ey * P - overlap), min(m.ny_nodes, ey * P + P + overlap + 1))
            iz = np.arange(max(0, ez * P - overlap), min(m.nz_nodes, ez * P + P + overlap + 1))
            g = (ix[:, None, None] * m.ny_nodes + iy[None, :, None]) * m.nz_nodes + iz[None, None, :]
            out.append(g.ravel())
        return out

    def schwarz_blocks(self, overlap=0):
        """Inverses of the subdomain blocks R_i A R_i^T (A the masked assembled matrix) and the
        weights W = (sum_i R_i R_i^T)^{-1} (one over the number of blocks holding a node)."""
        if self._blocks is None or self._blocks[2] != overlap:
            A = self.A.tocsr()
            nodes = self.block_nodes(overlap)
            inv = [np.linalg.inv(A[idx][:, idx].toarray()) for idx in nodes]
            w = 1.0 / np.bincount(np.concatenate(nodes), minlength=self.N)
            self._blocks = (inv, w, overlap, nodes)
        return self._blocks

    def schwarz(self, r, weighted=True, overlap=0):
        """S^{-1} r = W sum_i R_i^T (R_i A R_i^T)^{-1} R_i r (weighted=False: without W)."""
        inv, w, _, nodes = self.schwarz_blocks(overlap)
        z = np.zeros(self.N)
        for Ai, idx in zip(inv, nodes):
            np.add.at(z, idx, Ai @ r[idx])
        return w * z if weighted else z


class Hierarchy:
    """Levels 0 (finest) .. L-1 (P = 1), prolongations P_l : level l+1 -> level l."""

    def __init__(self, mesh_args, orders, smoother="chebyshev", nu_pre=2, nu_post=2,
                 cheb_degree=3, jacobi_omega=2.0 / 3.0, cheb_lo=0.1, cheb_hi=1.1,
                 coarse_dense_max=1200, gstore=None, schwarz_overlap=0,
                 cheb_degree_coarse=None):
        """orders: level orders, fine to coarse; in 2D an entry may be a pair (P_x, P_sigma)
        (semi-coarsened levels), a plain P meaning (P, P).  gstore: storage precision of the
        geometric factors on every level above the coarsest (None / "f64", "f32", "bf16"); the
        coarsest level is always exact."""
        self.dim = mesh_args["dim"]
        self.orders = list(orders)
        pairs = level_orders_2d(self.orders) if self.dim == 2 else None
        if (pairs[-1] if pairs else self.orders[-1]) not in (1, (1, 1)):
            raise ValueError("coarsest order must be 1")
        self.levels = []
        Pf = pairs[0][0] if pairs else self.orders[0]
        for li, p in enumerate(self.orders):
            gs = gstore if li + 1 < len(self.orders) else None
            if self.dim == 2:
                m = Mesh2D(mesh_args["Nx"], mesh_args["Nz"], pairs[li][0], mesh_args["Lx"],
                           mesh_args["h"], mesh_args["eta"], P_fine=Pf, Pz=pairs[li][1])
            else:
                m = Mesh3D(mesh_args["Nx"], mesh_args["Ny"], mesh_args["Nz"], p,
                           mesh_args["Lx"], mesh_args["Ly"], mesh_args["h"], mesh_args["eta"],
                           P_fine=Pf)
            self.levels.append(Level(m, gs))
        self.P = []
        for l in range(len(self.orders) - 1):
            if self.dim == 2:
                (pfx, pfz), (pcx, pcz) = pairs[l], pairs[l + 1]
                Pm = sp.kron(prolongation_1d(mesh_args["Nx"], pcx, pfx),
                             prolongation_1d(mesh_args["Nz"], pcz, pfz))
            else:
                pf, pc = self.orders[l], self.orders[l + 1]
                Px = prolongation_1d(mesh_args["Nx"], pc, pf)
                Pz = prolongation_1d(mesh_args["Nz"], pc, pf)
                Py = prolongation_1d(mesh_args["Ny"], pc, pf)
                Pm = sp.kron(sp.kron(Px, Py), Pz)
            self.P.append(Pm.tocsr())
        if self.dim == 3:
            # h-levels below P = 1 (x, y halved; vertices of the coarse mesh are fine vertices)
            Nx, Ny, Nz = mesh_args["Nx"], mesh_args["Ny"], mesh_args["Nz"]
            h, eta = np.asarray(mesh_args["h"]), np.asarray(mesh_args["eta"])
            nx, ny = Nx, Ny
            while (self.levels[-1].N > coarse_dense_max and nx % 2 == 0 and ny % 2 == 0
                   and len(self.levels) < 16):
                ncx, ncy = nx // 2, ny // 2
                f = (Nx // ncx) * Pf
                m = Mesh3D(ncx, ncy, Nz, 1, mesh_args["Lx"], mesh_args["Ly"], h[::f, ::f],
                           eta[::f, ::f], P_fine=1)
                self.levels.append(Level(m))
                Pm = sp.kron(sp.kron(prolongation_1d_linear(ncx), prolongation_1d_linear(ncy)),
                             sp.identity(Nz + 1))
                self.P.append(Pm.tocsr())
                nx, ny = ncx, ncy
        # every level above the (possibly h-coarsened) coarsest holds its factors in gstore
        for li in range(len(self.levels) - 1):
            if self.levels[li].gstore != gstore:
                self.levels[li] = Level(self.levels[li].mesh, gstore)
        last = self.levels[-1]
        last.lu = spla.splu(sp.csc_matrix(last.A))
        self.smoother = smoother
        self.schwarz_overlap = int(schwarz_overlap)
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.cheb_degree = cheb_degree
        self.cheb_degree_coarse = cheb_degree_coarse or cheb_degree   # levels 1 .. L-2
        self.omega = jacobi_omega
        self.cheb_lo, self.cheb_hi = cheb_lo, cheb_hi

    # ---- smoothing -------------------------------------------------------------------
    def set_lambda(self, l, lam):
        self.levels[l].lam = float(lam)

    def jacobi(self, l, b, x, sweeps):
        L = self.levels[l]
        for _ in range(sweeps):
            x = x + self.omega * L.dinv * (b - L.A @ x)
        return x

    def chebyshev(self, l, b, x, degree):
        L = self.levels[l]
        a_ = self.cheb_lo * L.lam
        b_ = self.cheb_hi * L.lam
        theta = 0.5 * (b_ + a_)
        delta = 0.5 * (b_ - a_)
        sigma1 = theta / delta
        rho = 1.0 / sigma1
        r = b - L.A @ x
        d = L.dinv * r / theta
        x = x + d
        for _ in range(1, degree):
            rho_new = 1.0 / (2.0 * sigma1 - rho)
            r = b - L.A @ x
            d = rho_new * rho * d + (2.0 * rho_new / delta) * (L.dinv * r)
            rho = rho_new
            x = x + d
        return x

    def schwarz_sweeps(self, l, b, x, sweeps):
        """Additive Schwarz smoothing (Sec. 5.3): x <- x - S^{-1}(A x - b), ``sweeps`` times."""
        L = self.levels[l]
        for _ in range(sweeps):
            x = x + L.schwarz(b - L.A @ x, overlap=self.schwarz_overlap)
        return x

    def smooth(self, l, b, x, pre):
        if self.smoother == "jacobi":
            return self.jacobi(l, b, x, self.nu_pre if pre else self.nu_post)
        if self.smoother == "asm":
            return self.schwarz_sweeps(l, b, x, self.nu_pre if pre else self.nu_post)
        return self.chebyshev(l, b, x, self.cheb_degree if l == 0 else self.cheb_degree_coarse)

    # ---- V-cycle -----------------------------------------------------------------------
    def restrict(self, l, r_fine):
        rc = self.P[l].T @ r_fine
        rc[self.levels[l + 1].dn] = 0.0
        return rc

    def prolong(self, l, e_coarse):
        return self.P[l] @ e_coarse

    def coarse_solve(self, b):
        return self.levels[-1].lu.solve(b)

    def vcycle(self, b, l=0, hook=None, hook_post=None):
        """z = B b with zero initial guess.  Two optional stages on level l, each a map
        (l, b, x) -> new x (used for the learned stage): ``hook`` after the pre-smoothing (before
        the residual that is restricted), ``hook_post`` after the coarse-grid correction has been
        added (before the post-smoothing)."""
        if l == len(self.levels) - 1:
            return self.coarse_solve(b)
        L = self.levels[l]
        x = self.smooth(l, b, np.zeros_like(b), pre=True)
        if hook is not None:
            x = hook(l, b, x)
        r = b - L.A @ x
        ec = self.vcycle(self.restrict(l, r), l + 1, hook, hook_post)
        x = x + self.prolong(l, ec)
        if hook_post is not None:
            x = hook_post(l, b, x)
        x = self.smooth(l, b, x, pre=False)
        return x


def lanczos_lambda_max(A, dinv, v0, steps=20):
    """Largest Ritz value of D^{-1/2} A D^{-1/2} after ``steps`` Lanczos steps from v0
    (which equals the largest eigenvalue estimate of D^{-1} A)."""
    s = np.sqrt(dinv)
    q = v0 / np.linalg.norm(v0)
    q_prev = np.zeros_like(q)
    alphas, betas = [], []
    beta = 0.0
    for k in range(steps):
        w = s * (A @ (s * q))
        alpha = float(q @ w)
        w = w - alpha * q - beta * q_prev
        alphas.append(alpha)
        beta = float(np.linalg.norm(w))
        if k == steps - 1 or beta == 0.0:
            break
        betas.append(beta)
        q_prev, q = q, w / beta
    T = np.diag(alphas) + np.diag(betas[:len(alphas) - 1], 1) + np.diag(betas[:len(alphas) - 1], -1)
    return float(np.linalg.eigvalsh(T)[-1])


def splitmix64_uniform(n, seed):
    """Counter-based start vector: SplitMix64 (Steele, Lea, Flood 2014) of (seed + i), mapped
    to [-1, 1) with the top 53 bits.  Both sides of the parity tests implement this
    published generator independently."""
    M = (1 << 64) - 1
    out = np.empty(n)
    for i in range(n):
        z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        z = z ^ (z >> 31)
        out[i] = (z >> 11) * (1.0 / (1 << 53)) * 2.0 - 1.0
    return out


def estimate_lambdas(H, steps=20, seed=12345):
    for l, L in enumerate(H.levels[:-1]):
        v0 = splitmix64_uniform(L.N, seed)
        v0[L.dn] = 0.0
        H.set_lambda(l, lanczos_lambda_max(L.A, L.dinv, v0, steps))


# ---- outer iterations ------------------------------------------------------------------
def pcg(A, b, x0, prec, tol, maxit=500):
    """Standard preconditioned CG (linear preconditioner); returns x, iterations, history."""
    x = x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    z = prec(r)
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / nb]
    for it in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= tol:
            return x, it, hist
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, hist


def fpcg(A, b, x0, prec, tol, maxit=500):
    """Flexible CG (Notay 2000), one-term Polak-Ribiere:
    beta = z_{k+1}.(r_{k+1} - r_k) / (r_k . z_k) = -alpha z_{k+1}.q_k / (r_k . z_k)."""
    x = x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    z = prec(r)
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / nb]
    if hist[-1] <= tol:
        return x, 0, hist
    for it in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= tol:
            return x, it, hist
        z = prec(r)
        beta = -alpha * (z @ q) / rz
        rz = r @ z
        p = z + beta * p
    return x, maxit, hist


def pdc(A, b, x0, prec, tol, maxit=500):
    """Preconditioned defect correction x_{k+1} = x_k + B (b - A x_k) (Sec. 5.4)."""
    x = x0.copy()
    nb = np.linalg.norm(b)
    r = b - A @ x
    hist = [np.linalg.norm(r) / nb]
    for it in range(1, maxit + 1):
        x = x + prec(r)
        r = b - A @ x
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= tol:
            return x, it, hist
    return x, maxit, hist


def gmres(A, b, x0, prec, tol, restart=30, maxit=500):
    """Right-preconditioned (flexible) GMRES(m): every step z_j = B v_j, w = A z_j orthogonalised
    against v_1 .. v_j (modified Gram-Schmidt) gives column j of the Hessenberg matrix H; the
    iterate x0 + Z y minimises ||beta e_1 - H y|| (least squares solved directly, no rotations).
    hist: relative residual norms ||b - A x|| / ||b|| of every iterate, computed from x."""
    x = x0.copy()
    nb = np.linalg.norm(b)
    r = b - A @ x
    hist = [np.linalg.norm(r) / nb]
    if hist[-1] <= tol:
        return x, 0, hist
    it = 0
    while it < maxit:
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        x_start = x.copy()
        for j in range(restart):
            z = prec(V[j])
            Z.append(z)
            w = A @ z
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            g = np.zeros(j + 2)
            g[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], g, rcond=None)[0]
            x = x_start + np.column_stack(Z) @ y
            r = b - A @ x
            it += 1
            hist.append(np.linalg.norm(r) / nb)
            if hist[-1] <= tol or it >= maxit or H[j + 1, j] == 0:
                break
        if hist[-1] <= tol:
            return x, it, hist
    return x, it, hist
