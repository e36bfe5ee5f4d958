"""Oracle: sigma-mapped spectral-element meshes and geometric factors (test infrastructure only).

The vertical coordinate is sigma = (z + h(x)) / d(x), d = eta + h (Sec. 2.2, eq. sigtrans),
so a node with horizontal position x and sigma-value sigma sits at z = -h(x) + sigma d(x).
Horizontal elements are affine; in the vertical the N_z element layers split [0,1] in sigma
evenly.  Following the sigma-derivative formulas (eq. 1_Scoef):
    sigma_x = (h_x - sigma d_x) / d,   sigma_z = 1 / d,
with h_x, d_x obtained by differentiating the nodal h, d on each element with the spectral
differentiation matrix (the paper evaluates such gradients "numerically using the spectral
element method").

The bilinear form is read as the symmetric Galerkin form int grad v . grad p dOmega in the
physical measure, with grad = grad_sigma of Sec. 2.2.  With GLL collocation (weights w) the
per-node geometric factors G = w |J| (grad xi)(grad xi)^T are, in 2D with reference
coordinates (r, s) <-> (x, sigma):
    G_rr = w_i w_j d dsig/dx,  G_rs = w_i w_j d sigma_x,  G_ss = w_i w_j (dx/dsig) d (sigma_x^2 + d^-2)
and the lumped mass is w_i w_j d dx dsig / 4.

Node numbering (global): 2D g = ix (Nz P + 1) + iz; 3D g = (ix (Ny P + 1) + iy)(Nz P + 1) + iz,
vertical index fastest.  Elements: 2D e = ex Nz + ez, 3D e = (ex Ny + ey) Nz + ez.
Element-local node (i[, m], j) with i along x, m along y, j along sigma; j fastest.
Level meshes take h and eta sampled at the FINE level's horizontal GLL nodes and
interpolate them element by element with the transfer matrix I_{Pp} of Sec. 5.2.

2D meshes may carry different orders along x (P) and sigma (Pz), as the semi-coarsened levels of
Sec. 5.1 do: the element is then the tensor product of the order-P GLL rule in x and the
order-Pz rule in sigma (local node (i, j), i = 0..P, j = 0..Pz, j fastest), and every formula
above takes its x factor from the first rule and its sigma factor from the second.
"""
import numpy as np

from . import gll


class Mesh2D:
    dim = 2

    def __init__(self, Nx, Nz, P, Lx, h_fine, eta_fine, P_fine=None, Pz=None):
        """P: order along x; Pz: order along sigma (default P); P_fine: horizontal order of
        the grid h_fine and eta_fine are sampled on."""
        P_fine = P if P_fine is None else P_fine
        Pz = P if Pz is None else int(Pz)
        self.Nx, self.Nz, self.P, self.Pz, self.Lx = int(Nx), int(Nz), int(P), Pz, float(Lx)
        self.NP = P + 1
        self.NPz = Pz + 1
        self.NL = self.NP * self.NPz
        self.E = self.Nx * self.Nz
        self.r = gll.gll_nodes(P)
        self.w = gll.gll_weights(P, self.r)
        self.D = gll.diff_matrix(P)
        self.rz = gll.gll_nodes(Pz)
        self.wz = gll.gll_weights(Pz, self.rz)
        self.Dz = gll.diff_matrix(Pz)
        self.dx = self.Lx / self.Nx
        self.dsig = 1.0 / self.Nz
        h_fine = np.asarray(h_fine, dtype=np.float64)
        eta_fine = np.asarray(eta_fine, dtype=np.float64)
        if h_fine.shape != (self.Nx * P_fine + 1,) or eta_fine.shape != h_fine.shape:
            raise ValueError("h/eta must be sampled at the fine horizontal GLL nodes")
        idx = np.arange(self.Nx)[:, None] * P_fine + np.arange(P_fine + 1)[None, :]
        I = np.eye(P + 1) if P == P_fine else gll.transfer_matrix(P_fine, P)
        # column data per element: (Nx, P+1)
        self.h = h_fine[idx] @ I.T
        self.eta = eta_fine[idx] @ I.T
        self.d = self.h + self.eta
        self.hx = (2.0 / self.dx) * (self.h @ self.D.T)
        self.dxd = (2.0 / self.dx) * (self.d @ self.D.T)
        # coordinates of element-local nodes, arrays (Nx, Nz, NP, NPz)
        ex = np.arange(self.Nx)[:, None, None, None]
        ez = np.arange(self.Nz)[None, :, None, None]
        ri = self.r[None, None, :, None]
        sj = self.rz[None, None, None, :]
        full = np.zeros((self.Nx, self.Nz, self.NP, self.NPz))
        self.X = self.Lx * (ex + (ri + 1.0) / 2.0) / self.Nx + full
        self.SIG = (ez + (sj + 1.0) / 2.0) / self.Nz + full
        d4 = self.d[:, None, :, None]
        h4 = self.h[:, None, :, None]
        self.Z = -h4 + self.SIG * d4
        sigx = (self.hx[:, None, :, None] - self.SIG * self.dxd[:, None, :, None]) / d4
        ww = (self.w[:, None] * self.wz[None, :])[None, None] * np.ones((self.Nx, self.Nz, 1, 1))
        EL = (self.E, self.NP, self.NPz)
        self.Grr = (ww * d4 * self.dsig / self.dx).reshape(EL)
        self.Grs = (ww * d4 * sigx).reshape(EL)
        self.Gss = (ww * (self.dx / self.dsig) * d4 * (sigx * sigx + 1.0 / (d4 * d4))).reshape(EL)
        self.mass = (ww * d4 * self.dx * self.dsig / 4.0).reshape(EL)
        self.sigx = sigx.reshape(EL)
        self.nx_nodes = self.Nx * P + 1
        self.nz_nodes = self.Nz * Pz + 1
        self.N = self.nx_nodes * self.nz_nodes
        gi = (np.arange(self.Nx)[:, None, None, None] * P + np.arange(self.NP)[None, None, :, None])
        gj = (np.arange(self.Nz)[None, :, None, None] * Pz
              + np.arange(self.NPz)[None, None, None, :])
        self.l2g = (gi * self.nz_nodes + gj).reshape(self.E, self.NL)
        self.Xe = self.X.reshape(self.E, -1)
        self.Ze = self.Z.reshape(self.E, -1)

    def fields(self):
        return [self.Grr, self.Grs, self.Gss]

    def node_coords(self):
        """Global node coordinates (x, z), each node taken from the first element holding it."""
        x = np.zeros(self.N)
        z = np.zeros(self.N)
        x[self.l2g[::-1].ravel()] = self.Xe[::-1].ravel()
        z[self.l2g[::-1].ravel()] = self.Ze[::-1].ravel()
        return x, z

    def dirichlet_nodes(self):
        """Global indices on the free surface (top, iz = Nz P)."""
        return np.arange(self.nx_nodes) * self.nz_nodes + (self.nz_nodes - 1)

    def face_weights(self):
        """GLL surface quadrature weights w * |dGamma| on the Neumann faces.

        Returns dict face -> (global node indices, weights), faces 'left' (x=0), 'right'
        (x=Lx) and 'bottom' (z=-h).  Walls: dGamma = d dsig/2; bottom: (dx/2) sqrt(1+h_x^2).
        """
        P, NP, Pz = self.P, self.NP, self.Pz
        out = {}
        for name, ex, i in (("left", 0, 0), ("right", self.Nx - 1, P)):
            idx = np.zeros(self.nz_nodes, dtype=np.int64)
            wts = np.zeros(self.nz_nodes)
            for ez in range(self.Nz):
                for j in range(self.NPz):
                    iz = ez * Pz + j
                    idx[iz] = (ex * P + i) * self.nz_nodes + iz
                    wts[iz] += self.wz[j] * self.d[ex, i] * self.dsig / 2.0
            out[name] = (idx, wts)
        idx = np.zeros(self.nx_nodes, dtype=np.int64)
        wts = np.zeros(self.nx_nodes)
        for ex in range(self.Nx):
            for i in range(NP):
                ix = ex * P + i
                idx[ix] = ix * self.nz_nodes
                wts[ix] += self.w[i] * (self.dx / 2.0) * np.sqrt(1.0 + self.hx[ex, i] ** 2)
        out["bottom"] = (idx, wts)
        return out


class Mesh3D:
    dim = 3

    def __init__(self, Nx, Ny, Nz, P, Lx, Ly, h_fine, eta_fine, P_fine=None):
        P_fine = P if P_fine is None else P_fine
        self.Nx, self.Ny, self.Nz, self.P = int(Nx), int(Ny), int(Nz), int(P)
        self.Lx, self.Ly = float(Lx), float(Ly)
        self.NP = P + 1
        self.NL = self.NP ** 3
        self.E = self.Nx * self.Ny * self.Nz
        self.r = gll.gll_nodes(P)
        self.w = gll.gll_weights(P, self.r)
        self.D = gll.diff_matrix(P)
        self.dx = self.Lx / self.Nx
        self.dy = self.Ly / self.Ny
        self.dsig = 1.0 / self.Nz
        h_fine = np.asarray(h_fine, dtype=np.float64)
        eta_fine = np.asarray(eta_fine, dtype=np.float64)
        shp = (self.Nx * P_fine + 1, self.Ny * P_fine + 1)
        if h_fine.shape != shp or eta_fine.shape != shp:
            raise ValueError("h/eta must be sampled at the fine horizontal GLL grid")
        ix = np.arange(self.Nx)[:, None] * P_fine + np.arange(P_fine + 1)[None, :]
        iy = np.arange(self.Ny)[:, None] * P_fine + np.arange(P_fine + 1)[None, :]
        I = np.eye(P + 1) if P == P_fine else gll.transfer_matrix(P_fine, P)

        def to_elems(F):
            # (Nx, Ny, Pf+1, Pf+1) -> interpolate both axes -> (Nx, Ny, NP, NP)
            Fe = F[ix[:, None, :, None], iy[None, :, None, :]]
            return np.einsum("ia,xyab,jb->xyij", I, Fe, I)

        self.h = to_elems(h_fine)
        self.eta = to_elems(eta_fine)
        self.d = self.h + self.eta
        D = self.D
        self.hx = (2.0 / self.dx) * np.einsum("ia,xyaj->xyij", D, self.h)
        self.hy = (2.0 / self.dy) * np.einsum("ja,xyia->xyij", D, self.h)
        self.dxd = (2.0 / self.dx) * np.einsum("ia,xyaj->xyij", D, self.d)
        self.dyd = (2.0 / self.dy) * np.einsum("ja,xyia->xyij", D, self.d)
        NP = self.NP
        shape6 = (self.Nx, self.Ny, self.Nz, NP, NP, NP)
        ex = np.arange(self.Nx).reshape(-1, 1, 1, 1, 1, 1)
        ey = np.arange(self.Ny).reshape(1, -1, 1, 1, 1, 1)
        ez = np.arange(self.Nz).reshape(1, 1, -1, 1, 1, 1)
        ri = self.r.reshape(1, 1, 1, -1, 1, 1)
        tm = self.r.reshape(1, 1, 1, 1, -1, 1)
        sj = self.r.reshape(1, 1, 1, 1, 1, -1)
        zero = np.zeros(shape6)
        self.X = self.Lx * (ex + (ri + 1.0) / 2.0) / self.Nx + zero
        self.Y = self.Ly * (ey + (tm + 1.0) / 2.0) / self.Ny + zero
        self.SIG = (ez + (sj + 1.0) / 2.0) / self.Nz + zero

        def col(a):
            return a[:, :, None, :, :, None]

        d6 = col(self.d)
        self.Z = -col(self.h) + self.SIG * d6
        sigx = (col(self.hx) - self.SIG * col(self.dxd)) / d6
        sigy = (col(self.hy) - self.SIG * col(self.dyd)) / d6
        w3 = (self.w[:, None, None] * self.w[None, :, None] * self.w[None, None, :])[None, None, None]
        jac = (self.dx / 2.0) * (self.dy / 2.0) * (d6 * self.dsig / 2.0)
        wj = w3 * jac + zero
        rx, ty, ss = 2.0 / self.dx, 2.0 / self.dy, 2.0 / self.dsig
        EL = (self.E, NP, NP, NP)
        self.Grr = (wj * rx * rx).reshape(EL)
        self.Gtt = (wj * ty * ty).reshape(EL)
        self.Grs = (wj * rx * ss * sigx).reshape(EL)
        self.Gts = (wj * ty * ss * sigy).reshape(EL)
        self.Gss = (wj * ss * ss * (sigx * sigx + sigy * sigy + 1.0 / (d6 * d6))).reshape(EL)
        self.mass = (w3 * (self.dx * self.dy * self.dsig / 8.0) * d6 + zero).reshape(EL)
        self.nx_nodes = self.Nx * P + 1
        self.ny_nodes = self.Ny * P + 1
        self.nz_nodes = self.Nz * P + 1
        self.N = self.nx_nodes * self.ny_nodes * self.nz_nodes
        gi = ex * P + np.arange(NP).reshape(1, 1, 1, -1, 1, 1)
        gm = ey * P + np.arange(NP).reshape(1, 1, 1, 1, -1, 1)
        gj = ez * P + np.arange(NP).reshape(1, 1, 1, 1, 1, -1)
        g = (gi * self.ny_nodes + gm) * self.nz_nodes + gj
        self.l2g = g.reshape(self.E, NP ** 3).astype(np.int64)
        self.Xe = self.X.reshape(self.E, -1)
        self.Ye = self.Y.reshape(self.E, -1)
        self.Ze = self.Z.reshape(self.E, -1)

    def fields(self):
        return [self.Grr, self.Gtt, self.Grs, self.Gts, self.Gss]

    def node_coords(self):
        x = np.zeros(self.N)
        y = np.zeros(self.N)
        z = np.zeros(self.N)
        x[self.l2g[::-1].ravel()] = self.Xe[::-1].ravel()
        y[self.l2g[::-1].ravel()] = self.Ye[::-1].ravel()
        z[self.l2g[::-1].ravel()] = self.Ze[::-1].ravel()
        return x, y, z

    def dirichlet_nodes(self):
        hz = np.arange(self.nx_nodes * self.ny_nodes)
        return hz * self.nz_nodes + (self.nz_nodes - 1)

    def face_weights(self):
        """Faces 'xlo', 'xhi', 'ylo', 'yhi' (vertical walls) and 'bottom'.

        Wall x=const: dGamma = (dy/2)(d dsig/2) w_m w_j; wall y=const: (dx/2)(d dsig/2) w_i w_j;
        bottom z=-h(x,y): (dx/2)(dy/2) sqrt(1+h_x^2+h_y^2) w_i w_m.
        Index arrays are over the face's own node grid, flattened with the later axis fastest.
        """
        P, NP = self.P, self.NP
        nyn, nzn, nxn = self.ny_nodes, self.nz_nodes, self.nx_nodes
        out = {}
        for name, ex, i in (("xlo", 0, 0), ("xhi", self.Nx - 1, P)):
            idx = np.zeros((nyn, nzn), dtype=np.int64)
            wts = np.zeros((nyn, nzn))
            for ey in range(self.Ny):
                for m in range(NP):
                    for ez in range(self.Nz):
                        for j in range(NP):
                            iy, iz = ey * P + m, ez * P + j
                            idx[iy, iz] = ((ex * P + i) * nyn + iy) * nzn + iz
                            wts[iy, iz] += (self.w[m] * self.w[j] * (self.dy / 2.0)
                                            * self.d[ex, ey, i, m] * self.dsig / 2.0)
            out[name] = (idx.ravel(), wts.ravel())
        for name, ey, m in (("ylo", 0, 0), ("yhi", self.Ny - 1, P)):
            idx = np.zeros((nxn, nzn), dtype=np.int64)
            wts = np.zeros((nxn, nzn))
            for ex in range(self.Nx):
                for i in range(NP):
                    for ez in range(self.Nz):
                        for j in range(NP):
                            ixx, iz = ex * P + i, ez * P + j
                            idx[ixx, iz] = (ixx * nyn + ey * P + m) * nzn + iz
                            wts[ixx, iz] += (self.w[i] * self.w[j] * (self.dx / 2.0)
                                             * self.d[ex, ey, i, m] * self.dsig / 2.0)
            out[name] = (idx.ravel(), wts.ravel())
        idx = np.zeros((nxn, nyn), dtype=np.int64)
        wts = np.zeros((nxn, nyn))
        for ex in range(self.Nx):
            for ey in range(self.Ny):
                for i in range(NP):
                    for m in range(NP):
                        ixx, iy = ex * P + i, ey * P + m
                        idx[ixx, iy] = (ixx * nyn + iy) * nzn
                        wts[ixx, iy] += (self.w[i] * self.w[m] * (self.dx / 2.0) * (self.dy / 2.0)
                                         * np.sqrt(1.0 + self.hx[ex, ey, i, m] ** 2
                                                   + self.hy[ex, ey, i, m] ** 2))
        out["bottom"] = (idx.ravel(), wts.ravel())
        return out
