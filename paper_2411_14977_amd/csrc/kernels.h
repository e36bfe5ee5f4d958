// Launch wrappers of the gfx950 kernels (implemented in kernels.hip).  All launches are
// asynchronous on the given stream; sizes are validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace semk {

constexpr int NRED = 1024;   // partial sums per reduction (fixed: deterministic results)
constexpr int RED_THREADS = 256;

// G_COL64 (2D FP64 operator): no stored factors; the kernel forms them from four FP64 values per
// element column and horizontal node, [ex][i] {w_i d dsig/dx, w_i dx/(dsig d), h_x, d_x}
// (d = h + eta): G_rr = w_j c0, G_rs = w_i w_j (h_x - sigma d_x), G_ss = w_j c3 ((h_x -
// sigma d_x)^2 + 1), which are the sigma-mapped factors of the stored layouts
enum GType { G_F64 = 0, G_F32 = 1, G_BF16 = 2, G_COL64 = 3 };
constexpr int COLGEO_N = 4;  // values per column node of G_COL64 (2D)
// 3D G_COL64: per element column (ex, ey) and horizontal node (i, m), eight FP64 values
// {W K d r_x^2, W K s_s^2 / d, h_x, d_x, h_y, d_y, W K r_x s_s, dx/dy} (W = w_i w_m,
// K = dx dy dsig / 8, r_x = 2/dx, s_s = 2/dsig), [c][i][m] with c = ex Ny + ey
constexpr int COLGEO3_N = 8;

// ---- operator --------------------------------------------------------------------------
// 2D: one workgroup per element column; y gets lines 0..P-1 of each column (and line P of
// the last column), S[(ex+1) * nzn + iz] the column's contribution to its right line.
// Full (A x)[g] = y[g] + S[(ix/P) nzn + iz] when ix % P == 0 (S rows 0 and Nx stay zero).
size_t apply2d_smem(int P, int Nz, bool dbl);   // LDS bytes per element column
int apply2d_cpb(int P, int Nx, int Nz, bool dbl);  // element columns per workgroup
// Device layout of the 2D operator's geometric factors: per element column, thread t owns the
// K = 3 (P+1) values (f, j), padded to Kp (a multiple of half a 16-byte chunk); NC full chunks
// of W = 16 / sizeof(TG) values ([c][t][W]), then a half chunk ([t][REM]) if REM > 0; columns
// are cstride values apart.
struct GLayout {
  int W, Kp, NC, REM;
  size_t cstride;
};
// Algorithmic-byte accounting (benchmark hook): while enabled, every launch wrapper of the solve
// path adds the bytes its kernel has to move at the least (each array it reads or writes once at
// its logical size, factors in their storage precision).  acct_enable(true) clears the total.
void acct_enable(bool on);
void acct_add(double bytes);
double acct_total(long* launches);
GLayout g2d_layout(int P, int Nz, size_t tgsize);
hipError_t apply2d(int P, bool dbl, GType gt, const void* x, void* y, void* S, const void* G,
                   int Nx, int Nz, int masked, hipStream_t st);
// 2D operator on elements of order PX along x and PZ along sigma (semi.hip): same output
// format as apply2d with P = PX (lines 0..PX-1 to y, line PX to S of the right neighbour);
// G in the layout [ex][field][ez][i][j] (j fastest, i < PX+1, j < PZ+1); Dx, Dz the row-major
// FP64 differentiation matrices.  apply2r_fits: the column fits one workgroup
// ((PX+1)(PZ+1) Nz <= 1024 threads, 64 KB of LDS).
bool apply2r_fits(int PX, int PZ, int Nz, bool dbl);
// nf = 4: a fourth field G_sr (layout [ex][field][ez][i][j] with four fields) for operators that
// are not symmetric (the mixed-stage form of two stage geometries); nf = 3: G_sr = G_rs
hipError_t apply2r(int PX, int PZ, bool dbl, GType gt, const void* x, void* y, void* S,
                   const void* G, const double* Dx, const double* Dz, int Nx, int Nz, int masked,
                   hipStream_t st, int nf = 3);
// the same, plus each workgroup's part of x . (A x) in dotp[0 .. apply2d_blocks) (P <= 8)
hipError_t apply2d_dot(int P, bool dbl, GType gt, const void* x, void* y, void* S, const void* G,
                       int Nx, int Nz, int masked, double* dotp, hipStream_t st);
int apply2d_blocks(int P, int Nx, int Nz, bool dbl);
// 2D smoother step fused with the operator (P <= 8):  r = b - A xi;  dn = cr dinv r (+ cd d when
// cd != 0);  d = dn (store_d);  xo = xi + dn, all nodes complete; xi and xo must differ.
// cheb2d_cpb returns 0 when the fused form does not fit this mesh (then use apply2d and
// smooth_update).
int cheb2d_cpb(int P, int Nx, int Nz, bool dbl);
hipError_t cheb2d(int P, bool dbl, GType gt, const void* xi, void* xo, void* d, const void* b,
                  const void* dinv, const void* G, int Nx, int Nz, int masked, double cd,
                  double cr, int store_d, hipStream_t st);
// the first two steps of a pre-smoothing from x = 0 in one fused kernel (where cheb2d_cpb > 0):
// x1 = d1 = cr0 dinv b; r = b - A x1; dn = cr dinv r (+ cd d1); d = dn (store_d); x = x1 + dn.
// r64 (optional): FP64 right-hand side, rounded into b.  x, d, b written in place.
hipError_t cheb2d_first(int P, bool dbl, GType gt, void* x, void* d, void* b, const double* r64,
                        const void* dinv, const void* G, int Nx, int Nz, int masked, double cr0,
                        double cd, double cr, int store_d, hipStream_t st);
int cheb2d_blocks(int P, int Nx, int Nz, bool dbl);  // workgroups of the fused kernels (0: none)
// Element-local corrections of the learned stage, line-major per element column: value (i, j)
// of element (ex, ez) at [((ex (P+1) + i) Nz + ez) (P+1) + j], so that the values along a
// vertical node line of a column are contiguous.
__host__ __device__ inline long ce_index(int ex, int i, int ez, int j, int Nz, int NP) {
  return (((long)ex * NP + i) * Nz + ez) * NP + j;
}
// learned stage (2D, where cheb2d_cpb > 0): c = average of the element corrections CE (layout
// of ce_index) at every node (0 on the Dirichlet surface when masked), q = A c complete, and
// each workgroup's part of c . q in dotp[0 .. cheb2d_blocks)
hipError_t stagecq2d(int P, bool dbl, GType gt, const float* CE, void* c, void* q, const void* G,
                     int Nx, int Nz, int masked, double* dotp, hipStream_t st);
// additive Schwarz sweep tail (2D, P <= 8): z_e = Ainv_e R_e r for every element (Ainv
// [E][(P+1)^2][(P+1)^2], symmetric, element e = ex Nz + ez; z in the layout of ce_index), then
// x = (set ? 0 : x) + W sum_e R_e^T z_e (W: one over the number of elements holding a node); the
// Dirichlet surface is left alone (set: zeroed) when masked
hipError_t asm_sweep(int P, bool dbl, const void* r, const void* Ainv, void* z, void* x, int Nx,
                     int Nz, int masked, int set, hipStream_t st);
// additive Schwarz sweep tail over box subdomains (2D with overlap, 3D): the subdomain of
// element e = (ex Ny + ey) Nz + ez (2D: Ny = 1, nyn = 1) is its node index box widened by ov
// layers per side, clipped to the grid.  z_e = Ainv_e R_e (r - y) (y optional: A x, complete),
// then x = (set ? 0 : x) + W sum_e R_e^T z_e; the Dirichlet surface is left alone (set: zeroed)
// when masked.  Ainv: [E][nmax * nmax], subdomain e's symmetric n_e x n_e inverse at its start;
// z: [E][nmax].  ainv_vals = sum_e n_e^2 and z_vals = sum_e n_e count the traffic only.
constexpr int ASM_BOX_NMAX = 4096;
struct AsmBox {
  int Nx = 1, Ny = 1, Nz = 1, P = 1, ov = 0, nmax = 0;
  unsigned nxn = 1, nyn = 1, nzn = 1;
  double ainv_vals = 0.0, z_vals = 0.0;
};
hipError_t asm_box_sweep(const AsmBox& bx, bool dbl, const void* r, const void* y,
                         const void* Ainv, void* z, void* x, int masked, int set, hipStream_t st);
// residual r = b - A x, complete at every node (2D); fused with the operator where cheb2d_cpb
// allows, else apply2d into the scratch y, S and an element-wise pass.  r must differ from x.
hipError_t resid2d(int P, bool dbl, GType gt, const void* x, void* r, const void* b,
                   const void* G, int Nx, int Nz, int masked, void* y, void* S, hipStream_t st);
// 3D operator (element columns (ex, ey) of Nz hexahedra, P <= 8): y = A x complete on return
// (side buffers Sx, Sy, Sxy are full-size scratch vectors); G in the layout of g3d_layout.
size_t apply3d_smem(int P, int Nz, bool dbl);
GLayout g3d_layout(int P, int Nz, size_t tgsize);
// With st3.b set the launch is a smoother step instead: with r = b - A x at every node,
// dn = cr dinv r (+ cd d when cd != 0), d = dn (store_d), x += dn, in place (x is read by other
// columns only on the shared planes, which are finished by the face fix-up after every column
// has read them); y then holds only the partial sums of the shared-plane lines.
struct Step3 {
  const void* b = nullptr;
  const void* dinv = nullptr;
  void* d = nullptr;
  double cd = 0.0, cr = 0.0;
  int store_d = 0;
};
hipError_t apply3d(int P, bool dbl, GType gt, const void* x, void* y, void* Sx, void* Sy,
                   void* Sxy, const void* G, int Nx, int Ny, int Nz, int masked, hipStream_t st,
                   Step3 st3 = Step3());
// 3D levels of order 1 (p1.hip): y = A x with the assembled 27-point stencil coef [27][N]
// (offset k = (dx+1) 9 + (dy+1) 3 + (dz+1), zero outside the grid and towards masked nodes,
// identity rows on them), complete at every node; with st3.b the smoother step of apply3d,
// written out of place into xo (xo != x)
hipError_t stencil3d(bool dbl, const void* x, void* y, const void* coef, unsigned nxn,
                     unsigned nyn, unsigned nzn, hipStream_t st, Step3 st3 = Step3(),
                     void* xo = nullptr);
// one 1D operator (CSR rows over the output index) along the middle axis of [outer][n][inner]
// arrays; in2 (optional) is subtracted from in; mask_nzn > 0 zeroes every mask_nzn-th output
// (the Dirichlet surface rows when inner is the vertical axis)
// nnz = entries of the CSR operator (nout rows).  The same operator as bands: band holds one
// int4 {first column, length, offset into wband, 0} per row, wband the weights dense over each
// band; bandmax = the longest band (null band or bandmax < 0: not available)
hipError_t axis_apply(int in_dbl, int out_dbl, const void* in, const void* in2, void* out,
                      int accumulate, unsigned n_outer, unsigned nin, unsigned nout,
                      unsigned n_inner, const int* rowptr, const int* cols, const double* w,
                      unsigned nnz, const int* band, const double* wband, int bandmax,
                      unsigned mask_nzn, hipStream_t st);
hipError_t dense_gemv(const double* Ainv, const double* b, double* x, int n, hipStream_t st);
// surface update (3D, fine level, FP64): factors G (g3d_layout) and lumped mass from the fine
// column samples hf, ef ((Nx P + 1) x (Ny P + 1), y fastest); r, w: GLL nodes and weights
hipError_t geom3d(int P, const double* hf, const double* ef, const double* r, const double* w,
                  double* G, int Nx, int Ny, int Nz, double dx, double dy, hipStream_t st);
// the G_COL64 records of the 3D fine level from its column samples (layout above)
hipError_t colrec3d(int P, const double* hf, const double* ef, double* CG, int Nx, int Ny, int Nz,
                    double dx, double dy, hipStream_t st);
hipError_t mass3d(const double* hf, const double* ef, const double* Wx, const double* Wy,
                  const double* Wz, double* mass, unsigned nyn, unsigned nzn, size_t N,
                  double scale, hipStream_t st);

// ---- stage loop pieces (FP64) ---------------------------------------------------------------
// w[s] = d phi / dz at the surface node of vertical node line s (s < ns): (2/dsig) times the
// top element's GLL derivative of order P at its top node, over the depth dsurf[s]
hipError_t surface_dz(int P, const double* phi, const double* dsurf, double* w, size_t ns,
                      unsigned nzn, double dsig, hipStream_t st);
// K = a K + dt F; y += b K over n values
hipError_t lserk_update(const double* F, double* K, double* y, size_t n, double a, double dt,
                        double b, hipStream_t st);

// ---- element-wise kernels in precision T (dbl selects double, else float) ----------------
// d = cd d + cr dinv r,  x = (from_zero ? 0 : x) + d,  r = b - (from_zero ? 0 : Ax)
// smoother step x += d, d = cd d + cr dinv r; the residual r by mode:
enum { SU_AX = 0,      // r = b - (y + S), the column output of the preceding apply
       SU_ZERO = 1,    // x = 0 on entry: r = b, and x = d
       SU_RESID = 2 }; // b holds the residual of the current x
hipError_t smooth_update(bool dbl, void* x, void* d, const void* b, const void* dinv,
                         const void* y, const void* S, unsigned N, unsigned nzn, unsigned P,
                         double cd, double cr, int mode, int store_d, hipStream_t st);
// first step of a V-cycle's pre-smoothing from x = 0, right-hand side taken from FP64 r64
// (stored rounded into b): d = cr dinv b, x = d
hipError_t smooth_first64(bool dbl, void* x, void* d, void* b, const double* r64,
                          const void* dinv, unsigned N, double cr, int store_d, hipStream_t st);
// out = (Ax)[g] with the side-buffer fix (test hook / Lanczos), widened to double if out64
hipError_t fix_ax(bool dbl, const void* y, const void* S, void* out, int out64, unsigned N,
                  unsigned nzn, unsigned P, hipStream_t st);
// casts between FP64 and the inner precision
hipError_t cast_to(bool dbl_dst, const double* src, void* dst, unsigned N, hipStream_t st);
hipError_t cast_from(bool dbl_src, const void* src, double* dst, unsigned N, hipStream_t st);
hipError_t fill(bool dbl, void* p, double v, size_t n, hipStream_t st);

// ---- p-transfers (2D, pull form, one workgroup per element column) ------------------------
// The learned stage's step folded into the transfers around the coarse correction (fine level,
// stage before the restriction): alpha = c.r / c.q from its partial sums (0 if not finite and
// positive; the restriction counts the rejection in skips[0]); the restriction takes the fine
// residual b - alpha q, the prolongation adds alpha c with the correction.  Null q / c: no fold.
struct StageFold {
  const void* q = nullptr;
  const void* c = nullptr;
  const double* pcr = nullptr;
  int ncr = 0;
  const double* pcq = nullptr;
  int ncq = 0;
  int* skips = nullptr;
};
// rc = P^T r with r = b - Ax (use_ax), r = b - alpha q (f.q) or r = b; coarse Dirichlet rows
// zero when masked.
size_t restrict2d_smem(int Pf, int Pc, int Nz, bool dbl);
hipError_t restrict2d(bool dbl, bool dbl_c, const void* b, const void* y, const void* S,
                      int use_ax, void* rc, const double* J, int Nx, int Nz, int Pf, int Pc,
                      int masked, hipStream_t st, StageFold f = StageFold());
// xf += P ec (+ alpha c with f.c)
size_t prolong2d_smem(int Pf, int Pc, int Nz, bool dbl);
hipError_t prolong2d(bool dbl, bool dbl_c, const void* ec, void* xf, const double* J, int Nx,
                     int Nz, int Pf, int Pc, hipStream_t st, StageFold f = StageFold());

// ---- a coarse level's smoothing sequence in one kernel (2D) --------------------------------
// step s of the sequence: d = cd[s] d + cr[s] dinv (b - A x); x += d.  PRE: x = 0 on entry (the
// first step needs no operator), then the residual is restricted to the next level: rc = R r
// (top node zero when masked), x written to xo.  POST: x_in + P ec (the next level's correction)
// is smoothed and written to xo (xo != x_in).  b, dinv, G: the level's; J: its prolongation
// matrix from the next level; TC of rc / ec: FP64 when dbl_c.  The plan (coarse2d_plan) fixes
// the window; W = 0: the level does not fit, use the per-step kernels.
constexpr int CO_MAXS = 8;
struct CoarseSeq {
  int ns = 0;
  double cd[CO_MAXS] = {0}, cr[CO_MAXS] = {0};
};
struct CoarsePlan {
  int W = 0, HL = 0, nslot = 0;
  size_t smem = 0;
};
// What a coarse-level launch does besides its smoothing steps: CO_FROM_X (pre family) start
// from x instead of x = 0; CO_RESTRICT (pre family) end with the residual and its restriction
// into rc; CO_PROLONG (post family) start by adding the prolongation of ec to x.  din (optional)
// holds the Chebyshev direction d at the start (a sequence continued from an earlier launch);
// dout (optional) receives d of the owned columns at the end.  A sequence too long for one
// window runs as two launches: the first writes x and d, the second continues from them.
constexpr int CO_FROM_X = 1, CO_RESTRICT = 2, CO_PROLONG = 4;
struct CoarseIO {
  const void* din = nullptr;
  void* dout = nullptr;
  int flags = 0;
};
// window of a launch with `applies` operator applies and the given CO_RESTRICT / CO_PROLONG
CoarsePlan coarse2d_plan(int P, int PC, int Nz, bool dbl, int flags, int applies);
bool coarse2d_supported(int P, int PC);
hipError_t coarse2d(bool pre, const CoarsePlan& pl, int P, int PC, bool dbl, GType gt, bool dbl_c,
                    const void* x, void* xo, const void* b, const void* dinv, const void* G,
                    const void* ec, void* rc, const double* J, int Nx, int Nz, int masked,
                    const CoarseSeq& sq, hipStream_t st, CoarseIO io);

// ---- exact coarse solve (block cyclic reduction, FP64, in place on b, result in x) ---------
// unknown r of block blk sits at blk * bstride + r + r / nzf (nzf = free nodes per line)
hipError_t bcr_fwd(double* b, const double* F, int n, int stride, int neven, int bstride,
                   int nzf, int nb, hipStream_t st);
hipError_t bcr_bwd(const double* b, double* x, const double* Bk, int n, int stride, int nodd,
                   int bstride, int nzf, int nb, hipStream_t st);
hipError_t bcr_dense(const double* Ainv, const double* b, double* x, int nd, int nb, int stride,
                     int bstride, int nzf, hipStream_t st);
// all reduction levels in one launch each way: fwd reads b and writes the reduced right-hand
// side to bred (every block); the dense step then solves the blocks that are multiples of
// 2^nl from bred into x, and bwd fills in the remaining blocks of x.  LDS per workgroup:
// bcr_{fwd,bwd}_all_smem (the host falls back to the per-level kernels beyond its limit).
constexpr int BCR_MAXL = 16;
struct BcrLevels {
  int nl = 0;
  long long offM[BCR_MAXL] = {0};
  long long offB[BCR_MAXL] = {0};
};
size_t bcr_fwd_all_smem(int nl, int nb);
size_t bcr_bwd_all_smem(int nl, int nb);
hipError_t bcr_fwd_all(const double* b, double* bred, const double* F, const BcrLevels& lv,
                       int nblocks, int bstride, int nzf, int nb, hipStream_t st);
hipError_t bcr_bwd_all(const double* bred, double* x, const double* Bk, const BcrLevels& lv,
                       int nblocks, int bstride, int nzf, int nb, hipStream_t st);

// ---- FP64 outer-loop kernels (deterministic two-stage reductions over NRED partials) -------
// FPCG direction step fused with the FP64 operator (2D where the fused layout fits with at most
// NRED workgroups): q = A (z + beta p) complete (first: q = A z), partials of p.q into ppq_new
// (entries beyond the workgroup count are left alone: keep them zero), beta into *beta_out;
// then update_xrp: p = z + beta p, x += alpha p, r -= alpha q with alpha = sum(prz_new) /
// sum(ppq_new), r.r partials, and the partial sets moved to prz_old / ppq_old.
bool fpcg2d_fits(int P, int Nx, int Nz);
// col: G holds G_COL64 column data instead of stored FP64 factors
hipError_t fpcg2d(int P, const double* z, const double* p, double* q, const double* G, int Nx,
                  int Nz, int masked, const double* prz_old, const double* ppq_old,
                  const double* pzq, int first, double* ppq_new, double* beta_out,
                  hipStream_t st, int col = 0);
hipError_t update_xrp(double* x, double* r, double* p, const double* z, const double* q,
                      const double* beta, int first, const double* prz_new,
                      const double* ppq_new, double* prz_old, double* ppq_old, double* prr,
                      unsigned N, hipStream_t st);
// r = b - Ax (with fix); partial sums of r.r into prr and (if pbb) b.b into pbb
hipError_t resid64(const double* b, const double* y, const double* S, double* r, double* prr,
                   double* pbb, unsigned N, unsigned nzn, unsigned P, hipStream_t st);
// q = Ax (fix); ppq = partial p.q; if rz_from/rz_to copy NRED partials (done by block 0)
hipError_t fixdot64(const double* y, const double* S, double* q, const double* p, double* ppq,
                    const double* rz_from, double* rz_to, unsigned N, unsigned nzn, unsigned P,
                    hipStream_t st);
// alpha = sum(prz)/sum(ppq); x += alpha p; r -= alpha q; prr = partial r.r
hipError_t update_xr(double* x, double* r, const double* p, const double* q, const double* prz,
                     const double* ppq, double* prr, unsigned N, hipStream_t st);
// out[k] = sum of partial set k (k < nsets), one block
hipError_t reduce_sets(const double* parts, int nsets, double* out, hipStream_t st);
// z = (double) x0; partial z.q (if q) and r.z
hipError_t castdot(bool dbl_src, const void* x0, double* z, const double* q, const double* r,
                   double* pzq, double* prz, unsigned N, hipStream_t st);
// p = z (first) or p = z + beta p with beta = -alpha sum(pzq)/sum(prz_old),
// alpha = sum(prz_old)/sum(ppq)
hipError_t pupdate(double* p, const double* z, const double* prz_old, const double* ppq,
                   const double* pzq, int first, unsigned N, hipStream_t st);
hipError_t axpy64(double* x, const double* z, double a, unsigned N, hipStream_t st);
// x[top nodes] = src[top nodes]
hipError_t copy_top(double* x, const double* src, unsigned ncols, unsigned nzn, hipStream_t st);
// partial dot of two vectors in precision T (double partials)
hipError_t dot_partial(bool dbl, const void* a, const void* b, double* part, unsigned N,
                       hipStream_t st);
// elementwise: out = a * s (T)
hipError_t vmul(bool dbl, const void* a, const void* s, void* out, unsigned N, hipStream_t st);
// out = alpha a + beta b (T), out may alias a or b
hipError_t vaxpby(bool dbl, double alpha, const void* a, double beta, const void* b, void* out,
                  unsigned N, hipStream_t st);

// ---- right-hand side assembly -------------------------------------------------------------
hipError_t rhs_mass(const double* mass, const double* f, double* rhs, unsigned N, hipStream_t st);
hipError_t rhs_face(const long long* idx, const double* w, const double* g, double* rhs,
                    unsigned n, hipStream_t st);
// rhs -= Ax (fix) on non-top rows; rhs = gD on top rows (gD may be NULL for 0)
hipError_t rhs_lift(double* rhs, const double* y, const double* S, const double* gD,
                    unsigned N, unsigned nzn, unsigned P, hipStream_t st);
hipError_t scatter_top(double* v, const double* gD, unsigned ncols, unsigned nzn, hipStream_t st);

}  // namespace semk
