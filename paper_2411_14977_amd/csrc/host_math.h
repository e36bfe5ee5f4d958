// Host-side FP64 set-up math of the spectral-element solver: GLL rules, differentiation and
// interpolation matrices, sigma-mapped geometric factors, assembled diagonals and the exact
// block-cyclic-reduction factorisation of the P = 1 coarse operator.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace semh {

// ---- 1D spectral pieces (paper Sec. 4.3) -------------------------------------------------
// GLL nodes (ascending) and weights of order P: end points plus the roots of P_P'.
void gll_rule(int P, std::vector<double>& r, std::vector<double>& w);
// Lagrange differentiation matrix at the GLL nodes, row-major D[i*(P+1)+k] = l_k'(r_i).
std::vector<double> diff_matrix(int P, const std::vector<double>& r);
// Lagrange basis of the source nodes rs evaluated at target points rt:
// M[a*(ns)+k] = l_k(rt[a]) (barycentric form; exact delta rows where points coincide).
std::vector<double> interp_matrix(const std::vector<double>& rs, const std::vector<double>& rt);

// ---- one level of the hierarchy ------------------------------------------------------------
struct LevelGeom {
  int dim = 2, P = 1, NP = 2;
  // 2D: order along sigma (differs from P, the order along x, on semi-coarsened levels); local
  // node (i, j) is i*NPz + j.  3D: equal to P.
  int Pz = 1, NPz = 2;
  int Nx = 1, Ny = 1, Nz = 1;
  double Lx = 1, Ly = 1;
  int nxn = 0, nyn = 1, nzn = 0;   // nodes per direction
  size_t N = 0;                    // assembled nodes
  size_t E = 0;                    // elements
  std::vector<double> r, w, D;     // GLL nodes, weights, differentiation matrix (x; 3D all)
  std::vector<double> rz, wz, Dz;  // the same along sigma (order Pz)
  // geometric factors, natural layout [field][e][local node] with local node
  // 2D (i*NP + j), 3D ((i*NP + m)*NP + j); fields 2D: rr, rs, ss; 3D: rr, tt, rs, ts, ss
  int nfields = 3;
  std::vector<double> G;
  std::vector<double> mass;        // [e][local] lumped mass w |J|
  std::vector<double> X, Y, Z;     // global node coordinates (N)
  // Neumann faces: node index + surface-quadrature weight, faces in the ABI packing order
  std::vector<std::vector<int64_t>> face_idx;
  std::vector<std::vector<double>> face_w;
  std::vector<double> col_h, col_eta;  // element-local column data (diagnostics)
};

// Build level geometry of order P from h, eta sampled at the fine horizontal GLL nodes of
// order Pf (2D: Nx*Pf+1 values; 3D: (Nx*Pf+1)*(Ny*Pf+1), y fastest).  Pz (2D only): order
// along sigma, default P.
void build_level(LevelGeom& L, int dim, int Nx, int Ny, int Nz, int P, int Pf, double Lx,
                 double Ly, const double* h_fine, const double* eta_fine, int Pz = -1);

// Global node of local node l (2D i*NPz + j; 3D (i*NP + m)*NP + j) of element e.
size_t local_to_global(const LevelGeom& L, size_t e, int l);

// Assembled diagonal of the masked operator from (possibly rounded) factors Gr (same layout
// as L.G).  Dirichlet rows get 1 when masked.
std::vector<double> assembled_diag(const LevelGeom& L, const std::vector<double>& Gr, bool masked);

// Dense element stiffness of element e, size NL x NL (NL = NP^dim), from factors Gr.
void element_matrix(const LevelGeom& L, const std::vector<double>& Gr, size_t e, double* Ae);

// Dense inverse by Gauss-Jordan elimination with partial pivoting (false if singular).
bool dense_inverse_public(int n, const double* A, double* Ainv);

// Round to bfloat16 (round to nearest even) and back.
double bf16_round(double v);
uint16_t bf16_bits(float f);

// ---- exact P = 1 coarse solve: block cyclic reduction ----------------------------------------
// The masked coarse operator is block tridiagonal over the x-lines (2D: blocks of the Nz free
// nodes of one vertical line; 3D: blocks of one (y, z) plane of free nodes).  The factors are
// stored level by level for a device solve that works in place on the level vector.
struct BcrPlan {
  int nb = 0;          // unknowns per block
  int bstride = 0;     // distance between consecutive blocks in the level vector
  int nblocks = 0;     // blocks at level 0
  struct Lev { int n, stride; size_t offM, offB; int neven, nodd; };
  std::vector<Lev> levs;       // reduction levels (n > 1)
  std::vector<double> fwd;     // per level: neven x {Mm, Mp} nb x nb, column-major
  std::vector<double> bwd;     // per level: nodd x {DO, DL, DU} nb x nb, column-major
  std::vector<double> last;    // inverse of the final block, nb x nb (unused when dense)
  // the reduction stops once at most `dense_max` blocks remain; the remaining reduced system
  // (dense_n blocks, spaced dense_stride apart at level 0) is solved with its explicit inverse
  int dense_n = 0, dense_stride = 1;
  std::vector<double> dense;   // (dense_n nb) x (dense_n nb), row-major
  // map from block-row (b, r) to the level-vector index: b * bstride + rowmap[r]
  std::vector<int> rowmap;
};
bool build_bcr(const LevelGeom& L, const std::vector<double>& Gr, BcrPlan& plan, char* err,
               size_t errlen, int dense_max = 65);

// Counter-based SplitMix64 uniform in [-1, 1) (Steele, Lea, Flood 2014), element i of seed.
double splitmix64_uniform(uint64_t seed, uint64_t i);

}  // namespace semh
