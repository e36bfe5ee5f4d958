// C ABI, set-up and solver driver of the MI355X spectral-element pressure-Poisson solver.
//
// Set-up (host FP64, then upload): GLL rules and matrices per level, sigma-mapped geometric
// factors (paper Sec. 2.2 eq. sigtrans / eq. 1_Scoef, Sec. 4.3), assembled inverse diagonals,
// lambda_hat of D^{-1}A by Lanczos on the device, and the exact block-cyclic-reduction factors of
// the P = 1 coarse operator.  Solve (device): V-cycles of Sec. 5 inside FP64 flexible CG or
// defect correction (Sec. 5.4); each outer iteration is one captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <chrono>
#include <climits>
#include <utility>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/sem.h"
#include "host_math.h"
#include "kernels.h"
#include "krylov.h"
#include "mlp.h"

namespace {

using semk::GType;

struct DLevel {
  int P = 1, NP = 2, Nx = 1, Ny = 1, Nz = 1, nxn = 0, nyn = 1, nzn = 0;
  // 2D: order along sigma (P is the order along x); rect: the two differ, and the level runs
  // the operator for such elements (Dx, Dz: its FP64 differentiation matrices)
  int Pz = 1;
  bool rect = false;
  double *Dx = nullptr, *Dz = nullptr;
  // 2D transfers from the next coarser level that change one direction only (axis 0: x,
  // 2: sigma; -1: both directions, by the equal-order transfer kernels)
  int axis = -1;
  unsigned N = 0;
  bool dbl = true;            // vector/compute type of this level (coarsest is always FP64)
  GType gt = semk::G_F64;
  semh::LevelGeom geo;
  void* G = nullptr;          // factors in storage precision, device column layout
  void* dinv = nullptr;       // inverse assembled diagonal
  double* J = nullptr;        // prolongation from the next coarser level, (P+1) x (Pc+1)
  void *x = nullptr, *b = nullptr, *d = nullptr, *y = nullptr, *S = nullptr;
  // 2D smoothed levels where the fused smoother step fits: the second solution vector; each
  // fused step reads x and writes xalt, then the two swap (x is always the current iterate)
  void* xalt = nullptr;
  // 2D coarse levels: the pre- and post-smoothing sequences as one kernel each (W = 0: no)
  semk::CoarsePlan cpre, cpost;
  // sequences too long for one window: the second launch's window and the steps in the first
  // (0: one launch)
  semk::CoarsePlan cpre2, cpost2;
  int cpre_k1 = 0, cpost_k1 = 0;
  // Schwarz smoother: inverses of the element blocks [E][n][n] and the element results [E][n];
  // with asm_box, of the box subdomains (overlap or 3D) [E][nmax^2] and [E][nmax]
  void *Ainv_s = nullptr, *Zs = nullptr;
  bool asm_box = false;
  semk::AsmBox abox;
  // 3D levels of order 1 above the coarsest: the assembled 27-point stencil [27][N] in the
  // level's precision and the second solution vector of its out-of-place smoother step
  void *st27 = nullptr, *x3alt = nullptr;
  size_t nS = 0;
  double lam = 0.0;
  // 3D: side buffers of the operator (completed into y by the face fix-up; S stays null) and
  // the 1D transfer operators from the next coarser level (x, y, z; P coarse->fine, R = P^T)
  void *Sx = nullptr, *Sy = nullptr, *Sxy = nullptr;
  struct Op1 {
    int* rp = nullptr;
    int* ci = nullptr;
    double* w = nullptr;
    unsigned nnz = 0;
    int* band = nullptr;  // per row {first column, length, offset into wband, 0}
    double* wband = nullptr;
    int bandmax = 0;  // longest band
  } P1[3], R1[3];
};

struct Ctx {
  sem_mesh_desc desc{};
  int dim = 2, Nx = 1, Ny = 1, Nz = 1, masked = 1;
  std::vector<DLevel> lev;
  int prec = SEM_F64;
  hipStream_t st = nullptr;       // internal stream (default priority)
  hipStream_t ust = nullptr;      // caller's stream
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // per-iteration partial sums copied to the host (two alternating slots; slot 2: the initial
  // residual's)
  hipEvent_t ev_it[3] = {nullptr, nullptr, nullptr};
  // fine-level FP64 operator for the outer loop: stored factors (3D, and 2D levels with two
  // orders), or in 2D the column records the operator forms its factors from (G_COL64)
  double* G64 = nullptr;
  double* CG64 = nullptr;
  // stage loop: depth d = h + eta at every surface node (fine samples), the model's right-hand
  // side and Poisson right-hand side buffers, a host copy of a stage's surface
  double* dsurf = nullptr;
  double *wF = nullptr, *wrhs = nullptr;
  std::vector<double> eta_h;
  // mixed-stage outer operator (2D): four FP64 factor fields of two stage geometries in the
  // layout of the two-order operator kernel, and its differentiation matrices
  bool mixed = false;
  double *Gmix = nullptr, *Dmx = nullptr, *Dmz = nullptr;
  bool G64_owned = false;
  double *xo = nullptr, *bo = nullptr, *ro = nullptr, *po = nullptr, *qo = nullptr,
         *zo = nullptr, *yo = nullptr, *So = nullptr, *mass = nullptr;
  double* parts = nullptr;        // partial-sum sets
  double* scal = nullptr;         // device scalars
  double* hscal = nullptr;        // pinned host scalars: three slots of 3 NRED partials + 1
  std::vector<long long*> face_idx;
  std::vector<double*> face_w;
  std::vector<size_t> face_n;
  // 3D: outer side buffers, transfer temporaries, dense inverse of the coarsest level
  double *Sxo = nullptr, *Syo = nullptr, *Sxyo = nullptr;
  double *tA = nullptr, *tB = nullptr;
  double* Ainv = nullptr;
  int nAinv = 0;
  // surface update: fine column samples (host copies; device copies for the 3D kernels)
  std::vector<double> hf_h, ef_h;
  int Pf = 1;
  double len0 = 1.0, len1 = 1.0;
  double *hf_d = nullptr, *ef_d = nullptr, *r_d = nullptr, *w_d = nullptr;
  double *Wx_d = nullptr, *Wy_d = nullptr, *Wz_d = nullptr;
  std::vector<uint8_t> stage_blob;  // the loaded network, to rebuild the stage's geometry
  // coarse solve
  semh::BcrPlan plan;
  double *bcrF = nullptr, *bcrB = nullptr, *bcrLast = nullptr, *bcrDense = nullptr;
  double* bcrRed = nullptr;  // reduced right-hand side of the one-launch reduction
  // GMRES: Arnoldi basis V (m + 1 vectors), preconditioned basis Z (m), reduction partials
  double *kV = nullptr, *kZ = nullptr, *kpart = nullptr, *hkpart = nullptr;
  double* kcoef = nullptr;  // GMRES on the device: h1, h2 [KRY_MAX + 1], ||w||^2, the step's column
  semk::BcrLevels bcrLv;     // its level table (nl = -1: per-level kernels)
  int* rowmap = nullptr;
  // FP64 right-hand side of the next V-cycle, read by the first smoothing step of level 0
  const double* vin64 = nullptr;
  // learned stage (fine level)
  semm::Stage stage;
  bool stage_alloc = false;
  int stage_mode = 1;          // bit 0: after pre-smoothing, bit 1: before post-smoothing
  void *Rbuf = nullptr, *cbuf = nullptr, *yq = nullptr, *Sq = nullptr;
  double* stparts = nullptr;
  std::vector<float> geo_h;    // [E x 4n] geometric features (host)
  std::vector<float> abar_h;   // [E] mean element-matrix diagonal (host)
  float* geo_d = nullptr;
  double* ainv_d = nullptr;    // [E x n x n] inverses of R_e A R_e^T (training targets)
  int* harvest_idx = nullptr;  // [E] elements sampled by sem_learned_harvest
  // graphs
  // iteration graphs (each ends with the copy of its partial sums into host slot 0 or 1)
  hipGraphExec_t g_first = nullptr, g_iter[2] = {nullptr, nullptr}, g_pdc[2] = {nullptr, nullptr};
  bool use_graphs = true;
  std::string err;
  bool sticky = false;
  std::vector<void*> allocs;
  std::unordered_map<const void*, size_t> asize;  // bytes of every allocation in allocs
};

// partial-sum sets; the first double of PS_SKIP holds the learned stage's rejection counter (an
// int), so one copy of sets RR, BB, PQ and that double brings everything the host checks
enum { PS_RR = 0, PS_BB, PS_PQ, PS_SKIP, PS_RZA, PS_RZB, PS_ZQ, PS_TMP, PS_PQ2, PS_NSETS };

struct HipFail {
  hipError_t e;
  const char* what;
};

#define HK(call)                                   \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) throw HipFail{e_, #call}; \
  } while (0)

struct ArgFail {
  std::string msg;
};

void* dalloc(Ctx* c, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) throw HipFail{e, "hipMalloc"};
  c->allocs.push_back(p);
  c->asize[p] = bytes;
  HK(hipMemsetAsync(p, 0, bytes, c->st));
  return p;
}

template <typename T>
T* upload(Ctx* c, const std::vector<T>& h) {
  T* p = (T*)dalloc(c, h.size() * sizeof(T));
  HK(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->st));
  HK(hipStreamSynchronize(c->st));
  return p;
}

size_t esz(bool dbl) { return dbl ? 8 : 4; }

template <typename T>
void* put_vec(Ctx* c, const std::vector<T>& h, void* dst) {
  if (!dst) return upload(c, h);
  HK(hipMemcpy(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return dst;
}

// natural [f][e][i*NP+j] -> device [ex][f][j][ez*NP+i]
template <typename TG, typename Conv>
std::vector<TG> permute_G2d(const semh::LevelGeom& L, const std::vector<double>& G, Conv conv) {
  // device layout of the operator's geometric factors (see semk::g2d_layout): per element
  // column, the 3 NP values (f, j) of each thread t = ez NP + i are split into 16-byte chunks,
  // chunk-major and thread-contiguous within a chunk, so every lane reads them with 16-byte
  // coalesced loads; the column stride is padded to a whole chunk row
  const int NP = L.NP, Nz = L.Nz, Nx = L.Nx;
  const size_t NL = NP * NP, nthr = (size_t)NP * Nz;
  const semk::GLayout lay = semk::g2d_layout(L.P, Nz, sizeof(TG));
  std::vector<TG> out((size_t)Nx * lay.cstride, TG(0));
  for (int ex = 0; ex < Nx; ++ex)
    for (int ez = 0; ez < Nz; ++ez)
      for (int i = 0; i < NP; ++i) {
        const size_t e = (size_t)ex * Nz + ez, t = (size_t)ez * NP + i;
        for (int f = 0; f < 3; ++f)
          for (int j = 0; j < NP; ++j) {
            const int k = f * NP + j;
            const int c = k / lay.W, w = k % lay.W;
            const size_t off = c < lay.NC ? ((size_t)c * nthr + t) * lay.W + w
                                          : (size_t)lay.NC * nthr * lay.W + t * lay.REM + (k - lay.NC * lay.W);
            out[(size_t)ex * lay.cstride + off] = conv(G[f * L.E * NL + e * NL + i * NP + j]);
          }
      }
  return out;
}

// device factors of a 2D level in its operator's layout: the chunked column layout of the
// equal-order kernels, or [ex][field][ez][i][j] for elements with different orders
template <typename TG, typename Conv>
std::vector<TG> layout_G2(const semh::LevelGeom& L, const std::vector<double>& G, Conv conv) {
  if (L.Pz == L.P) return permute_G2d<TG>(L, G, conv);
  const size_t nthr = (size_t)L.NP * L.NPz * L.Nz, E = L.E, nloc = (size_t)L.NP * L.NPz;
  std::vector<TG> out(3 * E * nloc);
  for (int ex = 0; ex < L.Nx; ++ex)
    for (int f = 0; f < 3; ++f)
      for (size_t t = 0; t < nthr; ++t)
        out[((size_t)ex * 3 + f) * nthr + t] = conv(G[f * E * nloc + (size_t)ex * nthr + t]);
  return out;
}

// G_COL64 records of a 2D equal-order level: per element column ex and horizontal node i,
// {w_i d dsig/dx, w_i dx/(dsig d), h_x, d_x} with d = h + eta and the x-derivatives by spectral
// differentiation within the element (the quantities the stored factors are built from)
std::vector<double> column_records(const semh::LevelGeom& L) {
  const int NP = L.NP;
  const double dx = L.Lx / L.Nx, dsig = 1.0 / L.Nz;
  std::vector<double> out((size_t)L.Nx * NP * semk::COLGEO_N);
  for (int ex = 0; ex < L.Nx; ++ex)
    for (int i = 0; i < NP; ++i) {
      double a = 0, b = 0;
      for (int k = 0; k < NP; ++k) {
        const double hk = L.col_h[(size_t)ex * NP + k], ek = L.col_eta[(size_t)ex * NP + k];
        a += L.D[i * NP + k] * hk;
        b += L.D[i * NP + k] * (hk + ek);
      }
      const double d = L.col_h[(size_t)ex * NP + i] + L.col_eta[(size_t)ex * NP + i];
      double* r = &out[((size_t)ex * NP + i) * semk::COLGEO_N];
      r[0] = L.w[i] * d * dsig / dx;
      r[1] = L.w[i] * dx / (dsig * d);
      r[2] = 2.0 / dx * a;
      r[3] = 2.0 / dx * b;
    }
  return out;
}

// G_COL64 records of a 3D level: per element column (ex, ey) and horizontal node (i, m),
// {W K d r_x^2, W K s_s^2 / d, h_x, d_x, h_y, d_y, W K r_x s_s, dx/dy} (W = w_i w_m,
// K = dx dy dsig / 8, r_x = 2/dx, s_s = 2/dsig), slopes by spectral differentiation of the
// element-local h, d (the quantities the stored factors are built from)
std::vector<double> column_records3d(const semh::LevelGeom& L) {
  const int NP = L.NP, NL = NP * NP;
  const double dx = L.Lx / L.Nx, dy = L.Ly / L.Ny, dsig = 1.0 / L.Nz;
  const double rx = 2.0 / dx, ty = 2.0 / dy, ss = 2.0 / dsig, K = dx * dy * dsig / 8.0;
  std::vector<double> out((size_t)L.Nx * L.Ny * NL * semk::COLGEO3_N);
  for (size_t col = 0; col < (size_t)L.Nx * L.Ny; ++col) {
    const double* h = &L.col_h[col * NL];
    const double* et = &L.col_eta[col * NL];
    for (int i = 0; i < NP; ++i)
      for (int m = 0; m < NP; ++m) {
        double a = 0, b = 0, cc = 0, e2 = 0;
        for (int k = 0; k < NP; ++k) {
          a += L.D[i * NP + k] * h[k * NP + m];
          b += L.D[i * NP + k] * (h[k * NP + m] + et[k * NP + m]);
          cc += L.D[m * NP + k] * h[i * NP + k];
          e2 += L.D[m * NP + k] * (h[i * NP + k] + et[i * NP + k]);
        }
        const double d = h[i * NP + m] + et[i * NP + m], W = L.w[i] * L.w[m];
        double* r = &out[(col * NL + i * NP + m) * semk::COLGEO3_N];
        r[0] = W * K * d * rx * rx;
        r[1] = W * K * ss * ss / d;
        r[2] = rx * a;
        r[3] = rx * b;
        r[4] = ty * cc;
        r[5] = ty * e2;
        r[6] = W * K * rx * ss;
        r[7] = dx / dy;
      }
  }
  return out;
}

// factor data of a 2D level: column records where its operator forms the factors itself
// (FP64 levels and SEM_F32_GCOL, equal orders), else stored factors in the inner precision
semk::GType level_gtype(const Ctx* c, const DLevel& L) {
  if (L.dbl) return L.rect ? semk::G_F64 : semk::G_COL64;
  if (c->prec == SEM_F32_GBF16) return semk::G_BF16;
  if (c->prec == SEM_F32_GCOL && !L.rect) return semk::G_COL64;
  return semk::G_F32;
}

// the level's factor data for geometry geo, uploaded into dst (null: a new allocation)
void* put_factors(Ctx* c, const DLevel& L, const semh::LevelGeom& geo, void* dst);

void* put_factors(Ctx* c, const DLevel& L, const semh::LevelGeom& geo, void* dst) {
  switch (L.gt) {
    case semk::G_COL64: return put_vec(c, column_records(geo), dst);
    case semk::G_F64: return put_vec(c, layout_G2<double>(geo, geo.G, [](double v) { return v; }), dst);
    case semk::G_F32:
      return put_vec(c, layout_G2<float>(geo, geo.G, [](double v) { return (float)v; }), dst);
    default:
      return put_vec(c, layout_G2<uint16_t>(geo, geo.G,
                                            [](double v) { return semh::bf16_bits((float)v); }),
                     dst);
  }
}

template <typename TG, typename Conv>
std::vector<TG> permute_G3d(const semh::LevelGeom& L, Conv conv);

// the same for a 3D level
void* put_factors3d(Ctx* c, const DLevel& L, const semh::LevelGeom& geo, void* dst) {
  switch (L.gt) {
    case semk::G_COL64: return put_vec(c, column_records3d(geo), dst);
    case semk::G_F64: return put_vec(c, permute_G3d<double>(geo, [](double v) { return v; }), dst);
    case semk::G_F32:
      return put_vec(c, permute_G3d<float>(geo, [](double v) { return (float)v; }), dst);
    default:
      return put_vec(c, permute_G3d<uint16_t>(geo, [](double v) { return semh::bf16_bits((float)v); }),
                     dst);
  }
}

// run f(lo, hi) over [0, n) on up to 16 host threads (set-up work only)
// grain: fewest items per thread (heavy items: a small grain spreads them over more threads)
void parallel_ranges(size_t n, const std::function<void(size_t, size_t)>& f, size_t grain = 64) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t T = std::min<size_t>(std::min(16u, hw), std::max<size_t>(1, n / std::max<size_t>(1, grain)));
  if (T <= 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  std::vector<std::exception_ptr> errs(T);
  for (size_t t = 0; t < T; ++t)
    th.emplace_back([&, t]() {
      try {
        f(n * t / T, n * (t + 1) / T);
      } catch (...) {
        errs[t] = std::current_exception();
      }
    });
  for (auto& x : th) x.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
}

// Inverses of the element blocks R_e A R_e^T of the masked assembled operator of a 2D level
// (the local matrices of the Schwarz smoother, Sec. 5.3), from factors Gr in the level's
// storage precision: each block is the element's own matrix plus, on the nodes it shares with
// its (up to eight) neighbours, their element matrices' entries between those nodes; rows and
// columns of Dirichlet surface nodes are identity when masked.  Output [E][n][n], host FP64.
std::vector<double> schwarz_inverses(const semh::LevelGeom& G, const std::vector<double>& Gr,
                                     bool masked) {
  const int P = G.P, NP = G.NP, n = NP * NP, Nx = G.Nx, Nz = G.Nz;
  const size_t E = G.E, nn = (size_t)n * n;
  std::vector<double> Aall(E * nn);
  parallel_ranges(E, [&](size_t lo, size_t hi) {
    for (size_t e = lo; e < hi; ++e) semh::element_matrix(G, Gr, e, &Aall[e * nn]);
  });
  std::vector<double> out(E * nn);
  parallel_ranges(E, [&](size_t lo, size_t hi) {
    std::vector<double> B(nn), Bi(nn);
    std::vector<std::pair<int, int>> sh;  // (neighbour local node, this element's local node)
    for (size_t e = lo; e < hi; ++e) {
      const int ex = (int)(e / Nz), ez = (int)(e % Nz);
      std::copy(&Aall[e * nn], &Aall[e * nn] + nn, B.begin());
      for (int dx = -1; dx <= 1; ++dx)
        for (int dz = -1; dz <= 1; ++dz) {
          const int nx = ex + dx, nz = ez + dz;
          if ((dx == 0 && dz == 0) || nx < 0 || nx >= Nx || nz < 0 || nz >= Nz) continue;
          sh.clear();
          for (int i = 0; i < NP; ++i)
            for (int j = 0; j < NP; ++j) {
              const int li = nx * P + i - ex * P, lj = nz * P + j - ez * P;
              if (li >= 0 && li <= P && lj >= 0 && lj <= P) sh.push_back({i * NP + j, li * NP + lj});
            }
          const double* An = &Aall[((size_t)nx * Nz + nz) * nn];
          for (const auto& a : sh)
            for (const auto& b : sh) B[(size_t)a.second * n + b.second] += An[(size_t)a.first * n + b.first];
        }
      if (masked && ez == Nz - 1)
        for (int i = 0; i < NP; ++i) {  // local nodes (i, P) lie on the surface
          const int t = i * NP + P;
          for (int k = 0; k < n; ++k) B[(size_t)t * n + k] = B[(size_t)k * n + t] = 0.0;
          B[(size_t)t * n + t] = 1.0;
        }
      if (!semh::dense_inverse_public(n, B.data(), Bi.data()))
        throw ArgFail{"singular element block in the Schwarz smoother"};
      std::copy(Bi.begin(), Bi.end(), out.begin() + e * nn);
    }
  });
  return out;
}

// node range of element k's Schwarz box along one axis (order p, ov overlap layers, nn nodes)
struct Span1 {
  int lo, len;
};
inline Span1 box_span(int k, int p, int ov, int nn) {
  const int lo = std::max(0, k * p - ov), hi = std::min(nn - 1, k * p + p + ov);
  return {lo, hi - lo + 1};
}

// The box subdomains of the Schwarz smoother (Sec. 5.3) on a level with equal orders: element
// e's node box widened by ov layers per side and clipped; bx gets the sizes the kernels need.
// Returns the inverses of R_e A R_e^T of the masked assembled operator (factors Gr in the
// level's storage precision), subdomain e's n_e x n_e inverse at e nmax^2 (host FP64); rows and
// columns of Dirichlet surface nodes are identity when masked.
std::vector<double> schwarz_box_inverses(const semh::LevelGeom& G, const std::vector<double>& Gr,
                                         bool masked, int ov, semk::AsmBox* bx) {
  const bool d3 = G.dim == 3;
  const int P = G.P, NP = G.NP;
  const int Nx = G.Nx, Ny = d3 ? G.Ny : 1, Nz = G.Nz;
  const int nxn = (int)G.nxn, nyn = d3 ? (int)G.nyn : 1, nzn = (int)G.nzn;
  const size_t NL = d3 ? (size_t)NP * NP * NP : (size_t)NP * NP;
  const size_t E = G.E;
  auto cap = [&](int nn) { return std::min(nn, P + 1 + 2 * ov); };
  const size_t nmax = (size_t)cap(nxn) * cap(nyn) * cap(nzn);
  if (nmax > (size_t)semk::ASM_BOX_NMAX)
    throw ArgFail{"Schwarz subdomains too large (at most 4096 nodes; lower schwarz_overlap)"};
  if ((double)E * nmax * nmax * 8.0 > 4.0 * (1ull << 30))
    throw ArgFail{"Schwarz subdomain inverses exceed 4 GiB on a level (lower schwarz_overlap or "
                  "the mesh size)"};
  bx->Nx = Nx;
  bx->Ny = Ny;
  bx->Nz = Nz;
  bx->P = P;
  bx->ov = ov;
  bx->nmax = (int)nmax;
  bx->nxn = nxn;
  bx->nyn = nyn;
  bx->nzn = nzn;
  std::vector<double> Aall(E * NL * NL);
  parallel_ranges(E, [&](size_t lo, size_t hi) {
    for (size_t e = lo; e < hi; ++e) semh::element_matrix(G, Gr, e, &Aall[e * NL * NL]);
  }, 4);
  auto elem = [&](size_t e, int* ex, int* ey, int* ez) {
    *ez = (int)(e % Nz);
    const size_t exy = e / Nz;
    *ey = (int)(exy % Ny);
    *ex = (int)(exy / Ny);
  };
  std::vector<double> out(E * nmax * nmax, 0.0);
  double vals = 0.0, zv = 0.0;
  std::mutex mu;
  parallel_ranges(E, [&](size_t lo, size_t hi) {
    std::vector<double> B, Bi;
    std::vector<std::pair<int, int>> in;  // (element-local node, box-local node)
    double v2 = 0.0, v1 = 0.0;
    for (size_t e = lo; e < hi; ++e) {
      int ex, ey, ez;
      elem(e, &ex, &ey, &ez);
      const Span1 sx = box_span(ex, P, ov, nxn), sy = box_span(ey, P, ov, nyn),
                  sz = box_span(ez, P, ov, nzn);
      const int n = sx.len * sy.len * sz.len;
      B.assign((size_t)n * n, 0.0);
      Bi.assign((size_t)n * n, 0.0);
      // elements whose nodes meet the box along every axis
      auto range = [&](const Span1& sp, int Ne, int* f0, int* f1) {
        const int hi = sp.lo + sp.len - 1;
        *f0 = sp.lo > P ? (sp.lo - 1) / P : 0;
        *f1 = std::min(Ne - 1, hi / P);
      };
      int fx0, fx1, fy0, fy1, fz0, fz1;
      range(sx, Nx, &fx0, &fx1);
      range(sy, Ny, &fy0, &fy1);
      range(sz, Nz, &fz0, &fz1);
      if (!d3) fy0 = fy1 = 0;
      for (int fx = fx0; fx <= fx1; ++fx)
        for (int fy = fy0; fy <= fy1; ++fy)
          for (int fz = fz0; fz <= fz1; ++fz) {
            const size_t f = ((size_t)fx * Ny + fy) * Nz + fz;
            in.clear();
            for (size_t a = 0; a < NL; ++a) {
              int ai, am, aj;
              if (d3) { aj = (int)(a % NP); am = (int)((a / NP) % NP); ai = (int)(a / (NP * NP)); }
              else { ai = (int)(a / NP); am = 0; aj = (int)(a % NP); }
              const int gx = fx * P + ai - sx.lo, gy = (d3 ? fy * P + am : 0) - sy.lo,
                        gz = fz * P + aj - sz.lo;
              if (gx < 0 || gx >= sx.len || gy < 0 || gy >= sy.len || gz < 0 || gz >= sz.len)
                continue;
              in.push_back({(int)a, (gx * sy.len + gy) * sz.len + gz});
            }
            const double* Af = &Aall[f * NL * NL];
            for (const auto& a : in)
              for (const auto& b : in)
                B[(size_t)a.second * n + b.second] += Af[(size_t)a.first * NL + b.first];
          }
      if (masked && sz.lo + sz.len == nzn)  // box-local nodes on the surface: identity rows
        for (int q = sz.len - 1; q < n; q += sz.len) {
          for (int k = 0; k < n; ++k) B[(size_t)q * n + k] = B[(size_t)k * n + q] = 0.0;
          B[(size_t)q * n + q] = 1.0;
        }
      if (!semh::dense_inverse_public(n, B.data(), Bi.data()))
        throw ArgFail{"singular subdomain block in the Schwarz smoother"};
      std::copy(Bi.begin(), Bi.end(), out.begin() + e * nmax * nmax);
      v2 += (double)n * n;
      v1 += n;
    }
    std::lock_guard<std::mutex> lk(mu);
    vals += v2;
    zv += v1;
  }, 1);
  bx->ainv_vals = vals;
  bx->z_vals = zv;
  return out;
}

// The assembled operator of a 3D level of order 1 as a 27-point stencil, offset-major [27][N]
// (offset k = (dx+1) 9 + (dy+1) 3 + (dz+1)), from the element matrices of factors Gr; masked:
// identity rows on the Dirichlet surface and no coupling towards it (the masked matrix).
std::vector<double> stencil27(const semh::LevelGeom& G, const std::vector<double>& Gr,
                              bool masked) {
  const size_t N = G.N, nyn = G.nyn, nzn = G.nzn;
  std::vector<double> co(27 * N, 0.0), Ae(64);
  auto coords = [&](size_t g, long* ix, long* iy, long* iz) {
    *iz = (long)(g % nzn);
    const size_t q = g / nzn;
    *iy = (long)(q % nyn);
    *ix = (long)(q / nyn);
  };
  for (size_t e = 0; e < G.E; ++e) {
    semh::element_matrix(G, Gr, e, Ae.data());
    for (int a = 0; a < 8; ++a) {
      const size_t ga = semh::local_to_global(G, e, a);
      long ax, ay, az;
      coords(ga, &ax, &ay, &az);
      for (int b = 0; b < 8; ++b) {
        long bx, by, bz;
        coords(semh::local_to_global(G, e, b), &bx, &by, &bz);
        const long k = (bx - ax + 1) * 9 + (by - ay + 1) * 3 + (bz - az + 1);
        co[(size_t)k * N + ga] += Ae[(size_t)a * 8 + b];
      }
    }
  }
  if (masked)
    for (size_t g = 0; g < N; ++g) {
      const bool top = g % nzn == nzn - 1;
      for (int k = 0; k < 27; ++k) {
        const int dz = k % 3 - 1;
        if (top) co[(size_t)k * N + g] = (k == 13) ? 1.0 : 0.0;
        else if ((long)(g % nzn) + dz == (long)nzn - 1) co[(size_t)k * N + g] = 0.0;
      }
    }
  return co;
}

// stencil of a 3D level of order 1 (set-up, or refresh into the existing buffer)
void stencil_setup(Ctx* c, DLevel& L, const std::vector<double>& Gr) {
  const std::vector<double> co = stencil27(L.geo, Gr, c->masked != 0);
  if (L.dbl) L.st27 = put_vec(c, co, L.st27);
  else L.st27 = put_vec(c, std::vector<float>(co.begin(), co.end()), L.st27);
  if (!L.x3alt) L.x3alt = dalloc(c, L.N * esz(L.dbl));
}

// Schwarz smoother data of a level above the coarsest: element blocks (2D without overlap) or
// box subdomains, inverses in the level's precision; refresh: recompute the inverses of a new
// geometry into the existing buffers
void schwarz_setup(Ctx* c, DLevel& L, const std::vector<double>& Gr, bool refresh = false) {
  const int ov = c->desc.schwarz_overlap;
  const size_t eb = esz(L.dbl);
  std::vector<double> inv;
  size_t zn;
  if (c->dim == 2 && ov == 0) {
    inv = schwarz_inverses(L.geo, Gr, c->masked != 0);
    zn = (size_t)L.NP * L.NP;
  } else {
    inv = schwarz_box_inverses(L.geo, Gr, c->masked != 0, ov, &L.abox);
    L.asm_box = true;
    zn = (size_t)L.abox.nmax;
  }
  void* dst = refresh ? L.Ainv_s : nullptr;
  if (L.dbl) L.Ainv_s = put_vec(c, inv, dst);
  else L.Ainv_s = put_vec(c, std::vector<float>(inv.begin(), inv.end()), dst);
  if (!refresh) L.Zs = dalloc(c, L.geo.E * zn * eb);
}

void set_err(Ctx* c, const std::string& s) { c->err = s; }

// ------------------------------------------------------------------------------------------
// enqueue helpers
// ------------------------------------------------------------------------------------------
void apply_level(Ctx* c, int l, const void* x, int masked) {
  DLevel& L = c->lev[l];
  if (c->dim == 3 && L.st27 && masked == c->masked)
    HK(semk::stencil3d(L.dbl, x, L.y, L.st27, L.nxn, L.nyn, L.nzn, c->st));
  else if (c->dim == 3)
    HK(semk::apply3d(L.P, L.dbl, L.gt, x, L.y, L.Sx, L.Sy, L.Sxy, L.G, L.Nx, L.Ny, L.Nz, masked,
                     c->st));
  else if (L.rect)
    HK(semk::apply2r(L.P, L.Pz, L.dbl, L.gt, x, L.y, L.S, L.G, L.Dx, L.Dz, L.Nx, L.Nz, masked,
                     c->st));
  else
    HK(semk::apply2d(L.P, L.dbl, L.gt, x, L.y, L.S, L.G, L.Nx, L.Nz, masked, c->st));
}

void apply_outer(Ctx* c, const double* x, int masked) {
  DLevel& L = c->lev[0];
  if (c->dim == 3)
    HK(semk::apply3d(L.P, true, semk::G_COL64, x, c->yo, c->Sxo, c->Syo, c->Sxyo, c->CG64, L.Nx, L.Ny,
                     L.Nz, masked, c->st));
  else if (c->mixed)
    HK(semk::apply2r(L.P, L.Pz, true, semk::G_F64, x, c->yo, c->So, c->Gmix, c->Dmx, c->Dmz,
                     L.Nx, L.Nz, masked, c->st, 4));
  else if (L.rect)
    HK(semk::apply2r(L.P, L.Pz, true, semk::G_F64, x, c->yo, c->So, c->G64, L.Dx, L.Dz, L.Nx,
                     L.Nz, masked, c->st));
  else
    HK(semk::apply2d(L.P, true, semk::G_COL64, x, c->yo, c->So, c->CG64, L.Nx, L.Nz, masked,
                     c->st));
}

// one smoother step from the current x:  r = b - A x;  d = cd d + cr dinv r;  x += d
void smooth_step(Ctx* c, int l, double cd, double cr, int store_d) {
  DLevel& L = c->lev[l];
  if (c->dim == 3) {  // the update rides in the operator and its face fix-up, in place
    semk::Step3 s3;
    s3.b = L.b;
    s3.dinv = L.dinv;
    s3.d = L.d;
    s3.cd = cd;
    s3.cr = cr;
    s3.store_d = store_d;
    if (L.st27) {  // out of place into the second vector, then the two swap
      HK(semk::stencil3d(L.dbl, L.x, L.y, L.st27, L.nxn, L.nyn, L.nzn, c->st, s3, L.x3alt));
      std::swap(L.x, L.x3alt);
      return;
    }
    HK(semk::apply3d(L.P, L.dbl, L.gt, L.x, L.y, L.Sx, L.Sy, L.Sxy, L.G, L.Nx, L.Ny, L.Nz,
                     c->masked, c->st, s3));
    return;
  }
  if (L.xalt) {  // operator and update in one kernel, into the other vector
    HK(semk::cheb2d(L.P, L.dbl, L.gt, L.x, L.xalt, L.d, L.b, L.dinv, L.G, L.Nx, L.Nz, c->masked,
                    cd, cr, store_d, c->st));
    std::swap(L.x, L.xalt);
    return;
  }
  apply_level(c, l, L.x, c->masked);
  HK(semk::smooth_update(L.dbl, L.x, L.d, L.b, L.dinv, L.y, L.S, L.N, L.nzn, L.P, cd, cr,
                         semk::SU_AX, store_d, c->st));
}

// Chebyshev degree on level l (the finest, or every coarser level above the coarsest)
int cheb_k(const Ctx* c, int l) {
  const sem_mesh_desc& d = c->desc;
  return (l > 0 && d.cheb_degree_coarse > 0) ? d.cheb_degree_coarse : d.cheb_degree;
}

// coefficient and d-store flag of the first post-smoothing step taken from a known residual
// (x += cr dinv r, d = that step when more steps follow)
void first_post_step(const Ctx* c, int l, double* cr, int* store_d) {
  const sem_mesh_desc& d = c->desc;
  if (d.smoother == SEM_SMOOTH_JACOBI) {
    *cr = d.jacobi_omega;
    *store_d = 0;
    return;
  }
  const double lam = c->lev[l].lam;
  *cr = 1.0 / (0.5 * (d.cheb_hi * lam + d.cheb_lo * lam));
  *store_d = cheb_k(c, l) > 1 ? 1 : 0;
}

// pre- or post-smoothing on level l; resid (post-smoothing only): the residual of the current x,
// already known to the caller, which saves the first operator apply; first_done: the caller has
// already taken the first step from resid (first_post_step)
void smooth(Ctx* c, int l, bool pre, const void* resid = nullptr, bool first_done = false) {
  DLevel& L = c->lev[l];
  const sem_mesh_desc& d = c->desc;
  if (d.smoother == SEM_SMOOTH_SCHWARZ) {
    const int nu = pre ? d.nu_pre : d.nu_post;
    for (int s = 0; s < nu; ++s) {
      const bool fz = pre && s == 0;  // x = 0 on entry: r = b
      const void* r = nullptr;
      const void* ax = nullptr;       // with r = b: A x, complete (3D), subtracted in the gather
      if (fz) {
        if (l == 0 && c->vin64) HK(semk::cast_to(L.dbl, c->vin64, L.b, L.N, c->st));
        r = L.b;
      } else if (!pre && s == 0 && resid) {
        r = resid;
      } else if (c->dim == 3) {
        apply_level(c, l, L.x, c->masked);
        r = L.b;
        ax = L.y;
      } else {  // residual of the current x into the level's d vector (unused by this smoother)
        HK(semk::resid2d(L.P, L.dbl, L.gt, L.x, L.d, L.b, L.G, L.Nx, L.Nz, c->masked, L.y, L.S,
                         c->st));
        r = L.d;
      }
      if (L.asm_box)
        HK(semk::asm_box_sweep(L.abox, L.dbl, r, ax, L.Ainv_s, L.Zs, L.x, c->masked, fz ? 1 : 0,
                               c->st));
      else
        HK(semk::asm_sweep(L.P, L.dbl, r, L.Ainv_s, L.Zs, L.x, L.Nx, L.Nz, c->masked,
                           fz ? 1 : 0, c->st));
    }
    return;
  }
  if (d.smoother == SEM_SMOOTH_JACOBI) {
    const int nu = pre ? d.nu_pre : d.nu_post;
    int s0 = 0;
    if (pre && nu > 1 && L.xalt) {  // sweeps 0 (from x = 0) and 1 in one fused kernel
      HK(semk::cheb2d_first(L.P, L.dbl, L.gt, L.x, L.d, L.b, l == 0 ? c->vin64 : nullptr, L.dinv,
                            L.G, L.Nx, L.Nz, c->masked, d.jacobi_omega, 0.0, d.jacobi_omega, 0,
                            c->st));
      s0 = 2;
    }
    for (int s = s0; s < nu; ++s) {
      const bool fz = pre && s == 0;
      if (fz && l == 0 && c->vin64) {
        HK(semk::smooth_first64(L.dbl, L.x, L.d, L.b, c->vin64, L.dinv, L.N, d.jacobi_omega, 0,
                                c->st));
        continue;
      }
      const bool given = !pre && s == 0 && resid;
      if (given && first_done) continue;
      if (!fz && !given) {
        smooth_step(c, l, 0.0, d.jacobi_omega, 0);
        continue;
      }
      HK(semk::smooth_update(L.dbl, L.x, L.d, given ? resid : L.b, L.dinv, L.y, L.S, L.N, L.nzn,
                             L.P, 0.0, d.jacobi_omega, fz ? semk::SU_ZERO : semk::SU_RESID, 0,
                             c->st));
    }
    return;
  }
  const double a = d.cheb_lo * L.lam, b = d.cheb_hi * L.lam;
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a);
  const double sigma1 = theta / delta;
  double rho = 1.0 / sigma1;
  const int k = cheb_k(c, l);
  const bool given = !pre && resid;
  int j0 = 1;
  if (!pre && !given) {
    smooth_step(c, l, 0.0, 1.0 / theta, k > 1 ? 1 : 0);
  } else if (given && first_done) {
    // taken by the caller with the same coefficient (first_post_step)
  } else if (pre && k > 1 && L.xalt) {  // steps 0 (from x = 0) and 1 in one fused kernel
    const double rho_new = 1.0 / (2.0 * sigma1 - rho);
    HK(semk::cheb2d_first(L.P, L.dbl, L.gt, L.x, L.d, L.b, l == 0 ? c->vin64 : nullptr, L.dinv,
                          L.G, L.Nx, L.Nz, c->masked, 1.0 / theta, rho_new * rho,
                          2.0 * rho_new / delta, k > 2 ? 1 : 0, c->st));
    rho = rho_new;
    j0 = 2;
  } else if (pre && l == 0 && c->vin64)
    HK(semk::smooth_first64(L.dbl, L.x, L.d, L.b, c->vin64, L.dinv, L.N, 1.0 / theta,
                            k > 1 ? 1 : 0, c->st));
  else
    HK(semk::smooth_update(L.dbl, L.x, L.d, given ? resid : L.b, L.dinv, L.y, L.S, L.N, L.nzn,
                           L.P, 0.0, 1.0 / theta, pre ? semk::SU_ZERO : semk::SU_RESID,
                           k > 1 ? 1 : 0, c->st));
  for (int j = j0; j < k; ++j) {
    const double rho_new = 1.0 / (2.0 * sigma1 - rho);
    smooth_step(c, l, rho_new * rho, 2.0 * rho_new / delta, j + 1 < k ? 1 : 0);
    rho = rho_new;
  }
}

void restrict_to(Ctx* c, int l, bool use_ax) {
  DLevel& F = c->lev[l];
  DLevel& C = c->lev[l + 1];
  if (c->dim == 3) {  // b_c = (R_x R_y R_z)(b - A x): z, then y, then x; Dirichlet rows zeroed
    const unsigned nxf = F.nxn, nyf = F.nyn, nzf = F.nzn, nxc = C.nxn, nyc = C.nyn, nzc = C.nzn;
    HK(semk::axis_apply(F.dbl, 1, F.b, use_ax ? F.y : nullptr, c->tA, 0, nxf * nyf, nzf, nzc, 1,
                        F.R1[2].rp, F.R1[2].ci, F.R1[2].w, F.R1[2].nnz, F.R1[2].band,
                        F.R1[2].wband, F.R1[2].bandmax, 0, c->st));
    HK(semk::axis_apply(1, 1, c->tA, nullptr, c->tB, 0, nxf, nyf, nyc, nzc, F.R1[1].rp,
                        F.R1[1].ci, F.R1[1].w, F.R1[1].nnz, F.R1[1].band,
                        F.R1[1].wband, F.R1[1].bandmax, 0, c->st));
    HK(semk::axis_apply(1, C.dbl, c->tB, nullptr, C.b, 0, 1, nxf, nxc, nyc * nzc, F.R1[0].rp,
                        F.R1[0].ci, F.R1[0].w, F.R1[0].nnz, F.R1[0].band,
                        F.R1[0].wband, F.R1[0].bandmax,
                        c->masked ? nzc : 0, c->st));
    return;
  }
  if (F.axis >= 0) {  // one direction changes: b_c = R (b - A x) along it, Dirichlet rows zeroed
    const void* r2 = nullptr;
    if (use_ax) {  // A x complete into d (dead between the smoothing sweeps)
      HK(semk::fix_ax(F.dbl, F.y, F.S, F.d, 0, F.N, F.nzn, F.P, c->st));
      r2 = F.d;
    }
    const DLevel::Op1& R = F.R1[F.axis];
    if (F.axis == 0)
      HK(semk::axis_apply(F.dbl, C.dbl, F.b, r2, C.b, 0, 1, F.nxn, C.nxn, F.nzn, R.rp, R.ci, R.w,
                          R.nnz, R.band, R.wband, R.bandmax, c->masked ? C.nzn : 0, c->st));
    else
      HK(semk::axis_apply(F.dbl, C.dbl, F.b, r2, C.b, 0, F.nxn, F.nzn, C.nzn, 1, R.rp, R.ci, R.w,
                          R.nnz, R.band, R.wband, R.bandmax, c->masked ? C.nzn : 0, c->st));
    return;
  }
  HK(semk::restrict2d(F.dbl, C.dbl, F.b, F.y, F.S, use_ax ? 1 : 0, C.b, F.J, F.Nx, F.Nz, F.P,
                      C.P, c->masked, c->st));
}

void prolong_from(Ctx* c, int l) {
  DLevel& F = c->lev[l];
  DLevel& C = c->lev[l + 1];
  if (c->dim == 3) {  // x_f += (P_x P_y P_z) x_c: x, then y, then z
    const unsigned nxf = F.nxn, nyf = F.nyn, nzf = F.nzn, nxc = C.nxn, nyc = C.nyn, nzc = C.nzn;
    HK(semk::axis_apply(C.dbl, 1, C.x, nullptr, c->tB, 0, 1, nxc, nxf, nyc * nzc, F.P1[0].rp,
                        F.P1[0].ci, F.P1[0].w, F.P1[0].nnz, F.P1[0].band,
                        F.P1[0].wband, F.P1[0].bandmax, 0, c->st));
    HK(semk::axis_apply(1, 1, c->tB, nullptr, c->tA, 0, nxf, nyc, nyf, nzc, F.P1[1].rp,
                        F.P1[1].ci, F.P1[1].w, F.P1[1].nnz, F.P1[1].band,
                        F.P1[1].wband, F.P1[1].bandmax, 0, c->st));
    HK(semk::axis_apply(1, F.dbl, c->tA, nullptr, F.x, 1, nxf * nyf, nzc, nzf, 1, F.P1[2].rp,
                        F.P1[2].ci, F.P1[2].w, F.P1[2].nnz, F.P1[2].band,
                        F.P1[2].wband, F.P1[2].bandmax, 0, c->st));
    return;
  }
  if (F.axis >= 0) {  // x_f += P x_c along the one direction that changes
    const DLevel::Op1& Pr = F.P1[F.axis];
    if (F.axis == 0)
      HK(semk::axis_apply(C.dbl, F.dbl, C.x, nullptr, F.x, 1, 1, C.nxn, F.nxn, F.nzn, Pr.rp,
                          Pr.ci, Pr.w, Pr.nnz, Pr.band, Pr.wband, Pr.bandmax, 0, c->st));
    else
      HK(semk::axis_apply(C.dbl, F.dbl, C.x, nullptr, F.x, 1, F.nxn, C.nzn, F.nzn, 1, Pr.rp,
                          Pr.ci, Pr.w, Pr.nnz, Pr.band, Pr.wband, Pr.bandmax, 0, c->st));
    return;
  }
  HK(semk::prolong2d(F.dbl, C.dbl, C.x, F.x, F.J, F.Nx, F.Nz, F.P, C.P, c->st));
}

void coarse_solve(Ctx* c) {
  DLevel& L = c->lev.back();
  double* b = (double*)L.b;
  double* x = (double*)L.x;
  if (c->Ainv) {  // 3D: dense inverse of the (masked) coarsest operator
    HK(semk::dense_gemv(c->Ainv, b, x, c->nAinv, c->st));
    return;
  }
  const semh::BcrPlan& pl = c->plan;
  const int nl = (int)pl.levs.size();
  {  // block reduction: each factor array read once, the right-hand side and solution
    auto sz = [&](const void* q) {
      auto it = c->asize.find(q);
      return it == c->asize.end() ? 0.0 : (double)it->second;
    };
    semk::acct_add(sz(c->bcrF) + sz(c->bcrB) + sz(c->bcrDense) + 4.0 * 8.0 * L.N);
  }
  if (c->bcrLv.nl >= 0) {
    const double* br = b;
    if (nl > 0) {
      HK(semk::bcr_fwd_all(b, c->bcrRed, c->bcrF, c->bcrLv, pl.nblocks, pl.bstride, L.nzn - 1,
                           pl.nb, c->st));
      br = c->bcrRed;
    }
    HK(semk::bcr_dense(c->bcrDense, br, x, pl.dense_n * pl.nb, pl.nb, pl.dense_stride,
                       pl.bstride, L.nzn - 1, c->st));
    if (nl > 0)
      HK(semk::bcr_bwd_all(br, x, c->bcrB, c->bcrLv, pl.nblocks, pl.bstride, L.nzn - 1, pl.nb,
                           c->st));
    return;
  }
  for (int l = 0; l < nl; ++l) {
    const auto& v = pl.levs[l];
    HK(semk::bcr_fwd(b, c->bcrF + v.offM, v.n, v.stride, v.neven, pl.bstride, L.nzn - 1, pl.nb,
                     c->st));
  }
  HK(semk::bcr_dense(c->bcrDense, b, x, pl.dense_n * pl.nb, pl.nb, pl.dense_stride, pl.bstride,
                     L.nzn - 1, c->st));
  for (int l = nl - 1; l >= 0; --l) {
    const auto& v = pl.levs[l];
    HK(semk::bcr_bwd(b, x, c->bcrB + v.offB, v.n, v.stride, v.nodd, pl.bstride, L.nzn - 1,
                     pl.nb, c->st));
  }
}

// learned stage on level 0: reads L.b, L.x; updates L.x, writes the new residual to Rbuf.  post:
// post-smoothing follows, and its first step from Rbuf is taken in the stage's update kernel.
// fold (pre-smoothing position): where the fused kernels apply, the update is left to the
// restriction (residual r - alpha q) and the prolongation (x += alpha c): *f is filled and Rbuf
// keeps r; otherwise f->q stays null and the update runs here
void learned_stage(Ctx* c, bool post = false, semk::StageFold* f = nullptr) {
  DLevel& L = c->lev[0];
  semm::Stage& s = c->stage;
  const int ncr = semm::stage_mlp_blocks(s.E);
  double* pcr = c->stparts;
  double* pcq = c->stparts + ncr;
  HK(semk::resid2d(L.P, L.dbl, L.gt, L.x, c->Rbuf, L.b, L.G, L.Nx, L.Nz, c->masked, L.y, L.S,
                   c->st));
  HK(semm::stage_mlp(s, L.dbl, c->Rbuf, c->masked, pcr, c->st));
  double sr = 0.0;
  int store_d = 0;
  if (post) first_post_step(c, 0, &sr, &store_d);
  const void* dinv = post ? L.dinv : nullptr;
  const int nfused = semk::cheb2d_blocks(L.P, L.Nx, L.Nz, L.dbl);
  if (nfused > 0) {  // assembly fused with the apply of c: q complete, no side buffer
    HK(semk::stagecq2d(L.P, L.dbl, L.gt, s.CE, c->cbuf, c->yq, L.G, L.Nx, L.Nz, c->masked, pcq,
                       c->st));
    if (f) {
      f->q = c->yq;
      f->c = c->cbuf;
      f->pcr = pcr;
      f->ncr = ncr;
      f->pcq = pcq;
      f->ncq = nfused;
      f->skips = s.skips;
      return;
    }
    HK(semm::stage_update(L.dbl, L.x, c->Rbuf, c->cbuf, c->yq, nullptr, pcr, ncr, pcq, nfused,
                          s.skips, L.N, L.nzn, L.P, dinv, L.d, sr, store_d, c->st));
    return;
  }
  HK(semm::stage_assemble(s, L.dbl, c->cbuf, c->masked, c->st));
  HK(semk::apply2d_dot(L.P, L.dbl, L.gt, c->cbuf, c->yq, c->Sq, L.G, L.Nx, L.Nz, c->masked, pcq,
                       c->st));
  HK(semm::stage_update(L.dbl, L.x, c->Rbuf, c->cbuf, c->yq, c->Sq, pcr, ncr, pcq,
                        semk::apply2d_blocks(L.P, L.Nx, L.Nz, L.dbl), s.skips, L.N, L.nzn, L.P,
                        dinv, L.d, sr, store_d, c->st));
}

// learned stage on the fine level of a 3D mesh: r = b - A x, the network's element corrections,
// their average c, q = A c, and the judged update x += alpha c (alpha = c.r / c.q)
void learned_stage3d(Ctx* c) {
  DLevel& L = c->lev[0];
  semm::Stage& s = c->stage;
  const int ncr = semm::stage_mlp_blocks(s.E);
  double* pcr = c->stparts;
  double* pcq = c->stparts + ncr;
  apply_level(c, 0, L.x, c->masked);
  HK(semk::vaxpby(L.dbl, 1.0, L.b, -1.0, L.y, c->Rbuf, L.N, c->st));
  HK(semm::stage_mlp(s, L.dbl, c->Rbuf, c->masked, pcr, c->st));
  HK(semm::stage_assemble(s, L.dbl, c->cbuf, c->masked, c->st));
  apply_level(c, 0, c->cbuf, c->masked);
  HK(semk::dot_partial(L.dbl, c->cbuf, L.y, pcq, L.N, c->st));
  HK(semm::stage_update(L.dbl, L.x, c->Rbuf, c->cbuf, L.y, nullptr, pcr, ncr, pcq, semk::NRED,
                        s.skips, L.N, L.nzn, L.P, nullptr, L.d, 0.0, 0, c->st));
}

// z = B r on level 0 buffers: input r (FP64, device), output lev[0].x
// the step coefficients of level l's smoothing sequence (as smooth() takes them) and the number
// of operator applies of its one-kernel form; false when that form does not apply
bool coarse_seq(const Ctx* c, int l, bool pre, semk::CoarseSeq* sq, int* applies) {
  const sem_mesh_desc& d = c->desc;
  const DLevel& L = c->lev[l];
  if (d.smoother == SEM_SMOOTH_CHEBYSHEV) {
    const int k = cheb_k(c, l);
    if (k < 1 || k > semk::CO_MAXS) return false;
    const double a = d.cheb_lo * L.lam, b = d.cheb_hi * L.lam;
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a);
    const double sigma1 = theta / delta;
    double rho = 1.0 / sigma1;
    sq->ns = k;
    sq->cd[0] = 0.0;
    sq->cr[0] = 1.0 / theta;
    for (int j = 1; j < k; ++j) {
      const double rho_new = 1.0 / (2.0 * sigma1 - rho);
      sq->cd[j] = rho_new * rho;
      sq->cr[j] = 2.0 * rho_new / delta;
      rho = rho_new;
    }
    *applies = k;
    return true;
  }
  if (d.smoother == SEM_SMOOTH_JACOBI) {
    const int nu = pre ? d.nu_pre : d.nu_post;
    if (nu < 1 || nu > semk::CO_MAXS) return false;
    sq->ns = nu;
    for (int j = 0; j < nu; ++j) {
      sq->cd[j] = 0.0;
      sq->cr[j] = d.jacobi_omega;
    }
    *applies = nu;
    return true;
  }
  return false;
}

// level l >= 1 (2D): pre-smoothing + residual + restriction, or prolongation + post-smoothing,
// in one kernel; false when the level keeps the per-step kernels
bool coarse_fused(Ctx* c, int l, bool pre) {
  DLevel& L = c->lev[l];
  const semk::CoarsePlan& pl = pre ? L.cpre : L.cpost;
  if (pl.W < 1) return false;
  semk::CoarseSeq sq;
  int applies = 0;
  if (!coarse_seq(c, l, pre, &sq, &applies)) return false;
  DLevel& C = c->lev[l + 1];
  const int k1 = pre ? L.cpre_k1 : L.cpost_k1;
  if (k1 == 0) {
    semk::CoarseIO io;
    io.flags = pre ? semk::CO_RESTRICT : semk::CO_PROLONG;
    if (pre) {
      HK(semk::coarse2d(true, pl, L.P, C.P, L.dbl, L.gt, C.dbl, nullptr, L.x, L.b, L.dinv, L.G,
                        nullptr, C.b, L.J, L.Nx, L.Nz, c->masked, sq, c->st, io));
    } else {
      HK(semk::coarse2d(false, pl, L.P, C.P, L.dbl, L.gt, C.dbl, L.x, L.xalt, L.b, L.dinv, L.G,
                        C.x, nullptr, L.J, L.Nx, L.Nz, c->masked, sq, c->st, io));
      std::swap(L.x, L.xalt);
    }
    return true;
  }
  // two launches: steps 0 .. k1-1 (x and d written), then k1 .. ns-1 continuing from them
  semk::CoarseSeq s1, s2;
  s1.ns = k1;
  s2.ns = sq.ns - k1;
  for (int j = 0; j < sq.ns; ++j) {
    semk::CoarseSeq& t = j < k1 ? s1 : s2;
    const int i = j < k1 ? j : j - k1;
    t.cd[i] = sq.cd[j];
    t.cr[i] = sq.cr[j];
  }
  const semk::CoarsePlan& pl2 = pre ? L.cpre2 : L.cpost2;
  semk::CoarseIO first, second;
  first.dout = L.d;
  second.din = L.d;
  if (pre) {
    second.flags = semk::CO_FROM_X | semk::CO_RESTRICT;
    HK(semk::coarse2d(true, pl, L.P, C.P, L.dbl, L.gt, C.dbl, nullptr, L.x, L.b, L.dinv, L.G,
                      nullptr, nullptr, L.J, L.Nx, L.Nz, c->masked, s1, c->st, first));
    HK(semk::coarse2d(true, pl2, L.P, C.P, L.dbl, L.gt, C.dbl, L.x, L.xalt, L.b, L.dinv, L.G,
                      nullptr, C.b, L.J, L.Nx, L.Nz, c->masked, s2, c->st, second));
    std::swap(L.x, L.xalt);
  } else {
    first.flags = semk::CO_PROLONG;
    HK(semk::coarse2d(false, pl, L.P, C.P, L.dbl, L.gt, C.dbl, L.x, L.xalt, L.b, L.dinv, L.G,
                      C.x, nullptr, L.J, L.Nx, L.Nz, c->masked, s1, c->st, first));
    std::swap(L.x, L.xalt);
    HK(semk::coarse2d(false, pl2, L.P, C.P, L.dbl, L.gt, C.dbl, L.x, L.xalt, L.b, L.dinv, L.G,
                      nullptr, nullptr, L.J, L.Nx, L.Nz, c->masked, s2, c->st, second));
    std::swap(L.x, L.xalt);
  }
  return true;
}

void vcycle(Ctx* c, const double* r) {
  const int L = (int)c->lev.size();
  DLevel& L0 = c->lev[0];
  const bool fused_entry =
      L > 1 && (c->desc.smoother == SEM_SMOOTH_CHEBYSHEV || c->desc.nu_pre > 0);
  if (fused_entry) c->vin64 = r;
  else HK(semk::cast_to(L0.dbl, r, L0.b, L0.N, c->st));
  if (L == 1) {
    coarse_solve(c);
    return;
  }
  semk::StageFold fold;  // the pre-smoothing stage's step, when folded into the transfers
  for (int l = 0; l < L - 1; ++l) {
    if (l >= 1 && coarse_fused(c, l, true)) continue;
    smooth(c, l, true);
    if (l == 0) c->vin64 = nullptr;
    if (l == 0 && c->dim == 3 && c->stage.enabled && (c->stage_mode & 1)) learned_stage3d(c);
    if (l == 0 && c->dim == 2 && c->stage.enabled && (c->stage_mode & 1)) {
      learned_stage(c, false, &fold);  // the step goes into the transfers when fold.q is set
      DLevel& F = c->lev[0];
      DLevel& C1 = c->lev[1];
      HK(semk::restrict2d(F.dbl, C1.dbl, c->Rbuf, nullptr, nullptr, 0, C1.b, F.J, F.Nx, F.Nz, F.P,
                          C1.P, c->masked, c->st, fold));
      continue;
    }
    apply_level(c, l, c->lev[l].x, c->masked);
    restrict_to(c, l, true);
  }
  coarse_solve(c);
  for (int l = L - 2; l >= 0; --l) {
    if (l >= 1 && coarse_fused(c, l, false)) continue;
    if (l == 0 && fold.c) {
      DLevel& F = c->lev[0];
      DLevel& C1 = c->lev[1];
      HK(semk::prolong2d(F.dbl, C1.dbl, C1.x, F.x, F.J, F.Nx, F.Nz, F.P, C1.P, c->st, fold));
    } else {
      prolong_from(c, l);
    }
    if (l == 0 && c->dim == 3 && c->stage.enabled && (c->stage_mode & 2)) learned_stage3d(c);
    if (l == 0 && c->dim == 2 && c->stage.enabled && (c->stage_mode & 2)) {
      const bool fold = c->desc.smoother != SEM_SMOOTH_SCHWARZ;
      learned_stage(c, fold);  // with fold, also the first post-smoothing step from its residual
      smooth(c, l, false, c->Rbuf, fold);
      continue;
    }
    smooth(c, l, false);
  }
  c->vin64 = nullptr;
}

double* pset(Ctx* c, int s) { return c->parts + (size_t)s * semk::NRED; }

// one FPCG iteration (see sem.h): V-cycle on r, direction update, outer FP64 apply, x/r update
void fpcg_iteration(Ctx* c, bool first) {
  DLevel& L0 = c->lev[0];
  const unsigned N = L0.N;
  vcycle(c, c->ro);
  HK(semk::castdot(L0.dbl, L0.x, c->zo, first ? nullptr : c->qo, c->ro, pset(c, PS_ZQ),
                   pset(c, PS_RZB), N, c->st));
  if (c->dim == 2 && !L0.rect && semk::fpcg2d_fits(L0.P, L0.Nx, L0.Nz)) {
    // direction update fused with the FP64 operator, then the x / r update (beta in scal[8])
    double* beta = c->scal + 8;
    HK(semk::fpcg2d(L0.P, c->zo, c->po, c->qo, c->CG64, L0.Nx, L0.Nz, c->masked,
                    pset(c, PS_RZA), pset(c, PS_PQ), pset(c, PS_ZQ), first ? 1 : 0,
                    pset(c, PS_PQ2), beta, c->st, 1));
    HK(semk::update_xrp(c->xo, c->ro, c->po, c->zo, c->qo, beta, first ? 1 : 0,
                        pset(c, PS_RZB), pset(c, PS_PQ2), pset(c, PS_RZA), pset(c, PS_PQ),
                        pset(c, PS_RR), N, c->st));
    return;
  }
  HK(semk::pupdate(c->po, c->zo, pset(c, PS_RZA), pset(c, PS_PQ), pset(c, PS_ZQ), first ? 1 : 0,
                   N, c->st));
  apply_outer(c, c->po, c->masked);
  HK(semk::fixdot64(c->yo, c->So, c->qo, c->po, pset(c, PS_PQ), pset(c, PS_RZB), pset(c, PS_RZA),
                    N, L0.nzn, L0.P, c->st));
  HK(semk::update_xr(c->xo, c->ro, c->po, c->qo, pset(c, PS_RZA), pset(c, PS_PQ),
                     pset(c, PS_RR), N, c->st));
}

void pdc_iteration(Ctx* c) {
  DLevel& L0 = c->lev[0];
  const unsigned N = L0.N;
  vcycle(c, c->ro);
  HK(semk::cast_from(L0.dbl, L0.x, c->zo, N, c->st));
  HK(semk::axpy64(c->xo, c->zo, 1.0, N, c->st));
  apply_outer(c, c->xo, c->masked);
  HK(semk::resid64(c->bo, c->yo, c->So, c->ro, pset(c, PS_RR), nullptr, N, L0.nzn, L0.P, c->st));
}

// copy partial-sum sets 0..2 (RR, BB, PQ) to the host and sum each in a fixed order
void read_sums(Ctx* c, double* sums) {
  HK(hipMemcpyAsync(c->hscal, c->parts, 3 * semk::NRED * sizeof(double), hipMemcpyDeviceToHost,
                    c->st));
  HK(hipStreamSynchronize(c->st));
  for (int s = 0; s < 3; ++s) {
    double v = 0.0;
    for (int k = 0; k < semk::NRED; ++k) v += c->hscal[s * semk::NRED + k];
    sums[s] = v;
  }
}

void drop_graphs(Ctx* c) {
  if (c->g_first) (void)hipGraphExecDestroy(c->g_first);
  c->g_first = nullptr;
  for (int k = 0; k < 2; ++k) {
    if (c->g_iter[k]) (void)hipGraphExecDestroy(c->g_iter[k]);
    if (c->g_pdc[k]) (void)hipGraphExecDestroy(c->g_pdc[k]);
    c->g_iter[k] = c->g_pdc[k] = nullptr;
  }
}

template <typename F>
hipGraphExec_t capture(Ctx* c, F body) {
  hipGraph_t g = nullptr;
  HK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
  try {
    body();
  } catch (...) {
    hipGraph_t tmp = nullptr;
    (void)hipStreamEndCapture(c->st, &tmp);
    if (tmp) (void)hipGraphDestroy(tmp);
    throw;
  }
  HK(hipStreamEndCapture(c->st, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) throw HipFail{e, "hipGraphInstantiate"};
  return ex;
}

// ------------------------------------------------------------------------------------------
// set-up
// ------------------------------------------------------------------------------------------
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  // largest eigenvalue of the symmetric tridiagonal (diag a, off-diag b) by bisection on the
  // Sturm count
  const int n = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {  // eigenvalues < x
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < n; ++i) {
      if (q == 0.0) q = 1e-300;
      q = a[i] - x - b[i - 1] * b[i - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= n) hi = mid;
    else lo = mid;
  }
  return hi;
}

double host_sum_partials(Ctx* c, int set) {
  std::vector<double> h(semk::NRED);
  HK(hipMemcpyAsync(h.data(), pset(c, set), semk::NRED * sizeof(double), hipMemcpyDeviceToHost,
                    c->st));
  HK(hipStreamSynchronize(c->st));
  double s = 0;
  for (double v : h) s += v;
  return s;
}

void lanczos(Ctx* c, int l) {
  DLevel& L = c->lev[l];
  const unsigned N = L.N;
  const bool dbl = L.dbl;
  const int steps = std::max(2, c->desc.lanczos_steps);
  // start vector: SplitMix64 on free nodes; sqrt(dinv)
  std::vector<double> v0(N), sq(N);
  std::vector<double> dinv_h(N);
  void* s = dalloc(c, N * esz(dbl));
  void* q = dalloc(c, N * esz(dbl));
  void* qp = dalloc(c, N * esz(dbl));
  void* w = dalloc(c, N * esz(dbl));
  void* tmp = dalloc(c, N * esz(dbl));
  // sqrt of dinv computed on the host from the device copy
  if (dbl) {
    HK(hipMemcpy(dinv_h.data(), L.dinv, N * 8, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(N);
    HK(hipMemcpy(f.data(), L.dinv, N * 4, hipMemcpyDeviceToHost));
    for (unsigned g = 0; g < N; ++g) dinv_h[g] = f[g];
  }
  double nrm = 0;
  for (unsigned g = 0; g < N; ++g) {
    const bool top = c->masked && (g % L.nzn) == (unsigned)(L.nzn - 1);
    v0[g] = top ? 0.0 : semh::splitmix64_uniform(c->desc.lanczos_seed, g);
    nrm += v0[g] * v0[g];
    sq[g] = std::sqrt(dinv_h[g]);
  }
  nrm = std::sqrt(nrm);
  for (auto& v : v0) v /= nrm;
  auto put = [&](void* dst, const std::vector<double>& h) {
    if (dbl) {
      HK(hipMemcpy(dst, h.data(), N * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> f(h.begin(), h.end());
      HK(hipMemcpy(dst, f.data(), N * 4, hipMemcpyHostToDevice));
    }
  };
  put(s, sq);
  put(q, v0);
  std::vector<double> al, be;
  double beta = 0.0;
  for (int k = 0; k < steps; ++k) {
    HK(semk::vmul(dbl, q, s, tmp, N, c->st));
    apply_level(c, l, tmp, c->masked);
    HK(semk::fix_ax(dbl, L.y, L.S, w, 0, N, L.nzn, L.P, c->st));
    HK(semk::vmul(dbl, w, s, w, N, c->st));
    HK(semk::dot_partial(dbl, q, w, pset(c, PS_TMP), N, c->st));
    const double alpha = host_sum_partials(c, PS_TMP);
    HK(semk::vaxpby(dbl, 1.0, w, -alpha, q, w, N, c->st));
    if (k > 0) HK(semk::vaxpby(dbl, 1.0, w, -beta, qp, w, N, c->st));
    al.push_back(alpha);
    HK(semk::dot_partial(dbl, w, w, pset(c, PS_TMP), N, c->st));
    beta = std::sqrt(std::max(0.0, host_sum_partials(c, PS_TMP)));
    if (k == steps - 1 || beta == 0.0) break;
    be.push_back(beta);
    std::swap(qp, q);
    HK(semk::vaxpby(dbl, 1.0 / beta, w, 0.0, w, q, N, c->st));
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  L.lam = tridiag_max_eig(al, be);
  HK(hipStreamSynchronize(c->st));
}

// learned-stage geometry of the fine level (2D): per-element features and mean element-matrix
// diagonal, from the level's current geometry
void learned_geometry3d(Ctx* c);
void learned_geometry(Ctx* c) {
  if (c->dim == 3) {
    learned_geometry3d(c);
    return;
  }
  const semh::LevelGeom& G = c->lev[0].geo;
  if (c->lev[0].rect || c->lev[0].axis >= 0) {  // no learned stage on such a fine level
    c->geo_h.clear();
    c->abar_h.clear();
    return;
  }
  const int NP = G.NP, n = NP * NP;
  const size_t E = G.E, NL = n;
  c->geo_h.assign(E * 4 * n, 0.f);
  c->abar_h.assign(E, 0.f);
  const double* Dm = G.D.data();
  for (size_t e = 0; e < E; ++e) {
    const double* Grr = &G.G[0 * E * NL + e * NL];
    const double* Grs = &G.G[1 * E * NL + e * NL];
    const double* Gss = &G.G[2 * E * NL + e * NL];
    const double* ms = &G.mass[e * NL];
    double gsum = 0, msum = 0, dsum = 0;
    for (int l = 0; l < n; ++l) {
      gsum += Grr[l] + Gss[l];
      msum += ms[l];
      const int i = l / NP, j = l % NP;
      double dl = 0;
      for (int k = 0; k < NP; ++k) dl += Dm[k * NP + i] * Dm[k * NP + i] * Grr[k * NP + j];
      dl += 2.0 * Dm[i * NP + i] * Dm[j * NP + j] * Grs[l];
      for (int k = 0; k < NP; ++k) dl += Dm[k * NP + j] * Dm[k * NP + j] * Gss[i * NP + k];
      dsum += dl;
    }
    const double g = gsum / n, mm = msum / n;
    float* out = &c->geo_h[e * 4 * n];
    for (int l = 0; l < n; ++l) {
      out[l] = (float)(Grr[l] / g);
      out[n + l] = (float)(Grs[l] / g);
      out[2 * n + l] = (float)(Gss[l] / g);
      out[3 * n + l] = (float)(ms[l] / mm);
    }
    c->abar_h[e] = (float)(dsum / n);
  }
}

// the same for hexahedra (P <= 6): [G_rr, G_tt, G_rs, G_ts, G_ss] / g_e with g_e the element mean
// of G_rr + G_tt + G_ss, then m_e / mean(m_e) (6n values per element), and a_e the mean of
// diag(A_e): sum_k D_ki^2 G_rr + D_km^2 G_tt + D_kj^2 G_ss along the three lines through the node,
// plus 2 D_ii D_jj G_rs + 2 D_mm D_jj G_ts at the node itself
void learned_geometry3d(Ctx* c) {
  const semh::LevelGeom& G = c->lev[0].geo;
  const int NP = G.NP, n = NP * NP * NP;
  if (G.P > semm::MAX_STAGE_P3) {
    c->geo_h.clear();
    c->abar_h.clear();
    return;
  }
  const size_t E = G.E, NL = n;
  c->geo_h.assign(E * 6 * n, 0.f);
  c->abar_h.assign(E, 0.f);
  const double* Dm = G.D.data();
  for (size_t e = 0; e < E; ++e) {
    const double* F[5];
    for (int f = 0; f < 5; ++f) F[f] = &G.G[(size_t)f * E * NL + e * NL];
    const double* ms = &G.mass[e * NL];
    double gsum = 0, msum = 0, dsum = 0;
    for (int l = 0; l < n; ++l) {
      gsum += F[0][l] + F[1][l] + F[4][l];
      msum += ms[l];
      const int i = l / (NP * NP), m = (l / NP) % NP, j = l % NP;
      double dl = 0;
      for (int k = 0; k < NP; ++k) {
        dl += Dm[k * NP + i] * Dm[k * NP + i] * F[0][(k * NP + m) * NP + j];
        dl += Dm[k * NP + m] * Dm[k * NP + m] * F[1][(i * NP + k) * NP + j];
        dl += Dm[k * NP + j] * Dm[k * NP + j] * F[4][(i * NP + m) * NP + k];
      }
      dl += 2.0 * Dm[i * NP + i] * Dm[j * NP + j] * F[2][l];
      dl += 2.0 * Dm[m * NP + m] * Dm[j * NP + j] * F[3][l];
      dsum += dl;
    }
    const double g = gsum / n, mm = msum / n;
    float* out = &c->geo_h[e * 6 * n];
    for (int l = 0; l < n; ++l) {
      for (int f = 0; f < 5; ++f) out[f * n + l] = (float)(F[f][l] / g);
      out[5 * n + l] = (float)(ms[l] / mm);
    }
    c->abar_h[e] = (float)(dsum / n);
  }
}

// ---------------------------------------------------------------------------------------------
// 3D set-up: p-levels as in 2D, then (below P = 1) levels coarsened by 2 in x and y with linear
// transfers until at most desc.coarse_dense_max nodes remain; that level is solved exactly with
// the dense inverse of its masked operator.
// ---------------------------------------------------------------------------------------------
template <typename TG, typename Conv>
std::vector<TG> permute_G3d(const semh::LevelGeom& L, Conv conv) {
  // per element column (ex, ey): thread t = (ez NP + i) NP + m owns the 5 NP values (f, j) of its
  // vertical line, chunked as in the 2D layout (semk::g3d_layout)
  const int NP = L.NP, Nz = L.Nz;
  const size_t NL3 = (size_t)NP * NP * NP, nthr = (size_t)NP * NP * Nz;
  const size_t ncol = (size_t)L.Nx * L.Ny;
  const semk::GLayout lay = semk::g3d_layout(L.P, Nz, sizeof(TG));
  std::vector<TG> out(ncol * lay.cstride, TG(0));
  for (size_t col = 0; col < ncol; ++col)
    for (int ez = 0; ez < Nz; ++ez)
      for (int i = 0; i < NP; ++i)
        for (int m = 0; m < NP; ++m) {
          const size_t e = col * Nz + ez, t = ((size_t)ez * NP + i) * NP + m;
          for (int f = 0; f < 5; ++f)
            for (int j = 0; j < NP; ++j) {
              const int k = f * NP + j, q = k / lay.W, w = k % lay.W;
              const size_t off = q < lay.NC ? ((size_t)q * nthr + t) * lay.W + w
                                            : (size_t)lay.NC * nthr * lay.W + t * lay.REM +
                                                  (size_t)(k - lay.NC * lay.W);
              out[col * lay.cstride + off] =
                  conv(L.G[f * L.E * NL3 + e * NL3 + ((size_t)i * NP + m) * NP + j]);
            }
        }
  return out;
}

typedef std::vector<std::vector<std::pair<int, double>>> Rows1;

// 1D prolongation between GLL orders Pf > Pc on Ne elements: coarse Lagrange basis at the fine
// nodes (J, (Pf+1) x (Pc+1)); a node shared by two elements gets one row (J's end rows are
// exact unit rows, so both elements agree)
Rows1 prol1d_p(int Ne, int Pf, int Pc, const std::vector<double>& J) {
  Rows1 r((size_t)Ne * Pf + 1);
  for (int e = 0; e < Ne; ++e)
    for (int a = 0; a <= Pf; ++a) {
      auto& row = r[(size_t)e * Pf + a];
      if (!row.empty()) continue;
      for (int b = 0; b <= Pc; ++b) {
        const double v = J[(size_t)a * (Pc + 1) + b];
        if (v != 0.0) row.push_back({e * Pc + b, v});
      }
    }
  return r;
}

// 1D linear interpolation from Nc to 2 Nc intervals (P = 1 nodes)
Rows1 prol1d_h(int Nc) {
  Rows1 r((size_t)2 * Nc + 1);
  for (int f = 0; f <= 2 * Nc; ++f) {
    if (f % 2 == 0) r[f].push_back({f / 2, 1.0});
    else {
      r[f].push_back({(f - 1) / 2, 0.5});
      r[f].push_back({(f + 1) / 2, 0.5});
    }
  }
  return r;
}

Rows1 ident1d(int n) {
  Rows1 r(n);
  for (int k = 0; k < n; ++k) r[k].push_back({k, 1.0});
  return r;
}

Rows1 transpose1d(const Rows1& r, int ncols) {
  Rows1 t(ncols);
  for (size_t f = 0; f < r.size(); ++f)
    for (const auto& e : r[f]) t[e.first].push_back({(int)f, e.second});
  return t;
}

void upload_op(Ctx* c, const Rows1& r, DLevel::Op1& op) {
  std::vector<int> rp(1, 0), ci, band;
  std::vector<double> w, wband;
  for (const auto& row : r) {
    int lo = INT_MAX, hi = -1;
    for (const auto& e : row) {
      ci.push_back(e.first);
      w.push_back(e.second);
      lo = std::min(lo, e.first);
      hi = std::max(hi, e.first);
    }
    rp.push_back((int)ci.size());
    // the row as a band [lo, hi] with zero weights where it has no entry
    const int len = hi >= lo ? hi - lo + 1 : 0, off = (int)wband.size();
    wband.resize(wband.size() + len, 0.0);
    for (const auto& e : row) wband[off + e.first - lo] += e.second;
    band.insert(band.end(), {len ? lo : 0, len, off, 0});
    op.bandmax = std::max(op.bandmax, len);
  }
  if (wband.empty()) wband.push_back(0.0);
  op.nnz = (unsigned)ci.size();
  op.rp = upload(c, rp);
  op.ci = upload(c, ci);
  op.w = upload(c, w);
  op.band = upload(c, band);
  op.wband = upload(c, wband);
}

}  // namespace
static void rebuild_levels(Ctx* c);  // defined with the surface update below
namespace {

// depth h + eta at every surface node, for the surface derivative of the stage loop
std::vector<double> surface_depths(const Ctx* c) {
  std::vector<double> d(c->hf_h.size());
  for (size_t k = 0; k < d.size(); ++k) d[k] = c->hf_h[k] + c->ef_h[k];
  return d;
}

// the V-cycle levels from the still-water geometry (eta = 0) when the descriptor asks for it;
// the outer operator, mass and faces keep the given surface
void still_water_levels(Ctx* c) {
  if (!c->desc.precond_still_water) return;
  const std::vector<double> e = c->ef_h;
  std::fill(c->ef_h.begin(), c->ef_h.end(), 0.0);
  try {
    rebuild_levels(c);
  } catch (...) {
    c->ef_h = e;
    throw;
  }
  c->ef_h = e;
}

void setup3d_impl(Ctx* c, const sem_mesh_desc* d, const std::vector<int>& orders) {
  c->Nx = d->ne[0];
  c->Ny = d->ne[1];
  c->Nz = d->ne[2];
  if (c->Nx < 1 || c->Ny < 1 || c->Nz < 1) throw ArgFail{"ne must be positive"};
  if (d->len[1] <= 0) throw ArgFail{"len[1] must be positive"};
  if (orders[0] > 8) throw ArgFail{"3D supports orders up to 8"};
  const int NPf = orders[0] + 1;
  if (NPf * NPf * c->Nz > 1024) throw ArgFail{"(P+1)^2 * ne[2] must not exceed 1024 in 3D"};
  if (semk::apply3d_smem(orders[0], c->Nz, true) > 160 * 1024)
    throw ArgFail{"3D operator kernel exceeds LDS for this size"};
  const double N64 = (double)(c->Nx * orders[0] + 1) * (c->Ny * orders[0] + 1) *
                     (c->Nz * orders[0] + 1);
  if (N64 > 2.0e9) throw ArgFail{"problem too large"};
  const int cdm = d->coarse_dense_max > 0 ? d->coarse_dense_max : 1200;

  // level list: (order, Nx, Ny)
  struct LD { int P, Nx, Ny; };
  std::vector<LD> lds;
  for (int p : orders) lds.push_back({p, c->Nx, c->Ny});
  auto nodes = [&](const LD& l) {
    return (double)(l.Nx * l.P + 1) * (l.Ny * l.P + 1) * (c->Nz * l.P + 1);
  };
  while (c->masked && nodes(lds.back()) > cdm && lds.back().Nx % 2 == 0 && lds.back().Ny % 2 == 0 &&
         lds.size() < 16)
    lds.push_back({1, lds.back().Nx / 2, lds.back().Ny / 2});
  if (c->masked && nodes(lds.back()) > 20000)
    throw ArgFail{"3D coarse level too large for a dense solve (make ne[0], ne[1] divisible by "
                  "powers of 2)"};
  const int nl = (int)lds.size();
  const int Pf = orders[0];
  const int nyf = c->Ny * Pf + 1;
  c->lev.resize(nl);
  for (int l = 0; l < nl; ++l) {
    DLevel& L = c->lev[l];
    const LD& ld = lds[l];
    if (ld.Nx == c->Nx) {
      semh::build_level(L.geo, 3, c->Nx, c->Ny, c->Nz, ld.P, Pf, d->len[0], d->len[1], d->h,
                        d->eta);
    } else {  // h-coarsened P = 1 level: h, eta at its vertices (a subset of the fine samples)
      const int f = c->Nx / ld.Nx;
      std::vector<double> hs((size_t)(ld.Nx + 1) * (ld.Ny + 1)), es(hs.size());
      for (int ix = 0; ix <= ld.Nx; ++ix)
        for (int iy = 0; iy <= ld.Ny; ++iy) {
          const size_t src = (size_t)(ix * f * Pf) * nyf + (size_t)iy * f * Pf;
          hs[(size_t)ix * (ld.Ny + 1) + iy] = d->h[src];
          es[(size_t)ix * (ld.Ny + 1) + iy] = d->eta[src];
        }
      semh::build_level(L.geo, 3, ld.Nx, ld.Ny, c->Nz, 1, 1, d->len[0], d->len[1], hs.data(),
                        es.data());
    }
    L.P = ld.P;
    L.NP = L.P + 1;
    L.Nx = ld.Nx;
    L.Ny = ld.Ny;
    L.Nz = c->Nz;
    L.nxn = L.geo.nxn;
    L.nyn = L.geo.nyn;
    L.nzn = L.geo.nzn;
    L.N = (unsigned)L.geo.N;
    const bool coarsest = (l == nl - 1);
    L.dbl = coarsest || c->prec == SEM_F64;
    L.gt = level_gtype(c, L);
    std::vector<double> Gr = L.geo.G;
    if (L.gt == semk::G_F32)
      for (auto& v : Gr) v = (double)(float)v;
    else if (L.gt == semk::G_BF16)
      for (auto& v : Gr) v = semh::bf16_round(v);
    L.G = put_factors3d(c, L, L.geo, nullptr);
    std::vector<double> diag = semh::assembled_diag(L.geo, Gr, c->masked);
    std::vector<double> dinv(diag.size());
    for (size_t g = 0; g < diag.size(); ++g) dinv[g] = 1.0 / diag[g];
    if (L.dbl) L.dinv = upload(c, dinv);
    else L.dinv = upload(c, std::vector<float>(dinv.begin(), dinv.end()));
    const size_t eb = esz(L.dbl);
    L.x = dalloc(c, L.N * eb);
    L.b = dalloc(c, L.N * eb);
    L.d = dalloc(c, L.N * eb);
    L.y = dalloc(c, L.N * eb);
    L.Sx = dalloc(c, L.N * eb);
    L.Sy = dalloc(c, L.N * eb);
    L.Sxy = dalloc(c, L.N * eb);
    L.S = nullptr;
    L.nS = 0;
    if (!coarsest && d->smoother == SEM_SMOOTH_SCHWARZ) schwarz_setup(c, L, Gr);
    // order-1 levels above the coarsest: the assembled stencil (SEM_NO_STENCIL=1: the
    // matrix-free operator with its face fix-up)
    const char* ns = std::getenv("SEM_NO_STENCIL");
    if (!coarsest && L.P == 1 && c->masked && !(ns && ns[0] == '1') &&
        27.0 * L.N * 8.0 <= 2.0 * (1ull << 30))  // host assembly within 2 GiB
      stencil_setup(c, L, Gr);
  }
  // transfers and their temporaries
  size_t tmax = 1;
  for (int l = 0; l + 1 < nl; ++l) {
    DLevel& F = c->lev[l];
    DLevel& C = c->lev[l + 1];
    Rows1 px, py, pz;
    if (F.Nx == C.Nx) {
      const std::vector<double> J = semh::interp_matrix(C.geo.r, F.geo.r);
      px = prol1d_p(F.Nx, F.P, C.P, J);
      py = prol1d_p(F.Ny, F.P, C.P, J);
      pz = prol1d_p(F.Nz, F.P, C.P, J);
    } else {
      px = prol1d_h(C.Nx);
      py = prol1d_h(C.Ny);
      pz = ident1d(F.nzn);
    }
    upload_op(c, px, F.P1[0]);
    upload_op(c, py, F.P1[1]);
    upload_op(c, pz, F.P1[2]);
    upload_op(c, transpose1d(px, C.nxn), F.R1[0]);
    upload_op(c, transpose1d(py, C.nyn), F.R1[1]);
    upload_op(c, transpose1d(pz, C.nzn), F.R1[2]);
    tmax = std::max(tmax, (size_t)F.nxn * F.nyn * C.nzn);
    tmax = std::max(tmax, (size_t)F.nxn * C.nyn * C.nzn);
  }
  c->tA = (double*)dalloc(c, tmax * 8);
  c->tB = (double*)dalloc(c, tmax * 8);
  // outer FP64 operator: column records
  DLevel& L0 = c->lev[0];
  c->CG64 = upload(c, column_records3d(L0.geo));
  const size_t N = L0.N;
  c->xo = (double*)dalloc(c, N * 8);
  c->bo = (double*)dalloc(c, N * 8);
  c->ro = (double*)dalloc(c, N * 8);
  c->po = (double*)dalloc(c, N * 8);
  c->qo = (double*)dalloc(c, N * 8);
  c->zo = (double*)dalloc(c, N * 8);
  c->yo = (double*)dalloc(c, N * 8);
  c->Sxo = (double*)dalloc(c, N * 8);
  c->Syo = (double*)dalloc(c, N * 8);
  c->Sxyo = (double*)dalloc(c, N * 8);
  c->So = nullptr;
  c->parts = (double*)dalloc(c, (size_t)PS_NSETS * semk::NRED * 8);
  c->scal = (double*)dalloc(c, 64 * 8);
  HK(hipHostMalloc((void**)&c->hscal, 3 * (3 * semk::NRED + 8) * 8, hipHostMallocDefault));
  {  // lumped mass and Neumann faces of the fine level
    const semh::LevelGeom& G = L0.geo;
    const size_t NL3 = (size_t)G.NP * G.NP * G.NP;
    std::vector<double> m(N, 0.0);
    for (size_t e = 0; e < G.E; ++e)
      for (size_t l = 0; l < NL3; ++l) m[semh::local_to_global(G, e, (int)l)] += G.mass[e * NL3 + l];
    c->mass = upload(c, m);
    for (size_t f = 0; f < G.face_idx.size(); ++f) {
      std::vector<long long> idx(G.face_idx[f].begin(), G.face_idx[f].end());
      c->face_idx.push_back(upload(c, idx));
      c->face_w.push_back(upload(c, G.face_w[f]));
      c->face_n.push_back(idx.size());
    }
  }
  if (c->masked) {  // dense inverse of the masked coarsest operator
    DLevel& LC = c->lev.back();
    const semh::LevelGeom& G = LC.geo;
    const int n = (int)G.N;
    const size_t NL3 = (size_t)G.NP * G.NP * G.NP;
    std::vector<double> A((size_t)n * n, 0.0), Ae(NL3 * NL3);
    for (size_t e = 0; e < G.E; ++e) {
      semh::element_matrix(G, G.G, e, Ae.data());
      for (size_t a = 0; a < NL3; ++a) {
        const size_t ga = semh::local_to_global(G, e, (int)a);
        for (size_t b = 0; b < NL3; ++b)
          A[ga * n + semh::local_to_global(G, e, (int)b)] += Ae[a * NL3 + b];
      }
    }
    for (int g = 0; g < n; ++g)
      if (g % G.nzn == G.nzn - 1) {
        for (int k = 0; k < n; ++k) A[(size_t)g * n + k] = A[(size_t)k * n + g] = 0.0;
        A[(size_t)g * n + g] = 1.0;
      }
    std::vector<double> Ai((size_t)n * n);
    if (!semh::dense_inverse_public(n, A.data(), Ai.data()))
      throw ArgFail{"coarse operator is singular"};
    c->Ainv = upload(c, Ai);
    c->nAinv = n;
    for (int l = 0; l + 1 < nl; ++l) lanczos(c, l);
  }
  learned_geometry(c);
  c->dsurf = upload(c, surface_depths(c));
  still_water_levels(c);
  HK(hipStreamSynchronize(c->st));
}

void setup_impl(Ctx* c, const sem_mesh_desc* d) {
  c->desc = *d;
  c->desc.h = nullptr;
  c->desc.eta = nullptr;
  c->dim = d->dim;
  if (d->dim != 2 && d->dim != 3) throw ArgFail{"dim must be 2 or 3"};
  c->Nx = d->ne[0];
  c->Nz = d->ne[2];
  c->Ny = 1;
  if (c->Nx < 1 || c->Nz < 1) throw ArgFail{"ne must be positive"};
  if (d->order < 1 || d->order > SEM_MAX_ORDER) throw ArgFail{"order out of range"};
  if (!d->h || !d->eta) throw ArgFail{"h and eta are required"};
  if (d->len[0] <= 0) throw ArgFail{"len[0] must be positive"};
  c->masked = (d->dirichlet_faces & SEM_FACE_TOP) ? 1 : 0;
  c->prec = d->inner_prec;
  if (c->prec < SEM_F64 || c->prec > SEM_F32_GCOL) throw ArgFail{"bad inner_prec"};

  if (d->smoother != SEM_SMOOTH_JACOBI && d->smoother != SEM_SMOOTH_CHEBYSHEV &&
      d->smoother != SEM_SMOOTH_SCHWARZ)
    throw ArgFail{"bad smoother"};
  if (d->smoother == SEM_SMOOTH_SCHWARZ && d->order > 8)
    throw ArgFail{"the Schwarz smoother is built for orders <= 8"};
  if (d->schwarz_overlap < 0 || d->schwarz_overlap > 8)
    throw ArgFail{"schwarz_overlap out of range (0..8)"};
  if (d->order_z < 0 || d->order_z > SEM_MAX_ORDER) throw ArgFail{"order_z out of range"};
  if (d->dim == 3 && d->order_z != 0 && d->order_z != d->order)
    throw ArgFail{"3D meshes take one order (order_z 0 or equal to order)"};
  if (d->outer != SEM_OUTER_FPCG && d->outer != SEM_OUTER_PDC && d->outer != SEM_OUTER_GMRES)
    throw ArgFail{"bad outer"};
  if (d->outer == SEM_OUTER_GMRES && (d->gmres_restart < 1 || d->gmres_restart > semk::KRY_MAX))
    throw ArgFail{"GMRES restart must be 1..64"};
  if (d->smoother == SEM_SMOOTH_CHEBYSHEV &&
      (d->cheb_degree < 1 || d->cheb_degree_coarse < 0 || !(d->cheb_hi > d->cheb_lo) ||
       d->cheb_lo <= 0))
    throw ArgFail{"bad Chebyshev parameters"};
  if (d->smoother != SEM_SMOOTH_CHEBYSHEV && (d->nu_pre < 0 || d->nu_post < 0))
    throw ArgFail{"bad sweep counts"};
  std::vector<int> orders;   // x orders of the levels
  std::vector<int> orders_z; // sigma orders (2D)
  const bool semi = d->dim == 2 && d->order_z > 0 && d->order_z != d->order;
  if (d->nlevels <= 0) {
    if (semi) {  // semi-coarsening: the larger order drops until the two match, then both
      int px = d->order, pz = d->order_z;
      orders.push_back(px);
      orders_z.push_back(pz);
      while (px > 1 || pz > 1) {
        if (px == pz) px = pz = (px + 1) / 2;
        else if (px > pz) px = std::max((px + 1) / 2, pz);
        else pz = std::max((pz + 1) / 2, px);
        orders.push_back(px);
        orders_z.push_back(pz);
      }
      if ((int)orders.size() > SEM_MAX_LEVELS) throw ArgFail{"too many levels"};
    } else {
      orders.push_back(d->order);
      while (orders.back() > 1) orders.push_back((orders.back() + 1) / 2);
    }
  } else {
    if (d->nlevels > SEM_MAX_LEVELS) throw ArgFail{"too many levels"};
    for (int k = 0; k < d->nlevels; ++k) orders.push_back(d->level_order[k]);
    if (orders[0] != d->order) throw ArgFail{"level_order[0] must equal order"};
    if (semi || (d->dim == 2 && d->order_z > 0)) {
      for (int k = 0; k < d->nlevels; ++k) orders_z.push_back(d->level_order_z[k]);
      if (orders_z[0] != d->order_z) throw ArgFail{"level_order_z[0] must equal order_z"};
      if (orders.back() != 1 || orders_z.back() != 1) throw ArgFail{"last level orders must be 1"};
      for (size_t k = 1; k < orders.size(); ++k) {
        const int fx = orders[k - 1], fz = orders_z[k - 1], cx = orders[k], cz = orders_z[k];
        if (cx < 1 || cz < 1 || cx > fx || cz > fz || (cx == fx && cz == fz))
          throw ArgFail{"level orders must not grow and one of them must drop"};
        if (cx < fx && cz < fz && !(fx == fz && cx == cz))
          throw ArgFail{"both orders may drop together only between levels of equal orders"};
      }
    } else {
      if (orders.back() != 1) throw ArgFail{"last level order must be 1"};
      for (size_t k = 1; k < orders.size(); ++k)
        if (orders[k] >= orders[k - 1] || orders[k] < 1)
          throw ArgFail{"level orders must decrease"};
    }
  }
  for (size_t k = 0; k < orders.size(); ++k)
    if (orders[k] > SEM_MAX_ORDER || (k < orders_z.size() && orders_z[k] > SEM_MAX_ORDER))
      throw ArgFail{"level order out of range"};
  if (orders_z.empty()) orders_z = orders;
  bool any_rect = false;
  for (size_t k = 0; k < orders.size(); ++k) any_rect |= orders[k] != orders_z[k];
  if (any_rect && d->smoother == SEM_SMOOTH_SCHWARZ)
    throw ArgFail{"the Schwarz smoother needs equal orders along x and sigma"};
  {
    const size_t nh = d->dim == 2 ? (size_t)d->ne[0] * orders[0] + 1
                                  : ((size_t)d->ne[0] * orders[0] + 1) * ((size_t)d->ne[1] * orders[0] + 1);
    c->hf_h.assign(d->h, d->h + nh);
    c->ef_h.assign(d->eta, d->eta + nh);
    c->Pf = orders[0];
    c->len0 = d->len[0];
    c->len1 = d->dim == 3 ? d->len[1] : 1.0;
  }
  if (d->dim == 3) {
    c->ust = (hipStream_t)d->stream;
    HK(hipStreamCreate(&c->st));
    HK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    for (auto& e : c->ev_it) HK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const char* ng = std::getenv("SEM_NO_GRAPH");
    c->use_graphs = !(ng && ng[0] == '1');
    setup3d_impl(c, d, orders);
    return;
  }
  for (size_t k = 0; k < orders.size(); ++k) {
    if (orders[k] == orders_z[k] && (orders[k] + 1) * c->Nz > 1024)
      throw ArgFail{"(P+1)*ne[2] must not exceed 1024"};
    if (orders[k] != orders_z[k] &&
        !semk::apply2r_fits(orders[k], orders_z[k], c->Nz, true))
      throw ArgFail{"(P_x+1)*(P_sigma+1)*ne[2] must not exceed 1024 on levels with different "
                    "orders"};
  }
  if (c->Nz > 256) throw ArgFail{"ne[2] too large for the coarse solve"};
  const double N64 = (double)(c->Nx * orders[0] + 1) * (c->Nz * orders_z[0] + 1);
  if (N64 > 2.0e9) throw ArgFail{"problem too large"};

  c->ust = (hipStream_t)d->stream;
  HK(hipStreamCreate(&c->st));
  HK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
  HK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
  for (auto& e : c->ev_it) HK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  const char* ng = std::getenv("SEM_NO_GRAPH");
  c->use_graphs = !(ng && ng[0] == '1');

  // SEM_NO_FUSED_STEP=1: every 2D smoother step as operator + element-wise update (the fused
  // step, its two-step entry form and the one-kernel coarse smoothing are then not used)
  const char* nfs = std::getenv("SEM_NO_FUSED_STEP");
  const bool no_fused_step = nfs && nfs[0] == '1';
  const int nl = (int)orders.size();
  c->lev.resize(nl);
  for (int l = 0; l < nl; ++l) {
    DLevel& L = c->lev[l];
    semh::build_level(L.geo, 2, c->Nx, 1, c->Nz, orders[l], orders[0], d->len[0], 1.0, d->h,
                      d->eta, orders_z[l]);
    L.P = orders[l];
    L.NP = L.P + 1;
    L.Pz = orders_z[l];
    L.rect = L.Pz != L.P;
    if (L.rect) {
      L.Dx = upload(c, L.geo.D);
      L.Dz = upload(c, L.geo.Dz);
    }
    L.Nx = c->Nx;
    L.Nz = c->Nz;
    L.nxn = L.geo.nxn;
    L.nzn = L.geo.nzn;
    L.N = (unsigned)L.geo.N;
    const bool coarsest = (l == nl - 1);
    L.dbl = coarsest || c->prec == SEM_F64;
    L.gt = level_gtype(c, L);
    // factors in storage precision; the diagonal is built from the same rounded values
    std::vector<double> Gr = L.geo.G;
    if (L.gt == semk::G_F32)
      for (auto& v : Gr) v = (double)(float)v;
    else if (L.gt == semk::G_BF16)
      for (auto& v : Gr) v = semh::bf16_round(v);
    L.G = put_factors(c, L, L.geo, nullptr);
    std::vector<double> diag = semh::assembled_diag(L.geo, Gr, c->masked);
    std::vector<double> dinv(diag.size());
    for (size_t g = 0; g < diag.size(); ++g) dinv[g] = 1.0 / diag[g];
    if (L.dbl) L.dinv = upload(c, dinv);
    else L.dinv = upload(c, std::vector<float>(dinv.begin(), dinv.end()));
    const size_t eb = esz(L.dbl);
    L.x = dalloc(c, L.N * eb);
    L.b = dalloc(c, L.N * eb);
    L.d = dalloc(c, L.N * eb);
    L.y = dalloc(c, L.N * eb);
    L.nS = (size_t)(c->Nx + 1) * L.nzn;
    L.S = dalloc(c, L.nS * eb);
    if (!coarsest && !L.rect && L.P <= 8 && semk::cheb2d_cpb(L.P, L.Nx, L.Nz, L.dbl) > 0 &&
        !no_fused_step)
      L.xalt = dalloc(c, L.N * eb);
    if (!coarsest && d->smoother == SEM_SMOOTH_SCHWARZ) schwarz_setup(c, L, Gr);
  }
  for (int l = 0; l + 1 < nl; ++l) {
    DLevel& F = c->lev[l];
    DLevel& C = c->lev[l + 1];
    if (F.P != C.P && F.Pz != C.Pz) {  // both directions (equal orders on both levels)
      F.J = upload(c, semh::interp_matrix(C.geo.r, F.geo.r));
      if (semk::restrict2d_smem(F.P, C.P, c->Nz, F.dbl) > 160 * 1024 ||
          semk::prolong2d_smem(F.P, C.P, c->Nz, F.dbl) > 160 * 1024)
        throw ArgFail{"transfer kernels exceed LDS for this size"};
      continue;
    }
    // one direction: 1D interpolation along it, its transpose for the restriction
    F.axis = F.P != C.P ? 0 : 2;
    const bool ax = F.axis == 0;
    const int Ne = ax ? c->Nx : c->Nz, pf = ax ? F.P : F.Pz, pc = ax ? C.P : C.Pz;
    const std::vector<double> J =
        semh::interp_matrix(ax ? C.geo.r : C.geo.rz, ax ? F.geo.r : F.geo.rz);
    const Rows1 Pr = prol1d_p(Ne, pf, pc, J);
    upload_op(c, Pr, F.P1[F.axis]);
    upload_op(c, transpose1d(Pr, Ne * pc + 1), F.R1[F.axis]);
  }
  // coarse levels whose smoothing sequences run as one kernel each (SEM_NO_COARSE_FUSED=1: none)
  {
    const char* nf = std::getenv("SEM_NO_COARSE_FUSED");
    const bool off = nf && nf[0] == '1';
    for (int l = 1; !off && l + 1 < nl; ++l) {
      DLevel& L = c->lev[l];
      const DLevel& C = c->lev[l + 1];
      if (!L.xalt || L.axis >= 0 || C.rect || !semk::coarse2d_supported(L.P, C.P)) continue;
      semk::CoarseSeq sq;
      int apre = 0, apost = 0;
      if (!coarse_seq(c, l, true, &sq, &apre)) continue;
      const int npre = sq.ns;
      if (!coarse_seq(c, l, false, &sq, &apost)) continue;
      const int npost = sq.ns;
      // one launch per sequence where the window fits, else two (the first writes x and d)
      auto plans = [&](bool pre, int ns, int applies, semk::CoarsePlan* p1, semk::CoarsePlan* p2,
                       int* k1) {
        const int fl = pre ? semk::CO_RESTRICT : semk::CO_PROLONG;
        *p1 = semk::coarse2d_plan(L.P, C.P, c->Nz, L.dbl, fl, applies);
        *p2 = semk::CoarsePlan();
        *k1 = 0;
        // one launch wherever its window owns two columns or more (a second launch costs more
        // than the recomputation it saves there, measured at degrees 3 and 6); else the sequence
        // splits after step a: pre, steps 0 .. a-1 from x = 0 (a - 1 applies), then the rest and
        // the residual; post, the prolongation and steps 0 .. a-1, then the rest, at the split
        // with the least recomputed work (applies times window slots per owned column, summed
        // over the two launches; one owned column among twelve slots recomputes far more)
        if (p1->W >= 2 || ns < 2) return;
        double best = p1->W >= 1 ? std::max(applies, 1) * (double)p1->nslot / p1->W : 1e300;
        for (int a = 1; a < ns; ++a) {
          semk::CoarsePlan q1, q2;
          int n1, n2;
          if (pre) {
            n1 = a - 1;
            n2 = ns - a + 1;
            q1 = semk::coarse2d_plan(L.P, C.P, c->Nz, L.dbl, 0, n1);
            q2 = semk::coarse2d_plan(L.P, C.P, c->Nz, L.dbl, semk::CO_RESTRICT, n2);
          } else {
            n1 = a;
            n2 = ns - a;
            q1 = semk::coarse2d_plan(L.P, C.P, c->Nz, L.dbl, semk::CO_PROLONG, n1);
            q2 = semk::coarse2d_plan(L.P, C.P, c->Nz, L.dbl, 0, n2);
          }
          if (q1.W < 1 || q2.W < 1) continue;
          const double cost = std::max(n1, 1) * (double)q1.nslot / q1.W +
                              std::max(n2, 1) * (double)q2.nslot / q2.W;
          if (cost < best) {
            best = cost;
            *p1 = q1;
            *p2 = q2;
            *k1 = a;
          }
        }
        if (*k1 == 0 && best >= 1e300) *p1 = semk::CoarsePlan();
      };
      plans(true, npre, apre, &L.cpre, &L.cpre2, &L.cpre_k1);
      plans(false, npost, apost, &L.cpost, &L.cpost2, &L.cpost_k1);
    }
  }
  if (!c->lev[0].rect && semk::apply2d_smem(orders[0], c->Nz, true) > 160 * 1024)
    throw ArgFail{"operator kernel exceeds LDS for this size"};
  // outer FP64 operator: column records (equal orders) or stored factors (two orders)
  DLevel& L0 = c->lev[0];
  if (L0.rect) {
    if (L0.dbl) c->G64 = (double*)L0.G;
    else c->G64 = upload(c, layout_G2<double>(L0.geo, L0.geo.G, [](double v) { return v; }));
  } else {
    c->CG64 = upload(c, column_records(L0.geo));
  }
  const size_t N = L0.N;
  c->xo = (double*)dalloc(c, N * 8);
  c->bo = (double*)dalloc(c, N * 8);
  c->ro = (double*)dalloc(c, N * 8);
  c->po = (double*)dalloc(c, N * 8);
  c->qo = (double*)dalloc(c, N * 8);
  c->zo = (double*)dalloc(c, N * 8);
  c->yo = (double*)dalloc(c, N * 8);
  c->So = (double*)dalloc(c, L0.nS * 8);
  c->parts = (double*)dalloc(c, (size_t)PS_NSETS * semk::NRED * 8);
  c->scal = (double*)dalloc(c, 64 * 8);
  HK(hipHostMalloc((void**)&c->hscal, 3 * (3 * semk::NRED + 8) * 8, hipHostMallocDefault));
  // lumped mass and Neumann faces of the fine level
  {
    std::vector<double> m(N, 0.0);
    const semh::LevelGeom& G = L0.geo;
    const size_t NL = (size_t)G.NP * G.NPz;
    for (size_t e = 0; e < G.E; ++e)
      for (size_t l = 0; l < NL; ++l)
        m[semh::local_to_global(G, e, (int)l)] += G.mass[e * NL + l];
    c->mass = upload(c, m);
    for (size_t f = 0; f < G.face_idx.size(); ++f) {
      std::vector<long long> idx(G.face_idx[f].begin(), G.face_idx[f].end());
      c->face_idx.push_back(upload(c, idx));
      c->face_w.push_back(upload(c, G.face_w[f]));
      c->face_n.push_back(idx.size());
    }
  }
  learned_geometry(c);
  // coarse factorisation
  {
    DLevel& LC = c->lev.back();
    char eb[256] = {0};
    if (c->masked) {
      if (!semh::build_bcr(LC.geo, LC.geo.G, c->plan, eb, sizeof eb)) throw ArgFail{eb};
      c->bcrF = upload(c, c->plan.fwd.empty() ? std::vector<double>(1, 0.0) : c->plan.fwd);
      c->bcrB = upload(c, c->plan.bwd.empty() ? std::vector<double>(1, 0.0) : c->plan.bwd);
      c->bcrLast = upload(c, c->plan.last);
      c->bcrDense = upload(c, c->plan.dense);
      c->rowmap = upload(c, c->plan.rowmap);
      // one launch per direction where the level table and the LDS windows fit
      const int nlv = (int)c->plan.levs.size();
      c->bcrLv.nl = -1;
      const int nbp = c->plan.nb;
      const char* nf = std::getenv("SEM_NO_BCR_FUSED");  // 1: the per-level kernels
      const bool nb_ok = !(nf && nf[0] == '1') && nbp <= 64;
      if (nb_ok && nlv <= semk::BCR_MAXL && semk::bcr_fwd_all_smem(nlv, c->plan.nb) <= 65536 &&
          semk::bcr_bwd_all_smem(nlv, c->plan.nb) <= 65536) {
        c->bcrLv.nl = nlv;
        for (int l = 0; l < nlv; ++l) {
          c->bcrLv.offM[l] = (long long)c->plan.levs[l].offM;
          c->bcrLv.offB[l] = (long long)c->plan.levs[l].offB;
        }
        c->bcrRed = (double*)dalloc(c, (size_t)LC.N * sizeof(double));
      }
    }
  }
  // lambda_hat per smoothed level
  if (c->masked)
    for (int l = 0; l + 1 < nl; ++l) lanczos(c, l);
  c->dsurf = upload(c, surface_depths(c));
  still_water_levels(c);
  HK(hipStreamSynchronize(c->st));
}

// stream ordering with the caller
void enter(Ctx* c) {
  HK(hipEventRecord(c->ev_in, c->ust));
  HK(hipStreamWaitEvent(c->st, c->ev_in, 0));
}
void leave(Ctx* c) {
  HK(hipEventRecord(c->ev_out, c->st));
  HK(hipStreamWaitEvent(c->ust, c->ev_out, 0));
}

template <typename F>
sem_status guarded(Ctx* c, F body) {
  if (!c) return SEM_ERR_ARG;
  if (c->sticky) {
    return SEM_ERR_HIP;
  }
  try {
    c->err.clear();
    return body();
  } catch (const HipFail& f) {
    c->sticky = true;
    c->err = std::string("HIP error in ") + f.what + ": " + hipGetErrorString(f.e);
    return SEM_ERR_HIP;
  } catch (const ArgFail& a) {
    c->err = a.msg;
    return SEM_ERR_ARG;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return SEM_ERR_ALLOC;
  } catch (...) {
    c->err = "unexpected internal error";
    return SEM_ERR_STATE;
  }
}

void release(Ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  drop_graphs(c);
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->hscal) (void)hipHostFree(c->hscal);
  c->hscal = nullptr;
  if (c->hkpart) (void)hipHostFree(c->hkpart);
  c->hkpart = nullptr;
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  c->ev_in = c->ev_out = nullptr;
  for (auto& e : c->ev_it) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (c->st) (void)hipStreamDestroy(c->st);
  c->st = nullptr;
}

}  // namespace

struct sem_ctx {
  Ctx c;
};

static thread_local char g_setup_err[512] = {0};

static Ctx* C(sem_ctx* p) { return p ? &p->c : nullptr; }
static const Ctx* C(const sem_ctx* p) { return p ? &p->c : nullptr; }

extern "C" {

void sem_mesh_desc_default(sem_mesh_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->dim = 2;
  d->ne[0] = d->ne[1] = d->ne[2] = 1;
  d->order = 4;
  d->nlevels = 0;
  d->len[0] = d->len[1] = 1.0;
  d->dirichlet_faces = SEM_FACE_TOP;
  d->inner_prec = SEM_F64;
  d->smoother = SEM_SMOOTH_CHEBYSHEV;
  d->nu_pre = 2;
  d->nu_post = 2;
  d->cheb_degree = 3;
  d->jacobi_omega = 2.0 / 3.0;
  d->cheb_lo = 0.1;
  d->cheb_hi = 1.1;
  d->outer = SEM_OUTER_FPCG;
  d->maxit = 500;
  d->lanczos_steps = 20;
  d->lanczos_seed = 12345ull;
  d->stream = nullptr;
  d->coarse_dense_max = 1200;
  d->gmres_restart = 30;
}

sem_status sem_mesh_setup(const sem_mesh_desc* desc, sem_ctx** out) {
  if (!desc || !out) return SEM_ERR_ARG;
  *out = nullptr;
  sem_ctx* h = nullptr;
  g_setup_err[0] = 0;
  try {
    h = new sem_ctx();
  } catch (...) {
    return SEM_ERR_ALLOC;
  }
  Ctx* c = &h->c;
  try {
    setup_impl(c, desc);
  } catch (const HipFail& f) {
    std::snprintf(g_setup_err, sizeof g_setup_err, "HIP error in %s: %s", f.what,
                  hipGetErrorString(f.e));
    release(c);
    delete h;
    return SEM_ERR_HIP;
  } catch (const ArgFail& a) {
    std::snprintf(g_setup_err, sizeof g_setup_err, "%s", a.msg.c_str());
    release(c);
    delete h;
    return SEM_ERR_ARG;
  } catch (const std::bad_alloc&) {
    std::snprintf(g_setup_err, sizeof g_setup_err, "host allocation failed");
    release(c);
    delete h;
    return SEM_ERR_ALLOC;
  }
  *out = h;
  return SEM_OK;
}

void sem_destroy(sem_ctx* ctx) {
  if (!ctx) return;
  release(&ctx->c);
  delete ctx;
}

sem_status sem_get_sizes(const sem_ctx* ctx, size_t* n_global, size_t* n_free, size_t* n_local) {
  const Ctx* c = C(ctx);
  if (!c) return SEM_ERR_ARG;
  const DLevel& L = c->lev[0];
  if (n_global) *n_global = L.N;
  if (n_free) *n_free = L.N - (c->masked ? (size_t)L.nxn * L.nyn : 0);
  if (n_local)
    *n_local = L.geo.E * (c->dim == 2 ? (size_t)L.geo.NP * L.geo.NPz : (size_t)std::pow(L.NP, 3));
  return SEM_OK;
}

sem_status sem_get_level(const sem_ctx* ctx, int level, int* order, size_t* n, double* lam) {
  const Ctx* c = C(ctx);
  if (!c) return SEM_ERR_ARG;
  if (level < 0 || level >= (int)c->lev.size()) return SEM_ERR_ARG;
  const DLevel& L = c->lev[level];
  if (order) *order = L.P;
  if (n) *n = L.N;
  if (lam) *lam = L.lam;
  return SEM_OK;
}

sem_status sem_get_level_orders(const sem_ctx* ctx, int level, int* order_x, int* order_z) {
  const Ctx* c = C(ctx);
  if (!c) return SEM_ERR_ARG;
  if (level < 0 || level >= (int)c->lev.size()) return SEM_ERR_ARG;
  const DLevel& L = c->lev[level];
  if (order_x) *order_x = L.P;
  if (order_z) *order_z = c->dim == 2 ? L.Pz : L.P;
  return SEM_OK;
}

int sem_num_levels(const sem_ctx* ctx) {
  const Ctx* c = C(ctx);
  return c ? (int)c->lev.size() : 0;
}

sem_status sem_gll(int P, double* nodes, double* weights) {
  if (P < 1 || P > 64) return SEM_ERR_ARG;
  std::vector<double> r, w;
  semh::gll_rule(P, r, w);
  if (nodes) std::memcpy(nodes, r.data(), r.size() * 8);
  if (weights) std::memcpy(weights, w.data(), w.size() * 8);
  return SEM_OK;
}

sem_status sem_node_coords(const sem_ctx* ctx, int level, double* x, double* y, double* z) {
  const Ctx* c = C(ctx);
  if (!c) return SEM_ERR_ARG;
  if (level < 0 || level >= (int)c->lev.size()) return SEM_ERR_ARG;
  const semh::LevelGeom& G = c->lev[level].geo;
  if (x) std::memcpy(x, G.X.data(), G.N * 8);
  if (y && !G.Y.empty()) std::memcpy(y, G.Y.data(), G.N * 8);
  if (z && level > 0) std::memcpy(z, G.Z.data(), G.N * 8);
  if (z && level == 0) {  // current surface: z = -h + sigma (h + eta) on each vertical line
    const int Ps = c->dim == 2 ? G.Pz : G.P, nzn = G.nzn;  // order along sigma
    const std::vector<double>& rs = c->dim == 2 ? G.rz : G.r;
    std::vector<double> sig(nzn);
    for (int iz = 0; iz < nzn; ++iz) {
      const int ez = iz == nzn - 1 ? G.Nz - 1 : iz / Ps, j = iz - ez * Ps;
      sig[iz] = (ez + (rs[j] + 1.0) / 2.0) / G.Nz;
    }
    for (size_t col = 0; col < c->hf_h.size(); ++col)
      for (int iz = 0; iz < nzn; ++iz)
        z[col * nzn + iz] = -c->hf_h[col] + sig[iz] * (c->hf_h[col] + c->ef_h[col]);
  }
  return SEM_OK;
}

sem_status sem_apply_laplacian(sem_ctx* ctx, const double* x, double* y) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!x || !y || x == y) throw ArgFail{"x, y must be distinct device pointers"};
    enter(c);
    apply_outer(c, x, c->masked);
    DLevel& L = c->lev[0];
    HK(semk::fix_ax(true, c->yo, c->So, y, 1, L.N, L.nzn, L.P, c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_apply_level(sem_ctx* ctx, int level, const double* x, double* y) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (level < 0 || level >= (int)c->lev.size()) throw ArgFail{"bad level"};
    if (!x || !y || x == y) throw ArgFail{"x, y must be distinct device pointers"};
    enter(c);
    DLevel& L = c->lev[level];
    HK(semk::cast_to(L.dbl, x, L.d, L.N, c->st));
    apply_level(c, level, L.d, c->masked);
    HK(semk::fix_ax(L.dbl, L.y, L.S, y, 1, L.N, L.nzn, L.P, c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_pmg_vcycle(sem_ctx* ctx, const double* r, double* z) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!c->masked) return SEM_ERR_STATE;
    if (!r || !z) throw ArgFail{"null vector"};
    enter(c);
    DLevel& L0 = c->lev[0];
    vcycle(c, r);
    HK(semk::cast_from(L0.dbl, L0.x, z, L0.N, c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_solve_bytes(sem_ctx* ctx, const double* rhs, double* x, double tol,
                           double* bytes, int* iters, long* launches) {
  Ctx* c = C(ctx);
  if (!c) return SEM_ERR_ARG;
  if (!bytes) return SEM_ERR_ARG;
  // the same solve with every launch issued directly (no graph replays), each launch wrapper
  // adding its algorithmic bytes
  const bool g = c->use_graphs;
  {
    sem_status st0 = guarded(c, [&]() {
      HK(hipStreamSynchronize(c->st));
      drop_graphs(c);
      return SEM_OK;
    });
    if (st0 != SEM_OK) return st0;
  }
  c->use_graphs = false;
  sem_solve_info inf{};
  semk::acct_enable(true);
  const sem_status st = sem_poisson_solve(ctx, rhs, x, tol, &inf);
  semk::acct_enable(false);
  c->use_graphs = g;
  long n = 0;
  *bytes = semk::acct_total(&n);
  if (iters) *iters = inf.iters;
  if (launches) *launches = n;
  return st;
}

sem_status sem_set_smoother_bounds(sem_ctx* ctx, int level, double lambda_hat) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (level < 0 || level + 1 >= (int)c->lev.size()) throw ArgFail{"bad level"};
    if (!(lambda_hat > 0) || !std::isfinite(lambda_hat)) throw ArgFail{"bad lambda_hat"};
    HK(hipStreamSynchronize(c->st));
    c->lev[level].lam = lambda_hat;
    drop_graphs(c);
    return SEM_OK;
  });
}

sem_status sem_restrict(sem_ctx* ctx, int level, const double* b, const double* x, double* rc) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (level < 0 || level + 1 >= (int)c->lev.size()) throw ArgFail{"bad level"};
    if (!b || !rc) throw ArgFail{"null vector"};
    enter(c);
    DLevel& F = c->lev[level];
    DLevel& Cc = c->lev[level + 1];
    HK(semk::cast_to(F.dbl, b, F.b, F.N, c->st));
    if (x) {
      HK(semk::cast_to(F.dbl, x, F.x, F.N, c->st));
      apply_level(c, level, F.x, c->masked);
    }
    restrict_to(c, level, x != nullptr);
    HK(semk::cast_from(Cc.dbl, Cc.b, rc, Cc.N, c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_prolong_add(sem_ctx* ctx, int level, const double* ec, double* xf) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (level < 0 || level + 1 >= (int)c->lev.size()) throw ArgFail{"bad level"};
    if (!ec || !xf) throw ArgFail{"null vector"};
    enter(c);
    DLevel& F = c->lev[level];
    DLevel& Cc = c->lev[level + 1];
    HK(semk::cast_to(Cc.dbl, ec, Cc.x, Cc.N, c->st));
    HK(semk::cast_to(F.dbl, xf, F.x, F.N, c->st));
    prolong_from(c, level);
    HK(semk::cast_from(F.dbl, F.x, xf, F.N, c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_smooth(sem_ctx* ctx, int level, int pre, const double* b, double* x) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (level < 0 || level + 1 >= (int)c->lev.size()) throw ArgFail{"bad level"};
    if (!b || !x) throw ArgFail{"null vector"};
    enter(c);
    DLevel& L = c->lev[level];
    HK(semk::cast_to(L.dbl, b, L.b, L.N, c->st));
    if (!pre) HK(semk::cast_to(L.dbl, x, L.x, L.N, c->st));
    smooth(c, level, pre != 0);
    HK(semk::cast_from(L.dbl, L.x, x, L.N, c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_coarse_solve(sem_ctx* ctx, const double* b, double* x) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!c->masked) return SEM_ERR_STATE;
    if (!b || !x) throw ArgFail{"null vector"};
    enter(c);
    DLevel& L = c->lev.back();
    HK(hipMemcpyAsync(L.b, b, L.N * 8, hipMemcpyDeviceToDevice, c->st));
    coarse_solve(c);
    HK(hipMemcpyAsync(x, L.x, L.N * 8, hipMemcpyDeviceToDevice, c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_assemble_rhs(sem_ctx* ctx, const double* f, const double* gN, const double* gD,
                            double* rhs) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!rhs) throw ArgFail{"null rhs"};
    enter(c);
    DLevel& L = c->lev[0];
    const unsigned N = L.N;
    HK(semk::rhs_mass(c->mass, f, rhs, N, c->st));
    if (gN) {
      size_t off = 0;
      for (size_t k = 0; k < c->face_idx.size(); ++k) {
        HK(semk::rhs_face(c->face_idx[k], c->face_w[k], gN + off, rhs, (unsigned)c->face_n[k],
                          c->st));
        off += c->face_n[k];
      }
    }
    if (c->masked) {
      if (gD) {
        HK(semk::fill(true, c->zo, 0.0, N, c->st));
        HK(semk::scatter_top(c->zo, gD, L.nxn * L.nyn, L.nzn, c->st));
        apply_outer(c, c->zo, 0);
        HK(semk::rhs_lift(rhs, c->yo, c->So, gD, N, L.nzn, L.P, c->st));
      } else {
        HK(semk::scatter_top(rhs, nullptr, L.nxn * L.nyn, L.nzn, c->st));
      }
    }
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_poisson_solve(sem_ctx* ctx, const double* rhs, double* x, double tol,
                             sem_solve_info* info) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    const auto t0 = std::chrono::steady_clock::now();
    if (!c->masked) return SEM_ERR_STATE;
    if (!rhs || !x || rhs == x) throw ArgFail{"rhs and x must be distinct device pointers"};
    if (!(tol >= 0)) throw ArgFail{"bad tol"};
    if (c->mixed && c->desc.outer == SEM_OUTER_FPCG) {
      set_err(c, "the mixed-stage operator is not symmetric: use GMRES or PDC");
      return SEM_ERR_STATE;
    }
    sem_solve_info loc{};
    sem_solve_info* inf = info ? info : &loc;
    std::memset(inf, 0, sizeof(*inf));
    enter(c);
    DLevel& L0 = c->lev[0];
    const unsigned N = L0.N;
    if (c->stage_alloc) HK(hipMemsetAsync(c->stage.skips, 0, sizeof(int), c->st));
    HK(hipMemcpyAsync(c->bo, rhs, (size_t)N * 8, hipMemcpyDeviceToDevice, c->st));
    HK(hipMemcpyAsync(c->xo, x, (size_t)N * 8, hipMemcpyDeviceToDevice, c->st));
    HK(semk::copy_top(c->xo, c->bo, L0.nxn * L0.nyn, L0.nzn, c->st));
    apply_outer(c, c->xo, c->masked);
    HK(semk::resid64(c->bo, c->yo, c->So, c->ro, pset(c, PS_RR), pset(c, PS_BB), N, L0.nzn, L0.P,
                     c->st));
    const bool fpcg = c->desc.outer == SEM_OUTER_FPCG;
    const size_t nset = 3 * (size_t)semk::NRED + 1;  // sets RR, BB, PQ and the skip counter
    double sums[3];
    // the initial residual's partial sums go to the host behind an event, and the first two
    // iterations are enqueued before the host looks at them (no GPU idle time at the start);
    // when the initial guess turns out to satisfy the tolerance already (or the right-hand side
    // is zero or not finite), their results are discarded: x keeps the caller's values
    double* hinit = c->hscal + 2 * nset;
    HK(hipMemcpyAsync(hinit, c->parts, nset * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HK(hipEventRecord(c->ev_it[2], c->st));
    // Each iteration's partial sums go to pinned host memory behind an event.  While the
    // residual trend says the iteration in flight cannot reach tol (its predicted residual is
    // above twice tol), the next iteration is enqueued before the host waits, so the GPU does not
    // idle between iterations.  A wrong guess runs one more iteration, which only improves x;
    // the reported count is the number executed and the loop stops only with rel <= tol.
    auto enqueue = [&](int k) {
      const bool first = (k == 0);
      const int hs = k & 1;  // host slot of this iteration's partial sums
      auto body = [&]() {
        if (fpcg) fpcg_iteration(c, first);
        else pdc_iteration(c);
        HK(hipMemcpyAsync(c->hscal + hs * nset, c->parts, nset * sizeof(double),
                          hipMemcpyDeviceToHost, c->st));
      };
      if (c->use_graphs) {
        hipGraphExec_t* slot = fpcg ? (first ? &c->g_first : &c->g_iter[hs]) : &c->g_pdc[hs];
        if (!*slot) *slot = capture(c, body);
        HK(hipGraphLaunch(*slot, c->st));
      } else {
        body();
      }
      HK(hipEventRecord(c->ev_it[hs], c->st));
    };
    int skips_seen = 0;  // rejection counter at the last collected iteration
    auto collect = [&](int k) {
      HK(hipEventSynchronize(c->ev_it[k & 1]));
      const double* h = c->hscal + (k & 1) * nset;
      for (int s = 0; s < 3; ++s) {
        double v = 0.0;
        for (int j = 0; j < semk::NRED; ++j) v += h[s * semk::NRED + j];
        sums[s] = v;
      }
      skips_seen = *reinterpret_cast<const int*>(h + 3 * semk::NRED);
    };
    // the learned stage is switched off for the rest of the solve after this many iterations in
    // a row in which the judge rejected every application (the plain V-cycle remains)
    constexpr int kStageOffAfter = 3;
    const bool stage_on = c->stage_alloc && c->stage.enabled;
    const int per_it = stage_on ? ((c->stage_mode & 1) + ((c->stage_mode >> 1) & 1)) : 0;
    int rejected_run = 0, skips_prev = 0;
    bool stage_off = false;
    int it = 0, launched = 0;
    const bool gmres = c->desc.outer == SEM_OUTER_GMRES;
    const int spec = gmres ? 0 : std::min(2, std::max(0, c->desc.maxit));
    while (launched < spec) enqueue(launched++);
    HK(hipEventSynchronize(c->ev_it[2]));
    for (int q = 0; q < 3; ++q) {
      double v = 0.0;
      for (int j = 0; j < semk::NRED; ++j) v += hinit[q * semk::NRED + j];
      sums[q] = v;
    }
    const double bb = sums[PS_BB];
    double rel = bb > 0 ? std::sqrt(sums[PS_RR] / bb) : 0.0;
    auto push = [&](double v) {
      if (inf->nhist < 512) inf->hist[inf->nhist++] = v;
    };
    push(rel);
    sem_status st = SEM_OK;
    bool keep_x = false;  // the caller's x is the answer: discard the iterations in flight
    if (!std::isfinite(bb) || !std::isfinite(sums[PS_RR])) {
      st = SEM_ERR_BREAKDOWN;
      set_err(c, "non-finite right-hand side or initial residual");
      keep_x = true;
    } else if (bb == 0.0 || rel <= tol) {
      keep_x = true;  // converged initial guess; zero right-hand side: zero solution below
    }
    if (st != SEM_OK || keep_x) {
      for (int k = 0; k < launched; ++k) HK(hipEventSynchronize(c->ev_it[k & 1]));
      launched = 0;
      if (bb == 0.0 && st == SEM_OK) {
        HK(semk::fill(true, c->xo, 0.0, N, c->st));
        rel = 0.0;
        keep_x = false;  // x = 0 is copied out below
      } else if (c->stage_alloc) {
        HK(hipMemsetAsync(c->stage.skips, 0, sizeof(int), c->st));
      }
    }
    // restarted right-preconditioned GMRES: Arnoldi steps z_j = B v_j, w = A z_j, classical
    // Gram-Schmidt against V twice, Givens rotations on the host; x += Z y closes a cycle, and
    // the cycle's true residual decides whether another one follows
    auto gmres_run = [&]() {
      const int m = c->desc.gmres_restart;
      const size_t Nn = N;
      constexpr int NR = semk::NRED;
      if (!c->kV) {
        c->kV = (double*)dalloc(c, (size_t)(m + 1) * Nn * 8);
        c->kZ = (double*)dalloc(c, (size_t)m * Nn * 8);
        c->kpart = (double*)dalloc(c, (size_t)(m + 2) * NR * 8);
        c->kcoef = (double*)dalloc(c, (size_t)(3 * (semk::KRY_MAX + 2)) * 8);
        HK(hipHostMalloc((void**)&c->hkpart, (size_t)(m + 2) * NR * 8, hipHostMallocDefault));
      }
      double* kh1 = c->kcoef;                            // [KRY_MAX + 2]
      double* kh2 = c->kcoef + (semk::KRY_MAX + 2);      // [KRY_MAX + 2]
      double* kcol = c->kcoef + 2 * (semk::KRY_MAX + 2); // [KRY_MAX + 2]: ||w||^2, then the column
      double* kww = kh2 + semk::KRY_MAX + 1;
      const double nb = std::sqrt(bb);
      double beta = rel * nb;
      std::vector<double> Hm((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
      auto H = [&](int i, int j) -> double& { return Hm[(size_t)i * m + j]; };
      while (st == SEM_OK && rel > tol && it < c->desc.maxit) {
        HK(hipMemcpyAsync(c->kV, c->ro, Nn * 8, hipMemcpyDeviceToDevice, c->st));
        HK(semk::kry_scale(c->kV, 1.0 / beta, N, c->st));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && it < c->desc.maxit; ++j) {
          double* vj = c->kV + (size_t)j * Nn;
          double* zj = c->kZ + (size_t)j * Nn;
          double* w = c->kV + (size_t)(j + 1) * Nn;
          vcycle(c, vj);
          HK(semk::castdot(L0.dbl, L0.x, zj, nullptr, vj, pset(c, PS_ZQ), pset(c, PS_RZB), N,
                           c->st));
          apply_outer(c, zj, c->masked);
          HK(semk::kry_first(c->yo, c->So, w, c->kV, Nn, j + 1, c->kpart, N, L0.nzn, L0.P,
                             c->st));
          // classical Gram-Schmidt twice with the coefficients kept on the device; the host
          // reads the finished column once per step (enqueuing the next step before that wait
          // was measured slower: the step run past the end of each cycle costs more than the
          // wait it hides at these sizes)
          HK(semk::kry_sums(c->kpart, j + 1, kh1, c->st));
          HK(semk::kry_sub_dev(w, c->kV, Nn, j + 1, kh1, 1, c->kpart, N, c->st));
          HK(semk::kry_sums(c->kpart, j + 1, kh2, c->st));
          HK(semk::kry_sub_dev(w, c->kV, Nn, j + 1, kh2, 0, c->kpart, N, c->st));
          HK(semk::kry_sums(c->kpart + (size_t)(j + 1) * NR, 1, kww, c->st));
          HK(semk::kry_finish(w, kww, kh1, kh2, j, kcol, N, c->st));
          HK(hipMemcpyAsync(c->hkpart, kcol, (size_t)(j + 2) * 8, hipMemcpyDeviceToHost, c->st));
          HK(hipStreamSynchronize(c->st));
          const double hn = c->hkpart[j + 1];
          for (int i = 0; i <= j; ++i) H(i, j) = c->hkpart[i];
          H(j + 1, j) = hn;
          if (!std::isfinite(hn)) {
            st = SEM_ERR_BREAKDOWN;
            set_err(c, "breakdown in GMRES (non-finite Arnoldi vector)");
            return;
          }
          for (int i = 0; i < j; ++i) {  // earlier rotations on the new column
            const double t = cs[i] * H(i, j) + sn[i] * H(i + 1, j);
            H(i + 1, j) = -sn[i] * H(i, j) + cs[i] * H(i + 1, j);
            H(i, j) = t;
          }
          const double den = std::hypot(H(j, j), H(j + 1, j));
          cs[j] = den > 0.0 ? H(j, j) / den : 1.0;
          sn[j] = den > 0.0 ? H(j + 1, j) / den : 0.0;
          H(j, j) = den;
          H(j + 1, j) = 0.0;
          g[j + 1] = -sn[j] * g[j];
          g[j] = cs[j] * g[j];
          ++it;
          ++k;
          inf->vcycles++;
          push(std::fabs(g[j + 1]) / nb);
          if (std::fabs(g[j + 1]) / nb <= tol || hn == 0.0) break;
        }
        semk::KryCoef yc;
        for (int i = k - 1; i >= 0; --i) {  // y = R^-1 g
          double v = g[i];
          for (int q = i + 1; q < k; ++q) v -= H(i, q) * yc.h[q];
          yc.h[i] = H(i, i) != 0.0 ? v / H(i, i) : 0.0;
        }
        HK(semk::kry_update(c->xo, c->kZ, Nn, k, yc, N, c->st));
        apply_outer(c, c->xo, c->masked);
        HK(semk::resid64(c->bo, c->yo, c->So, c->ro, pset(c, PS_RR), pset(c, PS_BB), N, L0.nzn,
                         L0.P, c->st));
        read_sums(c, sums);
        rel = std::sqrt(sums[PS_RR] / bb);
        beta = std::sqrt(sums[PS_RR]);
        if (inf->nhist > 0) inf->hist[inf->nhist - 1] = rel;  // the cycle's true residual
        if (!std::isfinite(rel)) {
          st = SEM_ERR_BREAKDOWN;
          set_err(c, "breakdown in GMRES (non-finite residual)");
        }
      }
      if (st == SEM_OK && rel > tol) {
        st = SEM_ERR_NOT_CONVERGED;
        set_err(c, "maximum number of outer iterations reached");
      }
    };
    if (gmres && st == SEM_OK && !keep_x && rel > tol) gmres_run();
    double rel_prev = -1.0;  // residual one iteration back (for the rate), < 0: unknown
    while (!gmres && st == SEM_OK && (rel > tol || launched > it)) {
      if (rel > tol) {
        if (it >= c->desc.maxit) {
          st = SEM_ERR_NOT_CONVERGED;
          set_err(c, "maximum number of outer iterations reached");
          break;
        }
        if (launched == it) enqueue(launched++);
        if (launched == it + 1 && launched < c->desc.maxit && rel_prev > 0.0 &&
            rel * (rel / rel_prev) > 2.0 * tol)
          enqueue(launched++);
      }
      collect(it);
      ++it;
      inf->vcycles++;
      rel_prev = rel;
      rel = std::sqrt(sums[PS_RR] / bb);
      push(rel);
      if (stage_on && !stage_off && per_it > 0) {
        rejected_run = (skips_seen - skips_prev >= per_it) ? rejected_run + 1 : 0;
        skips_prev = skips_seen;
        if (rejected_run >= kStageOffAfter && rel > tol) {
          // iterations already enqueued keep the stage; later ones are captured without it
          HK(hipStreamSynchronize(c->st));
          drop_graphs(c);
          c->stage.enabled = false;
          stage_off = true;
          inf->stage_off_at = it;
        }
      }
      if (!std::isfinite(rel) || (fpcg && !(sums[PS_PQ] > 0))) {
        st = SEM_ERR_BREAKDOWN;
        set_err(c, "breakdown in the outer iteration (non-finite residual or p.Ap <= 0)");
      }
    }
    while (launched > it) {  // after a breakdown: let the iteration in flight finish
      collect(it);
      ++it;
      inf->vcycles++;
    }
    if (!keep_x) HK(hipMemcpyAsync(x, c->xo, (size_t)N * 8, hipMemcpyDeviceToDevice, c->st));
    leave(c);
    HK(hipStreamSynchronize(c->st));
    inf->iters = it;
    inf->rel_res = rel;
    if (stage_off) {  // the next solve starts with the stage again (graphs captured anew)
      drop_graphs(c);
      c->stage.enabled = true;
    }
    if (stage_on) {
      int sk = 0;
      HK(hipMemcpy(&sk, c->stage.skips, sizeof(int), hipMemcpyDeviceToHost));
      inf->learned_skips = sk;
    }
    inf->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return st;
  });
}

static thread_local std::string g_mlp_err;

size_t sem_mlp_blob_size(int nin, int nout) {
  if (nin < 1 || nout < 1) return 0;
  return semm::blob_size(nin, nout);
}

static void stage_buffers(Ctx* c) {
  if (c->stage_alloc) return;
  DLevel& L = c->lev[0];
  const int n = c->dim == 3 ? L.NP * L.NP * L.NP : L.NP * L.NP;
  const size_t E = L.geo.E;
  semm::Stage& s = c->stage;
  s.dim = c->dim;
  s.P = L.P;
  s.Nx = L.Nx;
  s.Ny = c->dim == 3 ? L.Ny : 1;
  s.Nz = L.Nz;
  s.nyn = c->dim == 3 ? L.nyn : 1;
  s.nzn = L.nzn;
  s.E = E;
  s.nout = n;
  s.nin = (c->dim == 3 ? 7 : 5) * n;
  const int KR = semm::pad16(n), N3 = semm::pad16(n);
  s.W1r = (uint16_t*)dalloc(c, (size_t)KR * semm::NH * 2);
  s.W2 = (uint16_t*)dalloc(c, (size_t)semm::NH * semm::NH * 2);
  s.W3 = (uint16_t*)dalloc(c, (size_t)semm::NH * N3 * 2);
  s.b2 = (float*)dalloc(c, semm::NH * 4);
  s.b3 = (float*)dalloc(c, (size_t)N3 * 4);
  s.Z1geo = (float*)dalloc(c, E * semm::NH * 4);
  s.abar = upload(c, c->abar_h);
  s.CE = (float*)dalloc(c, E * n * 4);
  s.skips = reinterpret_cast<int*>(c->parts + (size_t)PS_SKIP * semk::NRED);
  const size_t eb = esz(L.dbl);
  c->Rbuf = dalloc(c, L.N * eb);
  c->cbuf = dalloc(c, L.N * eb);
  c->yq = dalloc(c, L.N * eb);
  c->Sq = c->dim == 2 ? dalloc(c, L.nS * eb) : nullptr;
  const size_t ncq = c->dim == 2 ? (size_t)std::max(semk::apply2d_blocks(L.P, L.Nx, L.Nz, L.dbl),
                                                    semk::cheb2d_blocks(L.P, L.Nx, L.Nz, L.dbl))
                                 : (size_t)semk::NRED;
  c->stparts = (double*)dalloc(c, ((size_t)semm::stage_mlp_blocks(E) + ncq) * 8);
  c->stage_alloc = true;
}

// inverses of the element blocks R_e A R_e^T of the masked assembled fine operator (host FP64)
// 3D: R_e A R_e^T from the element matrices of e and its (up to 26) neighbours, each entry the
// sum over the hexahedra that hold both nodes; surface rows and columns masked; then inverted
static std::vector<double> element_block_inverses3d(Ctx* c) {
  const semh::LevelGeom& G = c->lev[0].geo;
  const int NP = G.NP, P = G.P, n = NP * NP * NP;
  const size_t E = G.E, nn = (size_t)n * n;
  const int Nx = G.Nx, Ny = G.Ny, Nz = G.Nz;
  std::vector<double> Ae(E * nn);
  parallel_ranges(E, [&](size_t lo, size_t hi) {
    for (size_t e = lo; e < hi; ++e) semh::element_matrix(G, G.G, e, &Ae[e * nn]);
  }, 2);
  std::vector<double> out(E * nn);
  std::atomic<bool> singular{false};
  parallel_ranges(E, [&](size_t lo, size_t hi) {
    std::vector<double> Ab(nn), Ai(nn);
    std::vector<int> map(n);
    for (size_t e = lo; e < hi; ++e) {
      const int ez = (int)(e % Nz), exy = (int)(e / Nz), ey = exy % Ny, ex = exy / Ny;
      std::fill(Ab.begin(), Ab.end(), 0.0);
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            const int fx = ex + dx, fy = ey + dy, fz = ez + dz;
            if (fx < 0 || fx >= Nx || fy < 0 || fy >= Ny || fz < 0 || fz >= Nz) continue;
            const size_t f = ((size_t)fx * Ny + fy) * Nz + fz;
            // local index in e of each node of f (-1: not in e)
            for (int l = 0; l < n; ++l) {
              const int i = l / (NP * NP) + dx * P, m = (l / NP) % NP + dy * P, j = l % NP + dz * P;
              map[l] = (i >= 0 && i <= P && m >= 0 && m <= P && j >= 0 && j <= P)
                           ? (i * NP + m) * NP + j
                           : -1;
            }
            const double* A = &Ae[f * nn];
            for (int a = 0; a < n; ++a) {
              if (map[a] < 0) continue;
              for (int b = 0; b < n; ++b)
                if (map[b] >= 0) Ab[(size_t)map[a] * n + map[b]] += A[(size_t)a * n + b];
            }
          }
      if (c->masked && ez == Nz - 1)
        for (int a = 0; a < n; ++a)
          if (a % NP == P)
            for (int b = 0; b < n; ++b) {
              Ab[(size_t)a * n + b] = Ab[(size_t)b * n + a] = 0.0;
            }
      if (c->masked && ez == Nz - 1)
        for (int a = 0; a < n; ++a)
          if (a % NP == P) Ab[(size_t)a * n + a] = 1.0;
      if (!semh::dense_inverse_public(n, Ab.data(), Ai.data())) singular = true;
      std::copy(Ai.begin(), Ai.end(), out.begin() + e * nn);
    }
  }, 2);
  if (singular) throw ArgFail{"singular element block"};
  return out;
}

static std::vector<double> element_block_inverses(Ctx* c) {
  if (c->dim == 3) return element_block_inverses3d(c);
  const semh::LevelGeom& G = c->lev[0].geo;
  const int NP = G.NP, n = NP * NP;
  const size_t E = G.E;
  auto gidx = [&](size_t e, int l) {
    const size_t ex = e / G.Nz, ez = e % G.Nz;
    return (ex * G.P + l / NP) * (size_t)G.nzn + ez * G.P + l % NP;
  };
  auto top = [&](size_t g) { return c->masked && (g % G.nzn) == (size_t)(G.nzn - 1); };
  // assembled entries between nodes of one element, keyed by (gi, gj)
  std::vector<std::pair<uint64_t, double>> ent;
  std::vector<double> Ae((size_t)n * n);
  for (size_t e = 0; e < E; ++e) {
    semh::element_matrix(G, G.G, e, Ae.data());
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        const uint64_t gi = gidx(e, a), gj = gidx(e, b);
        ent.push_back({gi * (uint64_t)G.N + gj, Ae[(size_t)a * n + b]});
      }
  }
  std::sort(ent.begin(), ent.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  std::vector<std::pair<uint64_t, double>> asm_;
  for (const auto& p : ent) {
    if (!asm_.empty() && asm_.back().first == p.first) asm_.back().second += p.second;
    else asm_.push_back(p);
  }
  auto lookup = [&](uint64_t key) {
    auto it = std::lower_bound(asm_.begin(), asm_.end(), std::make_pair(key, -1e300),
                               [](const auto& x, const auto& y) { return x.first < y.first; });
    return (it != asm_.end() && it->first == key) ? it->second : 0.0;
  };
  std::vector<double> out(E * (size_t)n * n), Ab((size_t)n * n), Ai((size_t)n * n);
  for (size_t e = 0; e < E; ++e) {
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        const uint64_t gi = gidx(e, a), gj = gidx(e, b);
        double v = lookup(gi * (uint64_t)G.N + gj);
        if (top(gi) || top(gj)) v = (gi == gj) ? 1.0 : 0.0;
        Ab[(size_t)a * n + b] = v;
      }
    if (!semh::dense_inverse_public(n, Ab.data(), Ai.data()))
      throw ArgFail{"singular element block"};
    std::copy(Ai.begin(), Ai.end(), out.begin() + e * (size_t)n * n);
  }
  return out;
}

static std::vector<uint16_t> bf16_vec(const float* p, size_t rows, size_t cols, size_t prow,
                                      size_t pcol) {
  std::vector<uint16_t> out(prow * pcol, 0);
  for (size_t r = 0; r < rows; ++r)
    for (size_t q = 0; q < cols; ++q) out[r * pcol + q] = semh::bf16_bits(p[r * cols + q]);
  return out;
}

}  // extern "C"

// internal: load a network into the stage (see sem_learned_load); keeps a copy of the blob
static void learned_load_impl(Ctx* c, const void* blob, size_t nbytes, int enable) {
  semm::Net net;
  std::string e;
  if (!semm::net_from_blob(blob, nbytes, net, e)) throw ArgFail{e};
  DLevel& L = c->lev[0];
  const bool d3 = c->dim == 3;
  const int n = d3 ? L.NP * L.NP * L.NP : L.NP * L.NP;
  const int nfg = d3 ? 6 : 4;  // geometric feature blocks (factor fields and mass)
  if (!d3 && (L.rect || L.axis >= 0))
    throw ArgFail{"learned stage needs equal orders along x and sigma on the fine level and the "
                  "next"};
  if (!d3 && n > semm::MAX_STAGE_OUT) throw ArgFail{"learned stage needs fine order P <= 8"};
  if (d3 && L.P > semm::MAX_STAGE_P3) throw ArgFail{"learned stage on hexahedra needs fine order P <= 6"};
  if (net.nin != (1 + nfg) * n || net.nout != n) throw ArgFail{"network sizes do not match the mesh"};
  if (c->lev.size() < 2) throw ArgFail{"learned stage needs at least two levels"};
  HK(hipStreamSynchronize(c->st));
  stage_buffers(c);
  semm::Stage& s = c->stage;
  const int NH = semm::NH, KR = semm::pad16(n), N3 = semm::pad16(n), K4 = semm::pad16(nfg * n);
  const size_t E = s.E, Mp = (E + 15) / 16 * 16;
  auto put16 = [&](uint16_t* dst, const std::vector<uint16_t>& h) {
    HK(hipMemcpy(dst, h.data(), h.size() * 2, hipMemcpyHostToDevice));
  };
  // transposed (output-major) copies for the inference kernel
  auto transpose = [](const float* W, int rows, int cols) {
    std::vector<float> T((size_t)rows * cols);
    for (int r = 0; r < rows; ++r)
      for (int q = 0; q < cols; ++q) T[(size_t)q * rows + r] = W[(size_t)r * cols + q];
    return T;
  };
  // MFMA A-operand fragment order of an output-major [M][K] matrix (M, K multiples of 16):
  // fragment (t, k) = rows 16t.., columns 16k.., as 64 lanes x 4 values, lane l holding row
  // 16t + l%16, columns 16k + 4(l/16) + 0..3 (one contiguous 8-byte read per lane)
  auto frag = [](const std::vector<uint16_t>& W, int M, int K) {
    std::vector<uint16_t> F(W.size());
    size_t o = 0;
    for (int t = 0; t < M / 16; ++t)
      for (int k = 0; k < K / 16; ++k)
        for (int l = 0; l < 64; ++l)
          for (int v = 0; v < 4; ++v)
            F[o++] = W[(size_t)(16 * t + l % 16) * K + 16 * k + 4 * (l / 16) + v];
    return F;
  };
  put16(s.W1r, frag(bf16_vec(transpose(net.W1.data(), n, NH).data(), NH, n, NH, KR), NH, KR));
  put16(s.W2, frag(bf16_vec(transpose(net.W2.data(), NH, NH).data(), NH, NH, NH, NH), NH, NH));
  put16(s.W3, frag(bf16_vec(transpose(net.W3.data(), NH, n).data(), n, NH, N3, NH), N3, NH));
  HK(hipMemcpy(s.b2, net.b2.data(), NH * 4, hipMemcpyHostToDevice));
  std::vector<float> b3(N3, 0.f);
  std::copy(net.b3.begin(), net.b3.end(), b3.begin());
  HK(hipMemcpy(s.b3, b3.data(), N3 * 4, hipMemcpyHostToDevice));
  // Z1geo = Xg W1g + b1 (geometric part of layer 1), computed once per mesh on the GPU
  std::vector<uint16_t> xg = bf16_vec(c->geo_h.data(), E, nfg * n, Mp, K4);
  // W1g output-major [NH x K4], so that the product reads k-contiguous fragments of both operands
  std::vector<uint16_t> w1g =
      bf16_vec(transpose(net.W1.data() + (size_t)n * NH, nfg * n, NH).data(), NH, nfg * n, NH, K4);
  void *dx = nullptr, *dw = nullptr, *dz = nullptr, *db = nullptr;
  HK(hipMalloc(&dx, xg.size() * 2));
  HK(hipMalloc(&dw, w1g.size() * 2));
  HK(hipMalloc(&dz, Mp * NH * 4));
  HK(hipMalloc(&db, NH * 4));
  HK(hipMemcpy(dx, xg.data(), xg.size() * 2, hipMemcpyHostToDevice));
  HK(hipMemcpy(dw, w1g.data(), w1g.size() * 2, hipMemcpyHostToDevice));
  HK(hipMemcpy(db, net.b1.data(), NH * 4, hipMemcpyHostToDevice));
  HK(semm::gemm_bf16((const uint16_t*)dx, K4, 1, (const uint16_t*)dw, 1, K4, (float*)dz, NH,
                     (int)Mp, NH, K4, 0, c->st));
  HK(semm::add_bias((float*)dz, (const float*)db, (int)Mp, NH, c->st));
  HK(hipMemcpyAsync(s.Z1geo, dz, E * NH * 4, hipMemcpyDeviceToDevice, c->st));
  HK(hipStreamSynchronize(c->st));
  HK(hipFree(dx));
  HK(hipFree(dw));
  HK(hipFree(dz));
  HK(hipFree(db));
  s.enabled = (enable & 3) != 0;
  c->stage_mode = (enable & 3) ? (enable & 3) : 1;
  drop_graphs(c);
  c->stage_blob.assign((const uint8_t*)blob, (const uint8_t*)blob + nbytes);
}


// ---------------------------------------------------------------------------------------------
// surface update
// ---------------------------------------------------------------------------------------------
// sum of the GLL weights of the elements sharing each 1D node (Ne elements of order P)
static std::vector<double> shared_weights(int Ne, int P, const std::vector<double>& w) {
  std::vector<double> W((size_t)Ne * P + 1, 0.0);
  for (int e = 0; e < Ne; ++e)
    for (int a = 0; a <= P; ++a) W[(size_t)e * P + a] += w[a];
  return W;
}

// geometry of level l for the current column samples
static void level_geometry(Ctx* c, int l, semh::LevelGeom& geo) {
  DLevel& L = c->lev[l];
  if (c->dim == 2) {
    semh::build_level(geo, 2, c->Nx, 1, c->Nz, L.P, c->Pf, c->len0, 1.0, c->hf_h.data(),
                      c->ef_h.data(), L.Pz);
    return;
  }
  if (L.Nx == c->Nx) {
    semh::build_level(geo, 3, c->Nx, c->Ny, c->Nz, L.P, c->Pf, c->len0, c->len1, c->hf_h.data(),
                      c->ef_h.data());
    return;
  }
  const int f = c->Nx / L.Nx, nyf = c->Ny * c->Pf + 1;
  std::vector<double> hs((size_t)(L.Nx + 1) * (L.Ny + 1)), es(hs.size());
  for (int ix = 0; ix <= L.Nx; ++ix)
    for (int iy = 0; iy <= L.Ny; ++iy) {
      const size_t src = (size_t)(ix * f * c->Pf) * nyf + (size_t)iy * f * c->Pf;
      hs[(size_t)ix * (L.Ny + 1) + iy] = c->hf_h[src];
      es[(size_t)ix * (L.Ny + 1) + iy] = c->ef_h[src];
    }
  semh::build_level(geo, 3, L.Nx, L.Ny, c->Nz, 1, 1, c->len0, c->len1, hs.data(), es.data());
}

template <typename T>
static void copy_to(Ctx* c, void* dst, const std::vector<T>& h) {
  HK(hipMemcpy(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

// the outer FP64 operator, the lumped mass and the wall-face weights of the fine level for the
// current surface (the V-cycle keeps its own factors)
static void update_outer(Ctx* c) {
  DLevel& L0 = c->lev[0];
  const size_t N = L0.N;
  if (c->dsurf) copy_to(c, c->dsurf, surface_depths(c));
  if (c->G64 && (void*)c->G64 == L0.G) {  // FP64 inner levels share the fine factors: split them
    const size_t n = c->dim == 2
                         ? (L0.rect ? 3 * L0.geo.E * (size_t)L0.geo.NP * L0.geo.NPz
                                    : semk::g2d_layout(L0.P, c->Nz, 8).cstride * c->Nx)
                         : semk::g3d_layout(L0.P, c->Nz, 8).cstride * (size_t)c->Nx * c->Ny;
    c->G64 = (double*)dalloc(c, n * 8);
  }
  const std::vector<double>& w = L0.geo.w;
  const double dsig = 1.0 / c->Nz;
  const std::vector<double> Wz = shared_weights(c->Nz, L0.P, w);
  if (c->dim == 2) {
    semh::LevelGeom geo;
    level_geometry(c, 0, geo);
    if (c->CG64) copy_to(c, c->CG64, column_records(geo));
    else copy_to(c, c->G64, layout_G2<double>(geo, geo.G, [](double v) { return v; }));
    std::vector<double> m(N, 0.0);
    const size_t NL = (size_t)geo.NP * geo.NPz;
    for (size_t e = 0; e < geo.E; ++e)
      for (size_t l = 0; l < NL; ++l) m[semh::local_to_global(geo, e, (int)l)] += geo.mass[e * NL + l];
    copy_to(c, c->mass, m);
    for (size_t f = 0; f < geo.face_w.size() && f < c->face_w.size(); ++f)
      copy_to(c, c->face_w[f], geo.face_w[f]);
    return;
  }
  // 3D: on the device from the column samples
  const size_t nh = c->hf_h.size();
  if (!c->hf_d) {
    c->hf_d = upload(c, c->hf_h);
    c->ef_d = (double*)dalloc(c, nh * 8);
    c->r_d = upload(c, L0.geo.r);
    c->w_d = upload(c, w);
    c->Wx_d = upload(c, shared_weights(c->Nx, L0.P, w));
    c->Wy_d = upload(c, shared_weights(c->Ny, L0.P, w));
    c->Wz_d = upload(c, Wz);
  }
  copy_to(c, c->ef_d, c->ef_h);
  const double dx = c->len0 / c->Nx, dy = c->len1 / c->Ny;
  HK(semk::colrec3d(L0.P, c->hf_d, c->ef_d, c->CG64, c->Nx, c->Ny, c->Nz, dx, dy, c->st));
  HK(semk::mass3d(c->hf_d, c->ef_d, c->Wx_d, c->Wy_d, c->Wz_d, c->mass, L0.nyn, L0.nzn, N,
                  dx * dy * dsig / 8.0, c->st));
  // wall faces (x = 0, x = Lx: [iy][iz]; y = 0, y = Ly: [ix][iz]); the bottom depends on h only
  const std::vector<double> Wx = shared_weights(c->Nx, L0.P, w), Wy = shared_weights(c->Ny, L0.P, w);
  const int nxn = L0.nxn, nyn = L0.nyn, nzn = L0.nzn;
  auto dcol = [&](int ix, int iy) { return c->hf_h[(size_t)ix * nyn + iy] + c->ef_h[(size_t)ix * nyn + iy]; };
  for (int f = 0; f < 2 && f < (int)c->face_w.size(); ++f) {
    const int ix = f == 0 ? 0 : nxn - 1;
    std::vector<double> fw((size_t)nyn * nzn);
    for (int iy = 0; iy < nyn; ++iy)
      for (int iz = 0; iz < nzn; ++iz)
        fw[(size_t)iy * nzn + iz] = (dy / 2.0) * (dsig / 2.0) * dcol(ix, iy) * Wy[iy] * Wz[iz];
    copy_to(c, c->face_w[f], fw);
  }
  for (int f = 0; f < 2 && 2 + f < (int)c->face_w.size(); ++f) {
    const int iy = f == 0 ? 0 : nyn - 1;
    std::vector<double> fw((size_t)nxn * nzn);
    for (int ix = 0; ix < nxn; ++ix)
      for (int iz = 0; iz < nzn; ++iz)
        fw[(size_t)ix * nzn + iz] = (dx / 2.0) * (dsig / 2.0) * dcol(ix, iy) * Wx[ix] * Wz[iz];
    copy_to(c, c->face_w[2 + f], fw);
  }
}

// every level of the V-cycle rebuilt for the current surface: factors, inverse diagonals, the
// coarse solve, lambda_hat (and the learned stage's geometry, when a network is loaded)
static void rebuild_levels(Ctx* c) {
  const int nl = (int)c->lev.size();
  for (int l = 0; l < nl; ++l) {
    DLevel& L = c->lev[l];
    semh::LevelGeom geo;
    level_geometry(c, l, geo);
    L.geo = std::move(geo);
    std::vector<double> Gr = L.geo.G;
    if (L.gt == semk::G_F32)
      for (auto& v : Gr) v = (double)(float)v;
    else if (L.gt == semk::G_BF16)
      for (auto& v : Gr) v = semh::bf16_round(v);
    if (c->dim == 2) {
      put_factors(c, L, L.geo, L.G);
    } else {
      put_factors3d(c, L, L.geo, L.G);
    }
    std::vector<double> diag = semh::assembled_diag(L.geo, Gr, c->masked);
    std::vector<double> dinv(diag.size());
    for (size_t g = 0; g < diag.size(); ++g) dinv[g] = 1.0 / diag[g];
    if (L.dbl) copy_to(c, L.dinv, dinv);
    else copy_to(c, L.dinv, std::vector<float>(dinv.begin(), dinv.end()));
    if (L.Ainv_s) schwarz_setup(c, L, Gr, true);
    if (L.st27) stencil_setup(c, L, Gr);
  }
  if (c->masked) {
    DLevel& LC = c->lev.back();
    if (c->dim == 2) {
      semh::BcrPlan plan;
      char eb[256] = {0};
      if (!semh::build_bcr(LC.geo, LC.geo.G, plan, eb, sizeof eb)) throw ArgFail{eb};
      if (plan.fwd.size() != c->plan.fwd.size() || plan.bwd.size() != c->plan.bwd.size() ||
          plan.dense.size() != c->plan.dense.size() || plan.last.size() != c->plan.last.size())
        throw ArgFail{"coarse factorisation changed shape"};
      if (!plan.fwd.empty()) copy_to(c, c->bcrF, plan.fwd);
      if (!plan.bwd.empty()) copy_to(c, c->bcrB, plan.bwd);
      copy_to(c, c->bcrLast, plan.last);
      copy_to(c, c->bcrDense, plan.dense);
      c->plan = std::move(plan);
    } else {
      const semh::LevelGeom& G = LC.geo;
      const int n = (int)G.N;
      const size_t NL3 = (size_t)G.NP * G.NP * G.NP;
      std::vector<double> A((size_t)n * n, 0.0), Ae(NL3 * NL3);
      for (size_t e = 0; e < G.E; ++e) {
        semh::element_matrix(G, G.G, e, Ae.data());
        for (size_t a = 0; a < NL3; ++a) {
          const size_t ga = semh::local_to_global(G, e, (int)a);
          for (size_t b = 0; b < NL3; ++b)
            A[ga * n + semh::local_to_global(G, e, (int)b)] += Ae[a * NL3 + b];
        }
      }
      for (int g = 0; g < n; ++g)
        if (g % G.nzn == G.nzn - 1) {
          for (int k = 0; k < n; ++k) A[(size_t)g * n + k] = A[(size_t)k * n + g] = 0.0;
          A[(size_t)g * n + g] = 1.0;
        }
      std::vector<double> Ai((size_t)n * n);
      if (!semh::dense_inverse_public(n, A.data(), Ai.data())) throw ArgFail{"coarse operator is singular"};
      copy_to(c, c->Ainv, Ai);
    }
    for (int l = 0; l + 1 < nl; ++l) lanczos(c, l);
  }
  {
    learned_geometry(c);
    c->geo_d = nullptr;   // re-uploaded (and element-block inverses recomputed) on next use
    c->ainv_d = nullptr;
    if (c->stage_alloc) copy_to(c, c->stage.abar, c->abar_h);
    if (c->stage_alloc && !c->stage_blob.empty()) {
      const std::vector<uint8_t> blob = c->stage_blob;
      learned_load_impl(c, blob.data(), blob.size(), c->stage.enabled ? c->stage_mode : 0);
    }
  }
}

extern "C" {

sem_status sem_mesh_update_surface(sem_ctx* ctx, const double* eta, int refresh_precond) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!eta) throw ArgFail{"null eta"};
    for (size_t k = 0; k < c->ef_h.size(); ++k)
      if (!(c->hf_h[k] + eta[k] > 0.0)) throw ArgFail{"h + eta must stay positive"};
    HK(hipStreamSynchronize(c->st));
    std::copy(eta, eta + c->ef_h.size(), c->ef_h.begin());
    const double* g64 = c->G64;
    update_outer(c);
    // the captured iteration graphs read the rebuilt data in place; only a rebuild of the levels
    // or a newly split outer factor array changes what they point to
    const bool rebuild = refresh_precond && !c->desc.precond_still_water;
    if (rebuild) rebuild_levels(c);
    const bool was_mixed = c->mixed;
    c->mixed = false;  // a new surface ends the mixed-stage form (same-stage operator again)
    if (rebuild || c->G64 != g64 || was_mixed) drop_graphs(c);
    HK(hipStreamSynchronize(c->st));
    return SEM_OK;
  });
}

sem_status sem_mesh_mixed_stage(sem_ctx* ctx, const double* eta_prev) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (c->dim != 2) throw ArgFail{"the mixed-stage operator is built for 2D meshes"};
    HK(hipStreamSynchronize(c->st));
    if (!eta_prev) {
      if (c->mixed) drop_graphs(c);
      c->mixed = false;
      return SEM_OK;
    }
    for (size_t k = 0; k < c->ef_h.size(); ++k)
      if (!(c->hf_h[k] + eta_prev[k] > 0.0)) throw ArgFail{"h + eta_prev must stay positive"};
    const DLevel& L0 = c->lev[0];
    semh::LevelGeom gk, gp;  // stage k (current surface) and stage k-1
    semh::build_level(gk, 2, c->Nx, 1, c->Nz, L0.P, c->Pf, c->len0, 1.0, c->hf_h.data(),
                      c->ef_h.data(), L0.Pz);
    semh::build_level(gp, 2, c->Nx, 1, c->Nz, L0.P, c->Pf, c->len0, 1.0, c->hf_h.data(),
                      eta_prev, L0.Pz);
    // G_rr = w d_k dsig/dx, G_rs = w d_k sx_(k-1), G_ss = w (dx/dsig) d_k (sx_k sx_(k-1) +
    // 1/(d_k d_(k-1))), G_sr = w d_k sx_k, per node (e, i, j); sx = (h_x - sigma d_x)/d
    const int NP = gk.NP, NPz = gk.NPz, Nz = c->Nz;
    const size_t nloc = (size_t)NP * NPz, nthr = nloc * Nz;
    const double dx = c->len0 / c->Nx, dsig = 1.0 / Nz;
    std::vector<double> G(4 * nthr * c->Nx);
    for (int ex = 0; ex < c->Nx; ++ex) {
      std::vector<double> dk(NP), dp(NP), hx(NP), dxk(NP), dxp(NP);
      for (int i = 0; i < NP; ++i) {
        const size_t q = (size_t)ex * NP + i;
        dk[i] = gk.col_h[q] + gk.col_eta[q];
        dp[i] = gp.col_h[q] + gp.col_eta[q];
      }
      for (int i = 0; i < NP; ++i) {
        double a = 0, b = 0, e2 = 0;
        for (int k = 0; k < NP; ++k) {
          a += gk.D[i * NP + k] * gk.col_h[(size_t)ex * NP + k];
          b += gk.D[i * NP + k] * dk[k];
          e2 += gk.D[i * NP + k] * dp[k];
        }
        hx[i] = 2.0 / dx * a;
        dxk[i] = 2.0 / dx * b;
        dxp[i] = 2.0 / dx * e2;
      }
      for (int ez = 0; ez < Nz; ++ez)
        for (int i = 0; i < NP; ++i)
          for (int j = 0; j < NPz; ++j) {
            const double sig = (ez + (gk.rz[j] + 1.0) / 2.0) / Nz;
            const double sk = (hx[i] - sig * dxk[i]) / dk[i];
            const double sp = (hx[i] - sig * dxp[i]) / dp[i];
            const double w = gk.w[i] * gk.wz[j];
            const size_t t = (size_t)ez * nloc + (size_t)i * NPz + j;
            double* gc = &G[(size_t)ex * 4 * nthr];
            gc[0 * nthr + t] = w * dk[i] * dsig / dx;
            gc[1 * nthr + t] = w * dk[i] * sp;
            gc[2 * nthr + t] = w * (dx / dsig) * dk[i] * (sk * sp + 1.0 / (dk[i] * dp[i]));
            gc[3 * nthr + t] = w * dk[i] * sk;
          }
    }
    if (!semk::apply2r_fits(L0.P, L0.Pz, Nz, true))
      throw ArgFail{"the mixed-stage operator needs (P_x+1)(P_z+1) ne[2] <= 1024"};
    if (!c->Gmix) {
      c->Gmix = (double*)dalloc(c, G.size() * 8);
      c->Dmx = upload(c, gk.D);
      c->Dmz = upload(c, gk.Dz);
    }
    copy_to(c, c->Gmix, G);
    c->mixed = true;
    drop_graphs(c);
    HK(hipStreamSynchronize(c->st));
    return SEM_OK;
  });
}

// ---- stage loop -------------------------------------------------------------------------------
// five-stage fourth-order 2N-storage coefficients (Carpenter and Kennedy 1994, solution 3)
static const double kLserkA[5] = {0.0, -567301805773.0 / 1357537059087.0,
                                  -2404267990393.0 / 2016746695238.0,
                                  -3550918686646.0 / 2091501179385.0,
                                  -1275806237668.0 / 842570457699.0};
static const double kLserkB[5] = {1432997174477.0 / 9575080441755.0,
                                  5161836677717.0 / 13612068292357.0,
                                  1720146321549.0 / 2090206949498.0,
                                  3134564353537.0 / 4481467310338.0,
                                  2277821191437.0 / 14882151754819.0};
static const double kLserkC[5] = {0.0, 1432997174477.0 / 9575080441755.0,
                                  2526269341429.0 / 6820363962896.0,
                                  2006345519317.0 / 3224310063776.0,
                                  2802321613138.0 / 2924317926251.0};

void sem_lserk_coefficients(double* alpha, double* beta, double* c) {
  for (int k = 0; k < 5; ++k) {
    if (alpha) alpha[k] = kLserkA[k];
    if (beta) beta[k] = kLserkB[k];
    if (c) c[k] = kLserkC[k];
  }
}

sem_status sem_lserk_update(sem_ctx* ctx, int stage, double dt, const double* F, double* K,
                            double* y, size_t n) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (stage < 0 || stage > 4) throw ArgFail{"stage must be 0..4"};
    if (!F || !K || !y) throw ArgFail{"null vector"};
    enter(c);
    HK(semk::lserk_update(F, K, y, n, kLserkA[stage], dt, kLserkB[stage], c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_surface_dz(sem_ctx* ctx, const double* phi, double* w) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!phi || !w) throw ArgFail{"null vector"};
    enter(c);
    const DLevel& L0 = c->lev[0];
    const int Ps = c->dim == 2 ? L0.Pz : L0.P;
    HK(semk::surface_dz(Ps, phi, c->dsurf, w, c->hf_h.size(), L0.nzn, 1.0 / c->Nz, c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_wave_rhs(sem_ctx* ctx, const double* y, double* F, double* phi, double g,
                        double tol, sem_solve_info* info) {
  Ctx* c = C(ctx);
  const size_t ns = c ? c->hf_h.size() : 0;
  sem_status st = guarded(c, [&]() {
    if (!y || !F || !phi || y == F) throw ArgFail{"y, F, phi must be distinct device pointers"};
    if (!(g > 0.0)) throw ArgFail{"g must be positive"};
    if (!c->wrhs) c->wrhs = (double*)dalloc(c, (size_t)c->lev[0].N * 8);
    c->eta_h.resize(ns);
    enter(c);
    HK(hipMemcpyAsync(c->eta_h.data(), y, ns * 8, hipMemcpyDeviceToHost, c->st));
    HK(hipStreamSynchronize(c->st));
    return SEM_OK;
  });
  if (st != SEM_OK) return st;
  // the mesh of this stage's surface (the preconditioner stays), the Dirichlet problem, its solve
  if ((st = sem_mesh_update_surface(ctx, c->eta_h.data(), 0)) != SEM_OK) return st;
  if ((st = sem_assemble_rhs(ctx, nullptr, nullptr, y + ns, c->wrhs)) != SEM_OK) return st;
  if ((st = sem_poisson_solve(ctx, c->wrhs, phi, tol, info)) != SEM_OK) return st;
  return guarded(c, [&]() {
    enter(c);
    const DLevel& L0 = c->lev[0];
    const int Ps = c->dim == 2 ? L0.Pz : L0.P;
    HK(semk::surface_dz(Ps, phi, c->dsurf, F, ns, L0.nzn, 1.0 / c->Nz, c->st));
    HK(semk::vaxpby(true, -g, y, 0.0, y, F + ns, (unsigned)ns, c->st));
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_wave_step(sem_ctx* ctx, double* y, double* K, double* phi, double dt, double g,
                         double tol, int* iters) {
  Ctx* c = C(ctx);
  if (!c) return SEM_ERR_ARG;
  const size_t n = 2 * c->hf_h.size();
  sem_status st = guarded(c, [&]() {
    if (!y || !K || !phi || y == K) throw ArgFail{"y, K, phi must be distinct device pointers"};
    if (!c->wF) c->wF = (double*)dalloc(c, n * 8);
    return SEM_OK;
  });
  if (st != SEM_OK) return st;
  for (int k = 0; k < 5; ++k) {
    sem_solve_info inf{};
    if ((st = sem_wave_rhs(ctx, y, c->wF, phi, g, tol, &inf)) != SEM_OK) return st;
    if (iters) iters[k] = inf.iters;
    if ((st = sem_lserk_update(ctx, k, dt, c->wF, K, y, n)) != SEM_OK) return st;
  }
  return SEM_OK;
}

sem_status sem_learned_load(sem_ctx* ctx, const void* blob, size_t nbytes, int enable) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    learned_load_impl(c, blob, nbytes, enable);
    return SEM_OK;
  });
}

sem_status sem_learned_enable(sem_ctx* ctx, int enable) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!c->stage_alloc) return SEM_ERR_STATE;
    HK(hipStreamSynchronize(c->st));
    c->stage.enabled = (enable & 3) != 0;
    if (enable & 3) c->stage_mode = enable & 3;
    drop_graphs(c);
    return SEM_OK;
  });
}

sem_status sem_learned_judge(sem_ctx* ctx, const double* rhs, int cycles, sem_judge_result* out) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!c->stage_alloc || c->stage_blob.empty()) return SEM_ERR_STATE;
    if (!rhs) throw ArgFail{"null right-hand side"};
    if (cycles < 1 || cycles > 100) throw ArgFail{"cycles must be 1..100"};
    enter(c);
    DLevel& L0 = c->lev[0];
    const unsigned N = L0.N;
    const int mode = c->stage.enabled ? c->stage_mode : 1;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    HK(hipEventCreate(&t0));
    HK(hipEventCreate(&t1));
    double rho[2] = {1.0, 1.0}, ms[2] = {0.0, 0.0};
    hipGraphExec_t g = nullptr;
    try {
      for (int on = 0; on < 2; ++on) {
        c->stage.enabled = on != 0;
        if (on) c->stage_mode = mode;
        drop_graphs(c);
        HK(hipMemcpyAsync(c->bo, rhs, (size_t)N * 8, hipMemcpyDeviceToDevice, c->st));
        HK(hipMemsetAsync(c->xo, 0, (size_t)N * 8, c->st));
        HK(semk::copy_top(c->xo, c->bo, L0.nxn * L0.nyn, L0.nzn, c->st));
        apply_outer(c, c->xo, c->masked);
        HK(semk::resid64(c->bo, c->yo, c->So, c->ro, pset(c, PS_RR), pset(c, PS_BB), N, L0.nzn,
                         L0.P, c->st));
        // one cycle as a graph, as the solves run it (SEM_NO_GRAPH=1: launched directly)
        if (c->use_graphs) g = capture(c, [&]() { pdc_iteration(c); });
        auto cycle = [&]() {
          if (g) HK(hipGraphLaunch(g, c->st));
          else pdc_iteration(c);
        };
        cycle();  // the untimed cycle
        double s0[3], s1[3];
        read_sums(c, s0);
        HK(hipEventRecord(t0, c->st));
        for (int k = 0; k < cycles; ++k) cycle();
        HK(hipEventRecord(t1, c->st));
        read_sums(c, s1);
        float el = 0.f;
        HK(hipEventElapsedTime(&el, t0, t1));
        if (g) HK(hipGraphExecDestroy(g));
        g = nullptr;
        ms[on] = (double)el / cycles;
        rho[on] = (s0[0] > 0.0 && std::isfinite(s1[0]))
                      ? std::pow(std::sqrt(s1[0] / s0[0]), 1.0 / cycles) : 1.0;
      }
    } catch (...) {
      if (g) (void)hipGraphExecDestroy(g);
      (void)hipEventDestroy(t0);
      (void)hipEventDestroy(t1);
      throw;
    }
    HK(hipEventDestroy(t0));
    HK(hipEventDestroy(t1));
    const bool keep = rho[1] < 1.0 && rho[0] > 0.0 && ms[0] > 0.0 && ms[1] > 0.0 &&
                      (rho[0] >= 1.0 || std::log(rho[1]) / ms[1] < std::log(rho[0]) / ms[0]);
    c->stage.enabled = keep;
    c->stage_mode = mode;
    drop_graphs(c);
    HK(hipMemsetAsync(c->stage.skips, 0, sizeof(int), c->st));
    leave(c);
    HK(hipStreamSynchronize(c->st));
    if (out) {
      out->rho_plain = rho[0];
      out->rho_learned = rho[1];
      out->ms_plain = ms[0];
      out->ms_learned = ms[1];
      out->enabled = keep ? 1 : 0;
    }
    return SEM_OK;
  });
}

sem_status sem_learned_skips(sem_ctx* ctx, int* skips, int reset) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!c->stage_alloc) return SEM_ERR_STATE;
    int k = 0;
    HK(hipMemcpyAsync(&k, c->stage.skips, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HK(hipStreamSynchronize(c->st));
    if (skips) *skips = k;
    if (reset) {
      HK(hipMemsetAsync(c->stage.skips, 0, sizeof(int), c->st));
      HK(hipStreamSynchronize(c->st));
    }
    return SEM_OK;
  });
}

sem_status sem_launch_shape(const sem_ctx* ctx, int level, int* cols_per_block, int* coarse_w) {
  const Ctx* c = C(ctx);
  if (!c) return SEM_ERR_ARG;
  if (level < 0 || level >= (int)c->lev.size()) return SEM_ERR_ARG;
  const DLevel& L = c->lev[level];
  const bool smoothed = level + 1 < (int)c->lev.size();
  if (cols_per_block)
    *cols_per_block = (c->dim == 2 && smoothed && L.xalt) ? semk::cheb2d_cpb(L.P, L.Nx, L.Nz, L.dbl)
                                                         : 0;
  if (coarse_w) *coarse_w = (c->dim == 2 && smoothed && level >= 1) ? L.cpre.W : 0;
  return SEM_OK;
}

// training rows of the fine level (2D or 3D) for the elements in elist (null: all, in order)
static void stage_features(Ctx* c, const double* r, const double* e, float* X, float* T,
                           const int* elist, size_t nrows) {
  DLevel& L = c->lev[0];
  if (c->dim == 3)
    HK(semm::features3d(r, e, c->ainv_d, c->geo_d, c->stage.abar, X, T, L.geo.E, L.P, L.Ny, L.Nz,
                        L.nyn, L.nzn, c->st, elist, nrows));
  else
    HK(semm::features(r, e, c->ainv_d, c->geo_d, c->stage.abar, X, T, L.geo.E, L.P, L.Nz, L.nzn,
                      c->st, elist, nrows));
}

// the fine level can carry the stage: 2D P <= 8, 3D P <= 6
static void check_stage_mesh(Ctx* c) {
  DLevel& L = c->lev[0];
  if (c->dim == 2 && (L.rect || L.axis >= 0))
    throw ArgFail{"learned stage needs equal orders along x and sigma on the fine level and the "
                  "next"};
  if (c->dim == 2 && L.NP * L.NP > semm::MAX_STAGE_OUT)
    throw ArgFail{"learned stage needs fine order P <= 8"};
  if (c->dim == 3 && L.P > semm::MAX_STAGE_P3)
    throw ArgFail{"learned stage on hexahedra needs fine order P <= 6"};
}

// element-block inverses of the fine level for the training targets (training meshes only)
static void need_block_inverses(Ctx* c) {
  if (c->ainv_d) return;
  const size_t E = c->lev[0].geo.E;
  if ((c->dim == 2 && E > 4096) || (c->dim == 3 && E > 1024))
    throw ArgFail{"element-block targets are for training meshes (<= 4096 elements in 2D, "
                  "<= 1024 in 3D)"};
  c->ainv_d = upload(c, element_block_inverses(c));
}

sem_status sem_learned_features(sem_ctx* ctx, const double* r, const double* e, float* X,
                                float* T) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!r || !X) throw ArgFail{"null vector"};
    check_stage_mesh(c);
    HK(hipStreamSynchronize(c->st));
    stage_buffers(c);
    if (!c->geo_d) c->geo_d = upload(c, c->geo_h);
    if (T && !e) need_block_inverses(c);
    enter(c);
    stage_features(c, r, e, X, T, nullptr, 0);
    leave(c);
    return SEM_OK;
  });
}

// the stage-point residual of the V-cycle for the FP64 residual in c->ro: pre-smoothing from
// x = 0 on the fine level, then r_pre = r - A x_pre (FP64 outer operator) into c->qo
static void stage_point_residual(Ctx* c) {
  DLevel& L = c->lev[0];
  HK(semk::cast_to(L.dbl, c->ro, L.b, L.N, c->st));
  smooth(c, 0, true);
  HK(semk::cast_from(L.dbl, L.x, c->zo, L.N, c->st));
  apply_outer(c, c->zo, c->masked);
  HK(semk::resid64(c->ro, c->yo, c->So, c->qo, pset(c, PS_RR), nullptr, L.N, L.nzn, L.P, c->st));
}

// training rows of one residual: features and element-block targets of `per` elements drawn
// without replacement by a SplitMix64 Fisher-Yates prefix (all elements in order if per = 0)
static size_t harvest_rows(Ctx* c, const double* r, int per, unsigned long long seed,
                           unsigned long long* ctr, float* X, float* T) {
  DLevel& L = c->lev[0];
  const size_t E = L.geo.E;
  if (per <= 0 || (size_t)per >= E) {
    stage_features(c, r, nullptr, X, T, nullptr, 0);
    return E;
  }
  std::vector<int> idx(E);
  for (size_t i = 0; i < E; ++i) idx[i] = (int)i;
  for (int k = 0; k < per; ++k) {
    const double u = 0.5 * (semh::splitmix64_uniform(seed, (*ctr)++) + 1.0);  // [0, 1)
    size_t j = (size_t)k + (size_t)(u * (double)(E - k));
    if (j >= E) j = E - 1;
    std::swap(idx[k], idx[j]);
  }
  HK(hipMemcpyAsync(c->harvest_idx, idx.data(), per * sizeof(int), hipMemcpyHostToDevice, c->st));
  stage_features(c, r, nullptr, X, T, c->harvest_idx, (size_t)per);
  HK(hipStreamSynchronize(c->st));  // idx is a host vector
  return (size_t)per;
}

sem_status sem_learned_harvest(sem_ctx* ctx, const double* b, int cycles, int per,
                               unsigned long long seed, float* X, float* T, size_t* rows) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!b || !X || !T) throw ArgFail{"null vector"};
    if (cycles < 0 || cycles > 1000 || per < 0) throw ArgFail{"bad cycles / per"};
    if (!c->masked) return SEM_ERR_STATE;
    DLevel& L = c->lev[0];
    check_stage_mesh(c);
    if (c->lev.size() < 2) throw ArgFail{"harvesting needs at least two levels"};
    HK(hipStreamSynchronize(c->st));
    stage_buffers(c);
    if (!c->geo_d) c->geo_d = upload(c, c->geo_h);
    need_block_inverses(c);
    if (!c->harvest_idx) c->harvest_idx = (int*)dalloc(c, L.geo.E * sizeof(int));
    // the stage must not act inside the cycles that generate its own training data
    struct Restore {
      bool& flag;
      bool was;
      ~Restore() { flag = was; }
    } restore{c->stage.enabled, c->stage.enabled};
    c->stage.enabled = false;
    enter(c);
    const size_t N = L.N, n = c->dim == 3 ? (size_t)L.NP * L.NP * L.NP : (size_t)L.NP * L.NP;
    const size_t nin = (c->dim == 3 ? 7 : 5) * n;
    unsigned long long ctr = 0;
    size_t out = 0;
    if (cycles == 0) {  // b itself is a residual of the correction problem
      HK(hipMemcpyAsync(c->qo, b, N * 8, hipMemcpyDeviceToDevice, c->st));
      out += harvest_rows(c, c->qo, per, seed, &ctr, X, T);
    } else {
      HK(semk::fill(true, c->xo, 0.0, N, c->st));
      for (int k = 0; k < cycles; ++k) {
        // r = b - A x; training rows at the stage point; x += B r
        apply_outer(c, c->xo, c->masked);
        HK(semk::resid64(b, c->yo, c->So, c->ro, pset(c, PS_RR), nullptr, L.N, L.nzn, L.P, c->st));
        stage_point_residual(c);
        out += harvest_rows(c, c->qo, per, seed, &ctr, X + out * nin, T + out * n);
        vcycle(c, c->ro);
        HK(semk::cast_from(L.dbl, L.x, c->zo, L.N, c->st));
        HK(semk::axpy64(c->xo, c->zo, 1.0, L.N, c->st));
      }
    }
    leave(c);
    HK(hipStreamSynchronize(c->st));
    if (rows) *rows = out;
    return SEM_OK;
  });
}

sem_status sem_learned_train(sem_ctx* ctx, const float* X, const float* T, int n,
                             const sem_train_cfg* cfg, void* blob, size_t* nbytes) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!X || !T || !blob || !nbytes) throw ArgFail{"null argument"};
    check_stage_mesh(c);
    const DLevel& L = c->lev[0];
    const int nout = c->dim == 3 ? L.NP * L.NP * L.NP : L.NP * L.NP;
    const int nin = (c->dim == 3 ? 7 : 5) * nout;
    const size_t need = semm::blob_size(nin, nout);
    if (*nbytes < need) throw ArgFail{"blob buffer too small (see sem_mlp_blob_size)"};
    semm::TrainCfg tc;
    semm::Net init;
    bool have_init = false;
    if (cfg) {
      tc.epochs = cfg->epochs;
      tc.batch = cfg->batch;
      tc.lr = cfg->lr;
      tc.val_frac = cfg->val_frac;
      tc.seed = cfg->seed;
      if (cfg->init) {
        std::string e;
        if (!semm::net_from_blob(cfg->init, cfg->init_nbytes, init, e))
          throw ArgFail{"bad initial network: " + e};
        have_init = true;
      }
    }
    if (tc.epochs < 1 || tc.epochs > 100000 || tc.batch < 16 || tc.batch > 65536 ||
        !(tc.lr > 0) || tc.val_frac < 0 || tc.val_frac >= 1)
      throw ArgFail{"bad training configuration"};
    HK(hipStreamSynchronize(c->st));
    enter(c);
    semm::Net net;
    std::string e;
    if (!semm::train(X, T, n, nin, nout, tc, net, nullptr, c->st, e, have_init ? &init : nullptr))
      throw ArgFail{"training failed: " + e};
    HK(hipStreamSynchronize(c->st));
    semm::net_to_blob(net, blob);
    *nbytes = need;
    learned_load_impl(c, blob, need, c->stage.enabled ? c->stage_mode : 0);
    leave(c);
    return SEM_OK;
  });
}

sem_status sem_learned_stage(sem_ctx* ctx, const double* b, double* x, int* accepted) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (!c->stage_alloc) return SEM_ERR_STATE;
    if (!b || !x) throw ArgFail{"null vector"};
    enter(c);
    DLevel& L = c->lev[0];
    int before = 0, after = 0;
    HK(hipMemcpyAsync(&before, c->stage.skips, 4, hipMemcpyDeviceToHost, c->st));
    HK(semk::cast_to(L.dbl, b, L.b, L.N, c->st));
    HK(semk::cast_to(L.dbl, x, L.x, L.N, c->st));
    if (c->dim == 3) learned_stage3d(c);
    else learned_stage(c);
    HK(semk::cast_from(L.dbl, L.x, x, L.N, c->st));
    HK(hipMemcpyAsync(&after, c->stage.skips, 4, hipMemcpyDeviceToHost, c->st));
    HK(hipStreamSynchronize(c->st));
    leave(c);
    if (accepted) *accepted = (after == before) ? 1 : 0;
    return SEM_OK;
  });
}

sem_status sem_time_operator(sem_ctx* ctx, int level, int kind, int reps, int flush,
                             double* ms_avg) {
  Ctx* c = C(ctx);
  return guarded(c, [&]() {
    if (level < 0 || level >= (int)c->lev.size()) throw ArgFail{"bad level"};
    if (kind < 0 || kind > 2) throw ArgFail{"bad kind"};
    if (kind == 1 && level != 0) throw ArgFail{"the outer operator lives on level 0"};
    if (reps < 1 || !ms_avg) throw ArgFail{"bad reps / output"};
    DLevel& L = c->lev[level];
    if (kind == 2 && !L.xalt) throw ArgFail{"this level has no fused smoother step"};
    hipEvent_t e0, e1;
    HK(hipEventCreate(&e0));
    HK(hipEventCreate(&e1));
    void* junk = nullptr;
    const size_t fbytes = (size_t)512 << 20;
    if (flush == 1) HK(hipMalloc(&junk, fbytes));
    double total = 0.0;
    auto launch = [&]() {
      if (kind == 1) apply_outer(c, c->po, c->masked);
      else if (kind == 2) smooth_step(c, level, 0.5, 1e-3, 1);
      else apply_level(c, level, L.x, c->masked);
    };
    // flush == 2: every buffer the kernel reads or writes in R copies whose total exceeds three
    // times the 256 MB Infinity Cache, launched back to back in turn, so each launch streams its
    // data from HBM (the copies hold the same values, so the work is the same)
    std::vector<void**> slots;
    if (kind == 1) {
      slots = {(void**)&c->po, (void**)&c->yo, c->CG64 ? (void**)&c->CG64 : (void**)&c->G64};
      if (c->dim == 3) slots.insert(slots.end(), {(void**)&c->Sxo, (void**)&c->Syo, (void**)&c->Sxyo});
      else slots.push_back((void**)&c->So);
    } else if (kind == 2) {
      slots = {&L.x, &L.xalt, &L.b, &L.dinv, &L.d, &L.G};
    } else {
      slots = {&L.x, &L.y, &L.G};
      if (c->dim == 3) slots.insert(slots.end(), {&L.Sx, &L.Sy, &L.Sxy});
      else slots.push_back(&L.S);
    }
    std::vector<void*> orig;
    std::vector<size_t> sz;
    size_t set_bytes = 0;
    for (void** sl : slots) {
      orig.push_back(*sl);
      auto it = c->asize.find(*sl);
      if (!*sl || it == c->asize.end()) throw ArgFail{"buffer of the timed kernel not found"};
      sz.push_back(it->second);
      set_bytes += it->second;
    }
    int R = 1;
    std::vector<void*> rep;  // (R - 1) x slots copies
    auto restore = [&]() {
      for (size_t q = 0; q < slots.size(); ++q) *slots[q] = orig[q];
    };
    auto use = [&](int k) {
      for (size_t q = 0; q < slots.size(); ++q)
        *slots[q] = k == 0 ? orig[q] : rep[(size_t)(k - 1) * slots.size() + q];
    };
    auto free_rep = [&]() {
      restore();
      for (void* p : rep) (void)hipFree(p);
      rep.clear();
    };
    if (flush == 2) {
      const size_t want = (size_t)768 << 20;
      R = (int)std::min<size_t>(64, (want + set_bytes - 1) / set_bytes);
      R = std::max(R, 2);
      for (int k = 1; k < R; ++k)
        for (size_t q = 0; q < slots.size(); ++q) {
          void* p = nullptr;
          if (hipMalloc(&p, sz[q]) != hipSuccess) {
            free_rep();
            throw ArgFail{"not enough device memory for the rotated buffers"};
          }
          rep.push_back(p);
          HK(hipMemcpyAsync(p, orig[q], sz[q], hipMemcpyDeviceToDevice, c->st));
        }
      reps = std::max(reps, 2 * R);
    }
    try {
      launch();  // warm-up
      if (flush != 1) {
        if (flush == 2) {
          for (int k = 0; k < R; ++k) {  // one untimed pass over every copy
            use(k);
            launch();
          }
        }
        HK(hipEventRecord(e0, c->st));
        for (int k = 0; k < reps; ++k) {
          if (flush == 2) use(k % R);
          launch();
        }
        HK(hipEventRecord(e1, c->st));
        HK(hipEventSynchronize(e1));
        float ms = 0;
        HK(hipEventElapsedTime(&ms, e0, e1));
        total = ms;
      } else {
        for (int k = 0; k < reps; ++k) {
          HK(semk::fill(true, junk, (double)k, fbytes / 8, c->st));
          HK(hipEventRecord(e0, c->st));
          launch();
          HK(hipEventRecord(e1, c->st));
          HK(hipEventSynchronize(e1));
          float ms = 0;
          HK(hipEventElapsedTime(&ms, e0, e1));
          total += ms;
        }
      }
    } catch (...) {
      HK(hipStreamSynchronize(c->st));
      free_rep();
      throw;
    }
    HK(hipStreamSynchronize(c->st));
    free_rep();
    if (junk) HK(hipFree(junk));
    HK(hipEventDestroy(e0));
    HK(hipEventDestroy(e1));
    *ms_avg = total / reps;
    return SEM_OK;
  });
}

sem_status sem_operator_bytes(const sem_ctx* ctx, int level, int kind, double* bytes) {
  const Ctx* c = C(ctx);
  if (!c || !bytes || level < 0 || level >= (int)c->lev.size() || kind < 0 || kind > 2 ||
      (kind == 1 && level != 0))
    return SEM_ERR_ARG;
  const DLevel& L = c->lev[level];
  if (kind == 2 && !L.xalt) return SEM_ERR_ARG;
  const bool dbl = kind == 1 ? true : L.dbl;
  const semk::GType gt = kind == 1 ? semk::G_F64 : L.gt;
  const double sv = dbl ? 8.0 : 4.0;
  const double sg = gt == semk::G_F64 ? 8.0 : (gt == semk::G_F32 ? 4.0 : 2.0);
  const double nloc = c->dim == 2 ? (double)L.geo.E * L.geo.NP * L.geo.NPz
                                  : (double)L.geo.E * std::pow((double)L.NP, 3);
  const double nvec = kind == 2 ? 6.0 : 2.0;  // step: x, b, dinv, d read; x, d written
  *bytes = nvec * sv * L.N + L.geo.nfields * sg * nloc;
  // operators that form their factors from column records read those instead
  if ((kind == 1 && c->CG64) || (kind != 1 && L.gt == semk::G_COL64))
    *bytes = nvec * sv * L.N + (c->dim == 2 ? 8.0 * semk::COLGEO_N * (double)L.Nx * L.NP
                                            : 8.0 * semk::COLGEO3_N * (double)L.Nx * L.Ny *
                                                  L.NP * L.NP);
  return SEM_OK;
}

const char* sem_last_error(const sem_ctx* ctx) {
  const Ctx* c = C(ctx);
  if (c) return c->err.c_str();
  return g_mlp_err.empty() ? g_setup_err : g_mlp_err.c_str();
}

static sem_status mlp_guard(const std::function<bool(std::string&)>& body) {
  g_mlp_err.clear();
  try {
    std::string e;
    if (!body(e)) {
      g_mlp_err = e.empty() ? "training kernels failed" : e;
      return e.rfind("bad", 0) == 0 || e.find("mismatch") != std::string::npos ? SEM_ERR_ARG
                                                                               : SEM_ERR_HIP;
    }
    return SEM_OK;
  } catch (const std::bad_alloc&) {
    g_mlp_err = "host allocation failed";
    return SEM_ERR_ALLOC;
  } catch (...) {
    g_mlp_err = "unexpected internal error";
    return SEM_ERR_STATE;
  }
}

sem_status sem_mlp_train(const float* X, const float* T, int n, int nin, int nout,
                         const sem_train_cfg* cfg, void* blob, size_t nbytes, float* losses) {
  return mlp_guard([&](std::string& e) {
    if (!X || !T || !blob || nin < 1 || nout < 1) { e = "bad arguments"; return false; }
    if (nbytes != semm::blob_size(nin, nout)) { e = "bad blob size (size mismatch)"; return false; }
    semm::TrainCfg tc;
    if (cfg) {
      tc.epochs = cfg->epochs;
      tc.batch = cfg->batch;
      tc.lr = cfg->lr;
      tc.val_frac = cfg->val_frac;
      tc.seed = cfg->seed;
    }
    semm::Net init;
    const bool have_init = cfg && cfg->init;
    if (have_init && !semm::net_from_blob(cfg->init, cfg->init_nbytes, init, e)) {
      e = "bad initial network: " + e;
      return false;
    }
    if (tc.epochs < 1 || tc.epochs > 100000 || tc.batch < 16 || tc.batch > 65536 ||
        !(tc.lr > 0) || tc.val_frac < 0 || tc.val_frac >= 1) { e = "bad training configuration"; return false; }
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) { e = "stream creation failed"; return false; }
    semm::Net net;
    std::vector<float> ls;
    const bool ok = semm::train(X, T, n, nin, nout, tc, net, &ls, st, e, have_init ? &init : nullptr);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (!ok) return false;
    semm::net_to_blob(net, blob);
    if (losses) std::copy(ls.begin(), ls.end(), losses);
    return true;
  });
}

sem_status sem_mlp_forward(const void* blob, size_t nbytes, const float* X, int n, float* Y) {
  return mlp_guard([&](std::string& e) {
    semm::Net net;
    if (!semm::net_from_blob(blob, nbytes, net, e)) { e = "bad blob: " + e; return false; }
    if (!X || !Y || n < 1) { e = "bad arguments"; return false; }
    return semm::forward(net, X, n, Y, nullptr, e);
  });
}

sem_status sem_mlp_forward_noalloc(const void* blob, size_t nbytes, const float* X, int n,
                                   float* Y) {
  try {
    std::string e;  // stays empty (no allocation) unless the call fails
    if (semm::forward_noalloc(blob, nbytes, X, n, Y, e)) {
      g_mlp_err.clear();
      return SEM_OK;
    }
    g_mlp_err = e;
    return e.rfind("bad", 0) == 0 ? SEM_ERR_ARG : SEM_ERR_HIP;
  } catch (...) {
    return SEM_ERR_STATE;
  }
}

sem_status sem_mlp_gradients(const void* blob, size_t nbytes, const float* X, const float* T,
                             int n, float* grads, float* loss) {
  return mlp_guard([&](std::string& e) {
    semm::Net net;
    if (!semm::net_from_blob(blob, nbytes, net, e)) { e = "bad blob: " + e; return false; }
    if (!X || !T || !grads || n < 1 || n > 65536) { e = "bad arguments"; return false; }
    return semm::gradients(net, X, T, n, grads, loss, nullptr, e);
  });
}

const char* sem_status_string(sem_status s) {
  switch (s) {
    case SEM_OK: return "SEM_OK";
    case SEM_ERR_ARG: return "SEM_ERR_ARG";
    case SEM_ERR_ALLOC: return "SEM_ERR_ALLOC";
    case SEM_ERR_HIP: return "SEM_ERR_HIP";
    case SEM_ERR_NOT_CONVERGED: return "SEM_ERR_NOT_CONVERGED";
    case SEM_ERR_BREAKDOWN: return "SEM_ERR_BREAKDOWN";
    case SEM_ERR_STATE: return "SEM_ERR_STATE";
  }
  return "unknown";
}

}  // extern "C"
