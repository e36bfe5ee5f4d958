// gfx950 kernels of the spectral-element pressure-Poisson solver.
//
// Operator (paper Sec. 4.2, element matrices summed into the global matrix, eq. globallocal;
// stiffness read as sum_ab D_a^T G_ab D_b with GLL collocation): applied matrix-free and
// sum-factorised.  In 2D one workgroup owns one vertical column of Nz elements, so the faces
// between vertically stacked elements are summed in LDS; the vertical node lines shared by
// two columns are completed by the consumer from a side buffer (no atomics, no inter-group
// synchronisation, bitwise deterministic).  One thread owns one vertical line segment (i, ez)
// of an element: the sigma-direction contractions stay in registers, the x-direction ones go
// through LDS.  The work is HBM bound (about 1.5-2.2 flop/byte in FP64), so no MFMA is used.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <stdint.h>

#include <map>
#include <mutex>
#include <type_traits>

#include "gll_const.h"
#include "kernels.h"

namespace semk {

// ---- algorithmic-byte accounting (benchmark hook) -------------------------------------------
// While enabled, each launch wrapper of the solve path adds the bytes its kernel has to move at
// the least: every array it reads or writes once at its logical size (factors in their storage
// precision), nothing for re-reads, halos or scratch.
namespace {
bool g_acct_on = false;
double g_acct_bytes = 0.0;
long g_acct_n = 0;
inline double vsz(bool dbl) { return dbl ? 8.0 : 4.0; }
inline double gsz(GType gt) { return gt == G_F64 ? 8.0 : (gt == G_F32 ? 4.0 : 2.0); }
inline double nodes2(int P, int Nx, int Nz) { return (double)(Nx * P + 1) * (double)(Nz * P + 1); }
inline double local2(int P, int Nx, int Nz) { return (double)Nx * Nz * (P + 1) * (P + 1); }
// bytes of one pass over a 2D level's factors: stored (three per local node) or column records
inline double gbytes2(GType gt, int P, int Nx, int Nz) {
  return gt == G_COL64 ? 8.0 * COLGEO_N * Nx * (P + 1) : 3 * gsz(gt) * local2(P, Nx, Nz);
}
}  // namespace
void acct_enable(bool on) {
  g_acct_on = on;
  if (on) {
    g_acct_bytes = 0.0;
    g_acct_n = 0;
  }
}
void acct_add(double bytes) {
  if (!g_acct_on) return;
  g_acct_bytes += bytes;
  ++g_acct_n;
}
double acct_total(long* launches) {
  if (launches) *launches = g_acct_n;
  return g_acct_bytes;
}

// ------------------------------------------------------------------------------------------
// type helpers
// ------------------------------------------------------------------------------------------
template <typename T, typename TG>
__device__ __forceinline__ T gload(const TG* p);
template <>
__device__ __forceinline__ double gload<double, double>(const double* p) { return *p; }
template <>
__device__ __forceinline__ float gload<float, float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float gload<float, uint16_t>(const uint16_t* p) {
  return __uint_as_float(((uint32_t)(*p)) << 16);
}

static inline unsigned nblk(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// dynamic LDS above 64 KB (gfx950: 160 KB per workgroup) needs the kernel's limit raised; the
// limit is raised once per kernel to the largest size asked for (the host call stays out of the
// launch path afterwards)
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  const void* key = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lock(mu);
  auto it = done.find(key);
  if (it != done.end() && it->second >= bytes) return hipSuccess;
  const hipError_t e =
      hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done[key] = bytes;
  return e;
}

// (A x)[g] from the column output y and the side buffer S (2D; S null: y is complete)
template <typename T>
__device__ __forceinline__ T ax_at(const T* __restrict__ y, const T* __restrict__ S, unsigned g,
                                   unsigned nzn, unsigned P) {
  if (!S) return y[g];  // complete column output (3D, after the face fix-up)
  const unsigned ix = g / nzn;
  const unsigned iz = g - ix * nzn;
  T v = y[g];
  const unsigned q = ix / P;
  if (q * P == ix) v += S[q * nzn + iz];
  return v;
}

// deterministic block reduction (fixed shuffle pattern, fixed LDS tree); all threads get it
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < nw; ++k) s += sh[k];
  return s;
}

// sum of NRED partials (fixed order), computed identically by every block that calls it
__device__ double sum_partials(const double* __restrict__ p, double* sh) {
  double v = 0.0;
  for (int k = threadIdx.x; k < NRED; k += blockDim.x) v += p[k];
  return block_sum(v, sh);
}

// step length of the learned stage, alpha = c.r / c.q from its two partial-sum sets (fixed
// order, the same value in every block); 0 when not finite and positive (step rejected)
__device__ double stage_alpha(const double* __restrict__ pcr, int ncr,
                              const double* __restrict__ pcq, int ncq, double* sh, bool* ok) {
  double a0 = 0.0, a1 = 0.0;
  for (int k = threadIdx.x; k < ncr; k += blockDim.x) a0 += pcr[k];
  for (int k = threadIdx.x; k < ncq; k += blockDim.x) a1 += pcq[k];
  const double cr = block_sum(a0, sh);
  const double cq = block_sum(a1, sh);
  const double alpha = cr / cq;
  *ok = isfinite(alpha) && alpha > 0.0;
  return *ok ? alpha : 0.0;
}

// ------------------------------------------------------------------------------------------
// 2D operator apply
// ------------------------------------------------------------------------------------------
// n contiguous LDS values into registers, in 16-byte pieces where the alignment AL (in elements,
// known at compile time) allows
template <int N, int AL, typename T>
__device__ __forceinline__ void lds_get(const T* p, T (&o)[N]) {
  constexpr int V = (AL * sizeof(T) >= 16) ? 16 / (int)sizeof(T) : ((AL * sizeof(T) >= 8) ? 8 / (int)sizeof(T) : 1);
  int m = 0;
  if constexpr (V == 4) {
    typedef T v4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (; m + 4 <= N; m += 4) {
      const v4 a = *reinterpret_cast<const v4*>(p + m);
      o[m] = a[0]; o[m + 1] = a[1]; o[m + 2] = a[2]; o[m + 3] = a[3];
    }
  } else if constexpr (V == 2) {
    typedef T v2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (; m + 2 <= N; m += 2) {
      const v2 a = *reinterpret_cast<const v2*>(p + m);
      o[m] = a[0]; o[m + 1] = a[1];
    }
  }
#pragma unroll
  for (; m < N; ++m) o[m] = p[m];
}

template <typename T>
constexpr int lds_vec() { return 16 / (int)sizeof(T); }  // elements per 16-byte LDS access

template <int P, typename T>
constexpr int line_align() {  // alignment (elements) of an element's offset ez * P in a line
  return (P % lds_vec<T>() == 0) ? lds_vec<T>() : ((P % 2 == 0) ? 2 : 1);
}

// LDS layout of the apply, per element column: exchange array X1 [Nz][NP][NPp], then exchange
// array X2 [Nz][NP][NPp] whose space also holds, at other times, the input/output column
// [NP][nzp] and after it the element-top values [Nz][NP]; the slot is padded to 16 bytes
inline int apply2d_nzp(int P, int Nz, bool dbl) {
  const int V = dbl ? 2 : 4, nzn = Nz * P + 1;
  return (nzn + V - 1) / V * V;
}

template <typename I>
__host__ __device__ constexpr I slot2d_elems(I NP, I Nz, I nzp, I V) {
  const I NPp = (NP + V - 1) / V * V, ex = Nz * NP * NPp;
  const I col = NP * nzp + Nz * NP;
  return (ex + (col > ex ? col : ex) + V - 1) / V * V;
}

static size_t apply2d_slot(int P, int Nz, bool dbl) {  // elements per column
  return slot2d_elems<size_t>(P + 1, Nz, apply2d_nzp(P, Nz, dbl), dbl ? 2 : 4);
}

size_t apply2d_smem(int P, int Nz, bool dbl) { return apply2d_slot(P, Nz, dbl) * (dbl ? 8 : 4); }

// columns per workgroup: two when that still leaves at least 512 workgroups (a multiple of 8,
// so the XCD-aware order applies) within 1024 threads and 64 KB of LDS, else one.  Measured on
// the 1024 x 16 and 2048 x 16 column meshes at P = 8: two columns per workgroup with the XCD
// order is the fastest of 1-4; three (odd wave counts per workgroup) is the slowest.
int apply2d_cpb(int P, int Nx, int Nz, bool dbl) {
  const int nthr = (P + 1) * Nz;
  const int blocks2 = (Nx + 1) / 2;
  if (2 * nthr <= 1024 && 2 * apply2d_smem(P, Nz, dbl) <= 65536 && blocks2 >= 512 &&
      blocks2 % 8 == 0)
    return 2;
  return 1;
}

// geometric factors of the operator: layout in kernels.h (GLayout)
template <int P, typename TG>
struct G2dLayout {
  static constexpr int K = 3 * (P + 1);
  static constexpr int W = 16 / (int)sizeof(TG);
  static constexpr int H = W / 2 > 0 ? W / 2 : 1;
  static constexpr int Kp = (K + H - 1) / H * H;
  static constexpr int NC = Kp / W;
  static constexpr int REM = Kp - NC * W;
};

GLayout g2d_layout(int P, int Nz, size_t tgsize) {
  GLayout L;
  L.W = 16 / (int)tgsize;
  const int H = L.W / 2 > 0 ? L.W / 2 : 1, K = 3 * (P + 1);
  L.Kp = (K + H - 1) / H * H;
  L.NC = L.Kp / L.W;
  L.REM = L.Kp - L.NC * L.W;
  const size_t nk = (size_t)(P + 1) * Nz * L.Kp;
  L.cstride = (nk + L.W - 1) / L.W * L.W;
  return L;
}

// G_COL64: the factors of thread t = ez NP + i (vertical line i of element ez) formed from the
// column record of (ex, i), {c0 = w_i d dsig/dx, c3 = w_i dx/(dsig d), h_x, d_x}, and the
// compile-time GLL nodes and weights: with sigma_j = (ez + (r_j + 1)/2)/Nz and
// a = h_x - sigma_j d_x (= d sigma_x), G_rr = w_j c0, G_rs = w_i w_j a, G_ss = w_j c3 (a^2 + 1)
// (the same products as the stored factors' w_i w_j |J| J^-1 J^-T of the sigma mapping)
struct ColGeo64 {
  double v;
};
template <int P, typename T>
__device__ __forceinline__ void colgeo_g2d(const double* __restrict__ CG, int ex, int Nz, int t,
                                           T (&g)[3][P + 1]) {
  // the record is read in FP64 and the factors formed in the kernel's precision T: with
  // sigma_j = (ez + hr_j)/Nz, a_j = h_x - sigma_j d_x = A - hr_j B (A = h_x - (ez/Nz) d_x,
  // B = d_x / Nz), three multiply-adds and four multiplies per node
  constexpr int NP = P + 1;
  const int i = t % NP, ez = t / NP;
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2* c = reinterpret_cast<const d2*>(CG + ((size_t)ex * NP + i) * COLGEO_N);
  const d2 c03 = c[0], hd = c[1];
  T wi = 0;
  gllc::sfor<NP>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if (i == k) wi = (T)gllc::tab<P>.w[k];
  });
  const double inz = 1.0 / Nz;
  const T c0 = (T)c03[0], c3 = (T)c03[1];
  const T A = (T)fma(-(double)ez * inz, hd[1], hd[0]);
  const T Bv = (T)(hd[1] * inz);
  gllc::sfor<NP>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    constexpr T wj = (T)gllc::tab<P>.w[j];
    constexpr T hr = (T)(0.5 * (gllc::tab<P>.x[j] + 1.0));
    const T a = fma(-hr, Bv, A);
    g[0][j] = wj * c0;
    g[1][j] = (wi * wj) * a;
    g[2][j] = (wj * c3) * fma(a, a, (T)1);
  });
}

// this thread's 3 (P+1) factors (f, j) of element column ex, with 16-byte loads
template <int P, typename T, typename TG>
__device__ __forceinline__ void load_g2d_stored(const TG* __restrict__ G, int ex, int nthr, int t,
                                         T (&g)[3][P + 1]) {
  using Ly = G2dLayout<P, TG>;
  constexpr int NP = P + 1, W = Ly::W, NC = Ly::NC, REM = Ly::REM, Kp = Ly::Kp;
  typedef TG vW __attribute__((ext_vector_type(W)));
  const size_t cstride = ((size_t)nthr * Kp + W - 1) / W * W;
  const TG* Gc = G + (size_t)ex * cstride;
  TG raw[Kp];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const vW a = *reinterpret_cast<const vW*>(Gc + ((size_t)c * nthr + t) * W);
#pragma unroll
    for (int w = 0; w < W; ++w) raw[c * W + w] = a[w];
  }
  if constexpr (REM == 1) {
    raw[NC * W] = Gc[(size_t)NC * nthr * W + t];
  } else if constexpr (REM > 1) {
    typedef TG vR __attribute__((ext_vector_type(REM)));
    const vR a = *reinterpret_cast<const vR*>(Gc + (size_t)NC * nthr * W + (size_t)t * REM);
#pragma unroll
    for (int w = 0; w < REM; ++w) raw[NC * W + w] = a[w];
  }
#pragma unroll
  for (int f = 0; f < 3; ++f)
#pragma unroll
    for (int j = 0; j < NP; ++j) g[f][j] = gload<T, TG>(&raw[f * NP + j]);
}

// this thread's factors from the level's factor data: stored layout or column records
template <int P, typename T, typename TG>
__device__ __forceinline__ void load_g2d(const TG* __restrict__ G, int ex, int nthr, int t,
                                         T (&g)[3][P + 1]) {
  if constexpr (std::is_same<TG, ColGeo64>::value) {
    colgeo_g2d<P, T>(reinterpret_cast<const double*>(G), ex, nthr / (P + 1), t, g);
  } else {
    load_g2d_stored<P, T, TG>(G, ex, nthr, t, g);
  }
}

// The operator on one element column (slot) of a workgroup.  Thread t = ez * NP + q of the slot
// has two roles in element ez: the vertical line i = q (sigma-direction contractions, geometric
// factors) and the horizontal row j = q (x-direction contractions).  The roles swap data through
// LDS: u_r row -> line, w_r line -> row, D_r^T w_r row -> line.  All contractions run in
// registers against compile-time D (even-odd form).  On return (after a barrier) the slot's LDS
// column su[l * nzp + iz] holds the column's part of (A x) on its lines l = 0..P, with the faces
// between vertically stacked elements summed and, when masked, the Dirichlet top node equal to
// x; xin[l] holds x(line l, node t) for t < nzn, as filled by ldx(xin) (called when act and
// t < nzn).  Every thread of the block calls this.
// column_apply with the factors already in registers (g as load_g2d gives them)
template <int P, typename T, typename Ldx, typename Pre>
__device__ __forceinline__ void column_apply_g(const T (&g)[3][P + 1], Ldx&& ldx, int t, bool act,
                                               int Nz, int nzn, int nzp, int masked, T* base,
                                               T (&xin)[P + 1], Pre&& pre);

template <int P, typename T, typename TG, typename Ldx, typename Pre>
__device__ __forceinline__ void column_apply(Ldx&& ldx, const TG* __restrict__ G, int ex,
                                             int nthr, int t, bool act, int Nz, int nzn, int nzp,
                                             int masked, T* base, T (&xin)[P + 1], Pre&& pre) {
  // every global load of the block (the caller's through pre()) is issued before the first LDS
  // store
  T g[3][P + 1];
  if (act) load_g2d<P, T, TG>(G, ex, nthr, t, g);
  column_apply_g<P, T>(g, ldx, t, act, Nz, nzn, nzp, masked, base, xin, pre);
}

template <int P, typename T, typename Ldx, typename Pre>
__device__ __forceinline__ void column_apply_g(const T (&g)[3][P + 1], Ldx&& ldx, int t, bool act,
                                               int Nz, int nzn, int nzp, int masked, T* base,
                                               T (&xin)[P + 1], Pre&& pre) {
  constexpr int NP = P + 1;
  constexpr int V = lds_vec<T>();
  constexpr int NPp = (NP + V - 1) / V * V;
  constexpr int AL = line_align<P, T>();
  const int q = t % NP;
  const int ez = t / NP;
  T* X1 = base;                    // [Nz][NP(i)][NPp(j)]: u_r, later D_r^T w_r
  T* X2 = X1 + Nz * NP * NPp;      // [Nz][NP(j)][NPp(i)]: w_r (phases 3-4)
  T* su = X2;                      // [NP][nzp] column: input (phases 1-2), output (phase 6)
  T* stp = X2 + NP * nzp;          // [Nz][NP] element-top values (phases 5-6)
  if (act && t < nzn) ldx(xin);
  pre();
  if (act && t < nzn) {
#pragma unroll
    for (int l = 0; l < NP; ++l) su[l * nzp + t] = xin[l];
  }
  __syncthreads();

  const bool topel = (ez == Nz - 1);
  const bool mtop = masked && topel;  // Dirichlet surface: its values enter as zero
  T v[NP], us[NP];
  T xtop = 0;
  if (act) {
    // row role (j = q): u_r(i, j) = sum_k D_ik u(k, j)
    {
      T r[NP], ur[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) r[i] = su[i * nzp + ez * P + q];
      if (mtop && q == P) {
#pragma unroll
        for (int i = 0; i < NP; ++i) r[i] = 0;
      }
      contract_eo<P, false>(r, ur);
#pragma unroll
      for (int i = 0; i < NP; ++i) X1[(ez * NP + i) * NPp + q] = ur[i];
    }
    // line role (i = q): u_s(i, j) = sum_k D_jk u(i, k)
    T u[NP];
    lds_get<NP, AL>(su + q * nzp + ez * P, u);
    if (topel) xtop = u[P];
    if (mtop) u[P] = 0;
    contract_eo<P, false>(u, us);
  }
  __syncthreads();
  if (act) {
    // line role: (w_r, w_s) = G (u_r, u_s); v = D_s^T w_s; w_r to the rows
    T ur[NP], ws[NP];
    lds_get<NP, V>(X1 + (ez * NP + q) * NPp, ur);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      X2[(ez * NP + j) * NPp + q] = g[0][j] * ur[j] + g[1][j] * us[j];
      ws[j] = g[1][j] * ur[j] + g[2][j] * us[j];
    }
    contract_eo<P, true>(ws, v);
  }
  __syncthreads();
  if (act) {
    // row role: (D_r^T w_r)(i, j) = sum_k D_ki w_r(k, j)
    T w[NP], vr[NP];
    lds_get<NP, V>(X2 + (ez * NP + q) * NPp, w);
    contract_eo<P, true>(w, vr);
#pragma unroll
    for (int i = 0; i < NP; ++i) X1[(ez * NP + i) * NPp + q] = vr[i];
  }
  __syncthreads();
  if (act) {
    T vr[NP];
    lds_get<NP, V>(X1 + (ez * NP + q) * NPp, vr);
#pragma unroll
    for (int j = 0; j < NP; ++j) v[j] += vr[j];
    stp[ez * NP + q] = v[P];
  }
  __syncthreads();
  if (act) {
    // sum over the face shared with the element below; output line i = q of element ez
    if (ez > 0) v[0] += stp[(ez - 1) * NP + q];
    T* ocol = su + q * nzp + ez * P;
#pragma unroll
    for (int j = 0; j < P; ++j) ocol[j] = v[j];
    if (topel) ocol[P] = masked ? xtop : v[P];
  }
  __syncthreads();
}

// One workgroup per cpb element columns (column_apply per slot).  Output: lines 0..P-1 of each
// column to y, line P to the side buffer S of the right neighbour (to y for the last column).
// DOT: also the block's part of x . (A x) into dotp[block] (each node's product counted once:
// its column-output part and its side-buffer part are owned by different blocks, whose sum is
// the whole entry).
template <int P, typename T, typename TG, bool DOT = false>
__global__ __launch_bounds__(1024) void k_apply2d(const T* __restrict__ x, T* __restrict__ y,
                                                  T* __restrict__ S, const TG* __restrict__ G,
                                                  int Nx, int Nz, int masked, int cpb, int remap,
                                                  double* __restrict__ dotp) {
  constexpr int NP = P + 1;
  constexpr int V = lds_vec<T>();
  constexpr int NPp = (NP + V - 1) / V * V;
  const int nzn = Nz * P + 1;
  const int nzp = (nzn + V - 1) / V * V;
  const int nthr = NP * Nz;
  int bx = blockIdx.x;
  if (remap) {  // consecutive columns on the same XCD (blocks are dealt round-robin to 8 XCDs)
    const int per = gridDim.x >> 3;
    bx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  const int cs = threadIdx.x / nthr;       // column slot of this thread
  const int t = threadIdx.x - cs * nthr;   // thread within the column
  const int ex = bx * cpb + cs;
  const bool valid = cs < cpb && ex < Nx;  // uniform per column slot
  const int slot = slot2d_elems<int>(NP, Nz, nzp, V);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* base = reinterpret_cast<T*>(smem_raw) + (valid ? cs : 0) * slot;
  const T* su = base + Nz * NP * NPp;  // output column of this slot
  // column-relative 32-bit offsets from per-column base pointers
  const T* xc = x + (size_t)(valid ? ex : 0) * P * nzn;
  T* yc = y + (size_t)(valid ? ex : 0) * P * nzn;
  T xin[NP];
  column_apply<P, T, TG>(
      [&](T(&v)[NP]) {
#pragma unroll
        for (int l = 0; l < NP; ++l) v[l] = xc[l * nzn + t];
      },
      G, ex, nthr, t, valid, Nz, nzn, nzp, masked, base, xin, [] {});

  double part = 0.0;
  if (valid && t < nzn) {
#pragma unroll
    for (int l = 0; l < P; ++l) {
      const T o = su[l * nzp + t];
      yc[l * nzn + t] = o;
      if constexpr (DOT) part += (double)xin[l] * (double)o;
    }
    T last = su[P * nzp + t];
    if (ex == Nx - 1) {
      yc[P * nzn + t] = last;
    } else {
      if (masked && t == nzn - 1) last = (T)0;
      S[(size_t)(ex + 1) * nzn + t] = last;
    }
    if constexpr (DOT) part += (double)xin[P] * (double)last;
  }
  if constexpr (DOT) {
    __shared__ double red[16];
    const double tot = block_sum(part, red);
    if (threadIdx.x == 0) dotp[blockIdx.x] = tot;
  }
}

// One smoother step fused with the operator (2D):  r = b - A xi;  dn = cr dinv r (+ cd d);
// d = dn (store_d);  xo = xi + dn.  Workgroup bx owns element columns bx cpb .. bx cpb + cpb - 1
// (slots 1..cpb) and recomputes the column to their left (slot 0, the halo), so the vertical
// line shared with it is summed in LDS and every owned node gets its whole (A x) without a side
// buffer or a second kernel.  A column owns its lines 0..P-1, the last column also line P.
// xi and xo must be different vectors (other workgroups still read xi).  MODE 1 computes only
// the residual: xo = b - A xi (dinv, d, cd, cr unused).
template <int P, typename T, typename TG, int MODE = 0>
__global__ __launch_bounds__(1024) void k_cheb2d(const T* __restrict__ xi, T* __restrict__ xo,
                                                 T* __restrict__ d, const T* __restrict__ b,
                                                 const T* __restrict__ dinv,
                                                 const TG* __restrict__ G, int Nx, int Nz,
                                                 int masked, int cpb, int remap, T cd, T cr,
                                                 int store_d) {
  constexpr int NP = P + 1;
  constexpr int V = lds_vec<T>();
  constexpr int NPp = (NP + V - 1) / V * V;
  const int nzn = Nz * P + 1;
  const int nzp = (nzn + V - 1) / V * V;
  const int nthr = NP * Nz;
  int bx = blockIdx.x;
  if (remap) {
    const int per = gridDim.x >> 3;
    bx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  const int cs = threadIdx.x / nthr;  // slot 0: halo column, slots 1..cpb: owned columns
  const int t = threadIdx.x - cs * nthr;
  const int ex = bx * cpb + cs - 1;
  const bool valid = cs <= cpb && ex >= 0 && ex < Nx;
  const int slot = slot2d_elems<int>(NP, Nz, nzp, V);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* base = reinterpret_cast<T*>(smem_raw) + (valid ? cs : 0) * slot;
  const T* xc = xi + (size_t)(valid ? ex : 0) * P * nzn;
  // FP32: the owned nodes' b, dinv, d are loaded together with the operator's inputs (in FP64
  // the extra registers would spill; there they are loaded in the epilogue)
  constexpr bool PF = sizeof(T) == 4;
  const bool own = cs >= 1 && valid && t < nzn;
  const int nl = (ex == Nx - 1) ? NP : P;  // owned lines of this column
  const size_t g0 = (size_t)(valid ? ex : 0) * P * nzn + t;
  T pb[NP], pdi[NP], pd[NP];
  auto load_own = [&] {
    if (own) {
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        if (l < nl) {
          const size_t g = g0 + (size_t)l * nzn;
          pb[l] = b[g];
          if constexpr (MODE == 0) {
            pdi[l] = dinv[g];
            pd[l] = cd != (T)0 ? d[g] : (T)0;
          }
        }
      }
    }
  };
  T xin[NP];
  column_apply<P, T, TG>(
      [&](T(&v)[NP]) {
#pragma unroll
        for (int l = 0; l < NP; ++l) v[l] = xc[l * nzn + t];
      },
      G, valid ? ex : 0, nthr, t, valid, Nz, nzn, nzp, masked, base, xin, [&] {
                           if constexpr (PF) load_own();
                         });
  if constexpr (!PF) load_own();

  if (own) {
    const T* su = base + Nz * NP * NPp;  // this column's part of A x
    const T* sl = su - slot;             // the left column's (slot cs - 1, valid when ex > 0)
    const bool left = ex > 0 && !(masked && t == nzn - 1);
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      if (l < nl) {
        T ax = su[l * nzp + t];
        if (l == 0 && left) ax += sl[P * nzp + t];
        const size_t g = g0 + (size_t)l * nzn;
        const T r = pb[l] - ax;
        if constexpr (MODE == 1) {
          xo[g] = r;
        } else {
          T dn = cr * pdi[l] * r;
          if (cd != (T)0) dn += cd * pd[l];
          if (store_d) d[g] = dn;
          xo[g] = xin[l] + dn;
        }
      }
    }
  }
}

// The first two smoother steps of a pre-smoothing from x = 0 in one kernel: step 0,
// x1 = d1 = cr0 dinv b, is formed while loading (for the halo column too); then step 1 as in
// k_cheb2d: r = b - A x1, dn = cr dinv r (+ cd d1), d = dn (store_d), x = x1 + dn.  With r64
// the right-hand side arrives in FP64 and is rounded into b here (owned nodes written).  x and
// d are written in place: no workgroup reads them.
template <int P, typename T, typename TG>
__global__ __launch_bounds__(1024) void k_cheb2d_first(T* __restrict__ x, T* __restrict__ d,
                                                       T* __restrict__ b,
                                                       const double* __restrict__ r64,
                                                       const T* __restrict__ dinv,
                                                       const TG* __restrict__ G, int Nx, int Nz,
                                                       int masked, int cpb, int remap, T cr0,
                                                       T cd, T cr, int store_d) {
  constexpr int NP = P + 1;
  constexpr int V = lds_vec<T>();
  constexpr int NPp = (NP + V - 1) / V * V;
  const int nzn = Nz * P + 1;
  const int nzp = (nzn + V - 1) / V * V;
  const int nthr = NP * Nz;
  int bx = blockIdx.x;
  if (remap) {
    const int per = gridDim.x >> 3;
    bx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  const int cs = threadIdx.x / nthr;
  const int t = threadIdx.x - cs * nthr;
  const int ex = bx * cpb + cs - 1;
  const bool valid = cs <= cpb && ex >= 0 && ex < Nx;
  const int slot = slot2d_elems<int>(NP, Nz, nzp, V);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* base = reinterpret_cast<T*>(smem_raw) + (valid ? cs : 0) * slot;
  const size_t g0 = (size_t)(valid ? ex : 0) * P * nzn + t;
  // FP32 keeps b and dinv of its lines in registers for the update; FP64 (where they would
  // spill) reads them again after the apply
  constexpr bool KEEP = sizeof(T) == 4;
  T bl[NP], dl[NP], xin[NP];
  column_apply<P, T, TG>(
      [&](T(&v)[NP]) {
#pragma unroll
        for (int l = 0; l < NP; ++l) {
          const size_t g = g0 + (size_t)l * nzn;
          const T bv = r64 ? (T)r64[g] : b[g];
          const T dv = dinv[g];
          if constexpr (KEEP) {
            bl[l] = bv;
            dl[l] = dv;
          }
          v[l] = cr0 * dv * bv;
        }
      },
      G, valid ? ex : 0, nthr, t, valid, Nz, nzn, nzp, masked, base, xin, [] {});
  if constexpr (!KEEP) {
    if (cs >= 1 && valid && t < nzn) {
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        const size_t g = g0 + (size_t)l * nzn;
        bl[l] = r64 ? (T)r64[g] : b[g];
        dl[l] = dinv[g];
      }
    }
  }
  if (cs >= 1 && valid && t < nzn) {
    const T* su = base + Nz * NP * NPp;
    const T* sl = su - slot;
    const bool left = ex > 0 && !(masked && t == nzn - 1);
    const int nl = (ex == Nx - 1) ? NP : P;
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      if (l < nl) {
        T ax = su[l * nzp + t];
        if (l == 0 && left) ax += sl[P * nzp + t];
        const size_t g = g0 + (size_t)l * nzn;
        const T r = bl[l] - ax;
        T dn = cr * dl[l] * r;
        if (cd != (T)0) dn += cd * xin[l];
        if (store_d) d[g] = dn;
        x[g] = xin[l] + dn;
        if (r64) b[g] = bl[l];
      }
    }
  }
}

// owned columns per workgroup of the fused step.  Measured on the 1024 x 16 and 2048 x 16 column
// meshes (P = 8, 4, 2): four owned columns when two such workgroups fit a CU's 160 KB of LDS and
// the workgroup count is a multiple of 8 (XCD-aware order) and at least 256, else two (FP64 at
// P = 8: 2 is faster than 4); odd counts (no XCD order) are the slowest.  One owned column (the
// halo doubles the work) still beats operator + update.  0: the fused form does not fit.
// SEM_CHEB_CPB=1, 2 or 4 forces that count where it fits (read once per process; tuning only)
static int cpb_override() {
  static const int v = [] {
    const char* e = std::getenv("SEM_CHEB_CPB");
    const int k = e ? std::atoi(e) : 0;
    return (k == 1 || k == 2 || k == 4) ? k : 0;
  }();
  return v;
}

int cheb2d_cpb(int P, int Nx, int Nz, bool dbl) {
  const int nthr = (P + 1) * Nz;
  const size_t sm = apply2d_smem(P, Nz, dbl), lds = 160 * 1024;
  auto fits = [&](int c) { return (c + 1) * nthr <= 1024 && (c + 1) * sm <= lds; };
  if (const int f = cpb_override())
    if (fits(f)) return f;
  const int b4 = (Nx + 3) / 4;
  if (fits(4) && 2 * 5 * sm <= lds && b4 % 8 == 0 && b4 >= 256) return 4;
  if (fits(2)) return 2;
  if (fits(1)) return 1;
  return 0;
}

template <int P, typename T, typename TG, int MODE = 0>
static hipError_t launch_cheb2d(const void* xi, void* xo, void* d, const void* b, const void* dinv,
                                const void* G, int Nx, int Nz, int masked, double cd, double cr,
                                int store_d, int cpb, hipStream_t st) {
  const bool dbl = sizeof(T) == 8;
  if (cpb <= 0) return hipErrorInvalidValue;
  const int nthr = (P + 1) * Nz;
  const int threads = (((cpb + 1) * nthr + 63) / 64) * 64;
  const int blocks = (Nx + cpb - 1) / cpb;
  const size_t smem = apply2d_smem(P, Nz, dbl) * (cpb + 1);
  if (threads > 1024 || smem > 160 * 1024) return hipErrorInvalidValue;
  const int remap = (blocks % 8 == 0) ? 1 : 0;
  hipError_t e = allow_lds(k_cheb2d<P, T, TG, MODE>, smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_cheb2d<P, T, TG, MODE>), dim3(blocks), dim3(threads), smem, st, (const T*)xi,
                     (T*)xo, (T*)d, (const T*)b, (const T*)dinv, (const TG*)G, Nx, Nz, masked, cpb,
                     remap, (T)cd, (T)cr, store_d);
  return hipGetLastError();
}

template <int P>
static hipError_t cheb2d_p(bool dbl, GType gt, const void* xi, void* xo, void* d, const void* b,
                           const void* dinv, const void* G, int Nx, int Nz, int masked, double cd,
                           double cr, int store_d, int cpb, hipStream_t st) {
  if (gt == G_COL64)
    return dbl ? launch_cheb2d<P, double, ColGeo64>(xi, xo, d, b, dinv, G, Nx, Nz, masked, cd,
                                                    cr, store_d, cpb, st)
               : launch_cheb2d<P, float, ColGeo64>(xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr,
                                                   store_d, cpb, st);
  if (dbl)
    return launch_cheb2d<P, double, double>(xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr,
                                            store_d, cpb, st);
  if (gt == G_BF16)
    return launch_cheb2d<P, float, uint16_t>(xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr,
                                             store_d, cpb, st);
  return launch_cheb2d<P, float, float>(xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr, store_d,
                                        cpb, st);
}

hipError_t cheb2d(int P, bool dbl, GType gt, const void* xi, void* xo, void* d, const void* b,
                  const void* dinv, const void* G, int Nx, int Nz, int masked, double cd,
                  double cr, int store_d, hipStream_t st) {
  acct_add(vsz(dbl) * nodes2(P, Nx, Nz) * (4 + (cd != 0.0) + (store_d ? 1 : 0)) + gbytes2(gt, P, Nx, Nz));
  const int cpb = cheb2d_cpb(P, Nx, Nz, dbl);
  if (xi == xo) return hipErrorInvalidValue;
  switch (P) {
    case 1: return cheb2d_p<1>(dbl, gt, xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr, store_d, cpb, st);
    case 2: return cheb2d_p<2>(dbl, gt, xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr, store_d, cpb, st);
    case 3: return cheb2d_p<3>(dbl, gt, xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr, store_d, cpb, st);
    case 4: return cheb2d_p<4>(dbl, gt, xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr, store_d, cpb, st);
    case 5: return cheb2d_p<5>(dbl, gt, xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr, store_d, cpb, st);
    case 6: return cheb2d_p<6>(dbl, gt, xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr, store_d, cpb, st);
    case 7: return cheb2d_p<7>(dbl, gt, xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr, store_d, cpb, st);
    case 8: return cheb2d_p<8>(dbl, gt, xi, xo, d, b, dinv, G, Nx, Nz, masked, cd, cr, store_d, cpb, st);
    default: return hipErrorInvalidValue;
  }
}

// Assembly of the element-local corrections of the learned stage fused with the operator:
// c[g] = average of CE[e][local(g)] over the elements e holding node g (zero on the Dirichlet
// surface when masked; contributions added in the order (left, lower), (left, upper),
// (right, lower), (right, upper) element, as stage_assemble does), q = A c complete at every
// node, and each workgroup's part of c . q in dotp[workgroup].  Halo layout as in k_cheb2d; CE in
// the layout of ce_index.
template <int P, typename T, typename TG>
__global__ __launch_bounds__(1024) void k_stagecq2d(const float* __restrict__ CE,
                                                    T* __restrict__ c, T* __restrict__ q,
                                                    const TG* __restrict__ G, int Nx, int Nz,
                                                    int masked, int cpb, int remap,
                                                    double* __restrict__ dotp) {
  constexpr int NP = P + 1;
  constexpr int V = lds_vec<T>();
  constexpr int NPp = (NP + V - 1) / V * V;
  const int nzn = Nz * P + 1;
  const int nzp = (nzn + V - 1) / V * V;
  const int nthr = NP * Nz;
  int bx = blockIdx.x;
  if (remap) {
    const int per = gridDim.x >> 3;
    bx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  const int cs = threadIdx.x / nthr;
  const int t = threadIdx.x - cs * nthr;
  const int ex = bx * cpb + cs - 1;
  const bool valid = cs <= cpb && ex >= 0 && ex < Nx;
  const int slot = slot2d_elems<int>(NP, Nz, nzp, V);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* base = reinterpret_cast<T*>(smem_raw) + (valid ? cs : 0) * slot;
  T xin[NP];
  column_apply<P, T, TG>(
      [&](T(&v)[NP]) {
        const int qz = t / P, rz = t - qz * P;
        const bool zl = rz == 0 && qz > 0, zr = qz < Nz;
        const bool top = masked && t == nzn - 1;
        // every candidate is loaded unconditionally (indices clamped into the array) so that all
        // loads are in flight together; absent ones enter as exact zeros, in the same order
        const int zlo = zl ? qz - 1 : 0, zhi = zr ? qz : Nz - 1;
        float cv[NP][4];
#pragma unroll
        for (int l = 0; l < NP; ++l) {
          const int cl = l == 0 ? (ex > 0 ? ex - 1 : 0) : ex;
          const int cr = l == P ? (ex + 1 < Nx ? ex + 1 : ex) : ex, ir = l == P ? 0 : l;
          cv[l][0] = CE[ce_index(cl, P, zlo, P, Nz, NP)];
          cv[l][1] = CE[ce_index(cl, P, zhi, zr ? rz : 0, Nz, NP)];
          cv[l][2] = CE[ce_index(cr, ir, zlo, P, Nz, NP)];
          cv[l][3] = CE[ce_index(cr, ir, zhi, zr ? rz : 0, Nz, NP)];
        }
#pragma unroll
        for (int l = 0; l < NP; ++l) {
          // element columns left and right of line l of column ex
          const bool xl = l == 0 ? ex > 0 : l == P;
          const bool xr = l == P ? ex + 1 < Nx : true;
          const bool m0 = xl && zl, m1 = xl && zr, m2 = xr && zl, m3 = xr && zr;
          float sacc = 0.f;
          sacc += m0 ? cv[l][0] : 0.f;
          sacc += m1 ? cv[l][1] : 0.f;
          sacc += m2 ? cv[l][2] : 0.f;
          sacc += m3 ? cv[l][3] : 0.f;
          const int cnt = (int)m0 + (int)m1 + (int)m2 + (int)m3;
          v[l] = top ? (T)0 : (T)(sacc / (float)cnt);
        }
      },
      G, valid ? ex : 0, nthr, t, valid, Nz, nzn, nzp, masked, base, xin, [] {});

  double part = 0.0;
  if (cs >= 1 && valid && t < nzn) {
    const T* su = base + Nz * NP * NPp;
    const T* sl = su - slot;
    const bool left = ex > 0 && !(masked && t == nzn - 1);
    const int nl = (ex == Nx - 1) ? NP : P;
    const size_t g0 = (size_t)ex * P * nzn + t;
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      if (l < nl) {
        T ax = su[l * nzp + t];
        if (l == 0 && left) ax += sl[P * nzp + t];
        const size_t g = g0 + (size_t)l * nzn;
        c[g] = xin[l];
        q[g] = ax;
        part += (double)xin[l] * (double)ax;
      }
    }
  }
  __shared__ double red[16];
  const double tot = block_sum(part, red);
  if (threadIdx.x == 0) dotp[blockIdx.x] = tot;
}

template <int P, typename T, typename TG>
static hipError_t launch_stagecq2d(const float* CE, void* c, void* q, const void* G, int Nx,
                                   int Nz, int masked, double* dotp, int cpb, hipStream_t st) {
  const bool dbl = sizeof(T) == 8;
  const int nthr = (P + 1) * Nz;
  const int threads = (((cpb + 1) * nthr + 63) / 64) * 64;
  const int blocks = (Nx + cpb - 1) / cpb;
  const size_t smem = apply2d_smem(P, Nz, dbl) * (cpb + 1);
  if (cpb <= 0 || threads > 1024 || smem > 160 * 1024) return hipErrorInvalidValue;
  const int remap = (blocks % 8 == 0) ? 1 : 0;
  hipError_t e = allow_lds(k_stagecq2d<P, T, TG>, smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stagecq2d<P, T, TG>), dim3(blocks), dim3(threads), smem, st, CE, (T*)c,
                     (T*)q, (const TG*)G, Nx, Nz, masked, cpb, remap, dotp);
  return hipGetLastError();
}

template <int P>
static hipError_t stagecq2d_p(bool dbl, GType gt, const float* CE, void* c, void* q,
                              const void* G, int Nx, int Nz, int masked, double* dotp, int cpb,
                              hipStream_t st) {
  if (gt == G_COL64)
    return dbl ? launch_stagecq2d<P, double, ColGeo64>(CE, c, q, G, Nx, Nz, masked, dotp, cpb, st)
               : launch_stagecq2d<P, float, ColGeo64>(CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
  if (dbl) return launch_stagecq2d<P, double, double>(CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
  if (gt == G_BF16)
    return launch_stagecq2d<P, float, uint16_t>(CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
  return launch_stagecq2d<P, float, float>(CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
}

int cheb2d_blocks(int P, int Nx, int Nz, bool dbl) {
  const int cpb = cheb2d_cpb(P, Nx, Nz, dbl);
  return cpb > 0 ? (Nx + cpb - 1) / cpb : 0;
}

hipError_t stagecq2d(int P, bool dbl, GType gt, const float* CE, void* c, void* q, const void* G,
                     int Nx, int Nz, int masked, double* dotp, hipStream_t st) {
  acct_add(4.0 * local2(P, Nx, Nz) + 2 * vsz(dbl) * nodes2(P, Nx, Nz) + gbytes2(gt, P, Nx, Nz));
  const int cpb = P <= 8 ? cheb2d_cpb(P, Nx, Nz, dbl) : 0;
  if (cpb <= 0) return hipErrorInvalidValue;
  switch (P) {
    case 1: return stagecq2d_p<1>(dbl, gt, CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
    case 2: return stagecq2d_p<2>(dbl, gt, CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
    case 3: return stagecq2d_p<3>(dbl, gt, CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
    case 4: return stagecq2d_p<4>(dbl, gt, CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
    case 5: return stagecq2d_p<5>(dbl, gt, CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
    case 6: return stagecq2d_p<6>(dbl, gt, CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
    case 7: return stagecq2d_p<7>(dbl, gt, CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
    case 8: return stagecq2d_p<8>(dbl, gt, CE, c, q, G, Nx, Nz, masked, dotp, cpb, st);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------------------------------
// additive Schwarz smoothing (Sec. 5.3), element blocks
// ------------------------------------------------------------------------------------------
// z_e = (R_e A R_e^T)^{-1} R_e r for every element: one thread per row of an element block,
// 256 / (P+1)^2 elements per workgroup; the element's residual is staged in LDS and the
// (symmetric) inverse read column by column, so consecutive rows read consecutive addresses.
// Ainv: [E][n][n] (element e = ex Nz + ez); z in the layout of ce_index.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_asm_local(const T* __restrict__ r,
                                                   const T* __restrict__ Ainv, T* __restrict__ z,
                                                   int E, int Nz, int nzn) {
  constexpr int NP = P + 1, n = NP * NP, EPB = 256 / n;
  __shared__ T sr[EPB][n];
  const int el = threadIdx.x / n, row = threadIdx.x - el * n;
  const int e = blockIdx.x * EPB + el;
  const bool act = el < EPB && e < E;
  const int ex = act ? e / Nz : 0, ez = act ? e - ex * Nz : 0;
  const int i = row / NP, j = row - (row / NP) * NP;
  if (act) sr[el][row] = r[(size_t)(ex * P + i) * nzn + ez * P + j];
  __syncthreads();
  if (!act) return;
  const T* Ae = Ainv + (size_t)e * n * n + row;
  T acc = 0;
#pragma unroll 9
  for (int k = 0; k < n; ++k) acc += Ae[(size_t)k * n] * sr[el][k];
  z[ce_index(ex, i, ez, j, Nz, NP)] = acc;
}

// x = (set ? 0 : x) + W sum_e R_e^T z_e: at every node the average of the block results of the
// elements holding it (fixed order: (left, lower), (left, upper), (right, lower), (right,
// upper)); the Dirichlet surface keeps x (zero there in the V-cycle) when masked.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_asm_add(const T* __restrict__ z, T* __restrict__ x,
                                                 int Nx, int Nz, unsigned nzn, unsigned N,
                                                 int masked, int set) {
  constexpr int NP = P + 1;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    const int ix = g / nzn, iz = g - ix * nzn;
    if (masked && iz == (int)nzn - 1) {
      if (set) x[g] = (T)0;
      continue;
    }
    const int qx = ix / P, rx = ix - qx * P, qz = iz / P, rz = iz - qz * P;
    const bool xl = rx == 0 && qx > 0, xr = qx < Nx, zl = rz == 0 && qz > 0, zr = qz < Nz;
    T s = 0;
    int cnt = 0;
    if (xl && zl) { s += z[ce_index(qx - 1, P, qz - 1, P, Nz, NP)]; ++cnt; }
    if (xl && zr) { s += z[ce_index(qx - 1, P, qz, rz, Nz, NP)]; ++cnt; }
    if (xr && zl) { s += z[ce_index(qx, rx, qz - 1, P, Nz, NP)]; ++cnt; }
    if (xr && zr) { s += z[ce_index(qx, rx, qz, rz, Nz, NP)]; ++cnt; }
    const T c = s / (T)cnt;
    x[g] = set ? c : x[g] + c;
  }
}

template <int P>
static hipError_t asm_p(bool dbl, const void* r, const void* Ainv, void* z, void* x, int Nx,
                        int Nz, int masked, int set, hipStream_t st) {
  constexpr int n = (P + 1) * (P + 1), EPB = 256 / n;
  const int E = Nx * Nz, nzn = Nz * P + 1;
  const unsigned N = (unsigned)((size_t)(Nx * P + 1) * nzn);
  const unsigned b1 = (unsigned)((E + EPB - 1) / EPB), b2 = std::min(nblk(N, 256), 8192u);
  if (dbl) {
    hipLaunchKernelGGL((k_asm_local<P, double>), dim3(b1), dim3(256), 0, st, (const double*)r,
                       (const double*)Ainv, (double*)z, E, Nz, nzn);
    hipLaunchKernelGGL((k_asm_add<P, double>), dim3(b2), dim3(256), 0, st, (const double*)z,
                       (double*)x, Nx, Nz, (unsigned)nzn, N, masked, set);
  } else {
    hipLaunchKernelGGL((k_asm_local<P, float>), dim3(b1), dim3(256), 0, st, (const float*)r,
                       (const float*)Ainv, (float*)z, E, Nz, nzn);
    hipLaunchKernelGGL((k_asm_add<P, float>), dim3(b2), dim3(256), 0, st, (const float*)z,
                       (float*)x, Nx, Nz, (unsigned)nzn, N, masked, set);
  }
  return hipGetLastError();
}

hipError_t asm_sweep(int P, bool dbl, const void* r, const void* Ainv, void* z, void* x, int Nx,
                     int Nz, int masked, int set, hipStream_t st) {
  acct_add(vsz(dbl) * (local2(P, Nx, Nz) * ((P + 1) * (P + 1) + 2) + nodes2(P, Nx, Nz) * (set ? 2 : 3)));
  switch (P) {
    case 1: return asm_p<1>(dbl, r, Ainv, z, x, Nx, Nz, masked, set, st);
    case 2: return asm_p<2>(dbl, r, Ainv, z, x, Nx, Nz, masked, set, st);
    case 3: return asm_p<3>(dbl, r, Ainv, z, x, Nx, Nz, masked, set, st);
    case 4: return asm_p<4>(dbl, r, Ainv, z, x, Nx, Nz, masked, set, st);
    case 5: return asm_p<5>(dbl, r, Ainv, z, x, Nx, Nz, masked, set, st);
    case 6: return asm_p<6>(dbl, r, Ainv, z, x, Nx, Nz, masked, set, st);
    case 7: return asm_p<7>(dbl, r, Ainv, z, x, Nx, Nz, masked, set, st);
    case 8: return asm_p<8>(dbl, r, Ainv, z, x, Nx, Nz, masked, set, st);
    default: return hipErrorInvalidValue;
  }
}

// One FPCG direction step of the outer loop fused with the FP64 operator (2D, halo layout of
// k_cheb2d): every node's p = z + beta p_old (first: p = z) is formed while loading, with
// beta = -alpha_old (z.q_old) / (r.z)_old and alpha_old = (r.z)_old / (p.q)_old from the partial
// sets prz_old, ppq_old, pzq; then q = A p, complete at every owned node, and each workgroup's
// part of p . q into ppq_new.  p itself is not written here (other workgroups still read the old
// p); block 0 stores beta in *beta_out for the update kernel.
template <int P, bool COL>
__global__ __launch_bounds__(1024) void k_fpcg2d(const double* __restrict__ z,
                                                 const double* __restrict__ p,
                                                 double* __restrict__ q,
                                                 const double* __restrict__ G, int Nx, int Nz,
                                                 int masked, int cpb, int remap,
                                                 const double* __restrict__ prz_old,
                                                 const double* __restrict__ ppq_old,
                                                 const double* __restrict__ pzq, int first,
                                                 double* __restrict__ ppq_new,
                                                 double* __restrict__ beta_out) {
  constexpr int NP = P + 1;
  constexpr int V = lds_vec<double>();
  constexpr int NPp = (NP + V - 1) / V * V;
  const int nzn = Nz * P + 1;
  const int nzp = (nzn + V - 1) / V * V;
  const int nthr = NP * Nz;
  __shared__ double sh[16];
  int bx = blockIdx.x;
  if (remap) {
    const int per = gridDim.x >> 3;
    bx = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  }
  const int cs = threadIdx.x / nthr;
  const int t = threadIdx.x - cs * nthr;
  const int ex = bx * cpb + cs - 1;
  const bool valid = cs <= cpb && ex >= 0 && ex < Nx;
  const int slot = slot2d_elems<int>(NP, Nz, nzp, V);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* base = reinterpret_cast<double*>(smem_raw) + (valid ? cs : 0) * slot;
  const size_t cb = (size_t)(valid ? ex : 0) * P * nzn + t;
  // every global input is requested before beta is formed: the factors, z and p of this
  // thread's nodes and the three partial-sum sets (each summed in the order sum_partials uses)
  double g[3][NP], zr[NP], pr[NP];
  if constexpr (COL) {
    if (valid) load_g2d<P, double, ColGeo64>(reinterpret_cast<const ColGeo64*>(G), ex, nthr, t, g);
  } else {
    if (valid) load_g2d<P, double, double>(G, valid ? ex : 0, nthr, t, g);
  }
  if (valid && t < nzn) {
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      zr[l] = z[cb + (size_t)l * nzn];
      pr[l] = first ? 0.0 : p[cb + (size_t)l * nzn];
    }
  }
  double beta = 0.0;
  if (!first) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int u = 0; u < NRED / 64; ++u) {
      const int k = (int)threadIdx.x + u * (int)blockDim.x;
      if (k < NRED) {
        a0 += prz_old[k];
        a1 += ppq_old[k];
        a2 += pzq[k];
      }
    }
    const double rz = block_sum(a0, sh);
    const double pq = block_sum(a1, sh);
    const double zq = block_sum(a2, sh);
    beta = -(rz / pq) * zq / rz;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *beta_out = beta;
  double xin[NP];
  column_apply_g<P, double>(
      g,
      [&](double(&v)[NP]) {
#pragma unroll
        for (int l = 0; l < NP; ++l) v[l] = first ? zr[l] : fma(beta, pr[l], zr[l]);
      },
      t, valid, Nz, nzn, nzp, masked, base, xin, [] {});
  double part = 0.0;
  if (cs >= 1 && valid && t < nzn) {
    const double* su = base + Nz * NP * NPp;
    const double* sl = su - slot;
    const bool left = ex > 0 && !(masked && t == nzn - 1);
    const int nl = (ex == Nx - 1) ? NP : P;
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      if (l < nl) {
        double ax = su[l * nzp + t];
        if (l == 0 && left) ax += sl[P * nzp + t];
        q[cb + (size_t)l * nzn] = ax;
        part += xin[l] * ax;
      }
    }
  }
  const double tot = block_sum(part, sh);
  if (threadIdx.x == 0) ppq_new[blockIdx.x] = tot;
}

template <int P, bool COL>
static hipError_t launch_fpcg2d(const double* z, const double* p, double* q, const double* G,
                                int Nx, int Nz, int masked, const double* prz_old,
                                const double* ppq_old, const double* pzq, int first,
                                double* ppq_new, double* beta_out, hipStream_t st) {
  const int cpb = cheb2d_cpb(P, Nx, Nz, true);
  if (cpb <= 0) return hipErrorInvalidValue;
  const int nthr = (P + 1) * Nz;
  const int threads = (((cpb + 1) * nthr + 63) / 64) * 64;
  const int blocks = (Nx + cpb - 1) / cpb;
  const size_t smem = apply2d_smem(P, Nz, true) * (cpb + 1);
  if (threads > 1024 || smem > 160 * 1024 || blocks > NRED) return hipErrorInvalidValue;
  const int remap = (blocks % 8 == 0) ? 1 : 0;
  hipError_t e = allow_lds(k_fpcg2d<P, COL>, smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fpcg2d<P, COL>), dim3(blocks), dim3(threads), smem, st, z, p, q, G, Nx,
                     Nz, masked, cpb, remap, prz_old, ppq_old, pzq, first, ppq_new, beta_out);
  return hipGetLastError();
}

bool fpcg2d_fits(int P, int Nx, int Nz) {
  return P >= 1 && P <= 8 && cheb2d_blocks(P, Nx, Nz, true) > 0 &&
         cheb2d_blocks(P, Nx, Nz, true) <= NRED;
}

hipError_t fpcg2d(int P, const double* z, const double* p, double* q, const double* G, int Nx,
                  int Nz, int masked, const double* prz_old, const double* ppq_old,
                  const double* pzq, int first, double* ppq_new, double* beta_out,
                  hipStream_t st, int col) {
  acct_add(8.0 * nodes2(P, Nx, Nz) * (first ? 2 : 3) +
           (col ? 8.0 * COLGEO_N * Nx * (P + 1) : 24.0 * local2(P, Nx, Nz)));
  switch (P) {
#define SEM_FPCG2D(PP) \
  case PP: return col ? launch_fpcg2d<PP, true>(z, p, q, G, Nx, Nz, masked, prz_old, ppq_old, pzq, first, ppq_new, beta_out, st) \
                      : launch_fpcg2d<PP, false>(z, p, q, G, Nx, Nz, masked, prz_old, ppq_old, pzq, first, ppq_new, beta_out, st);
    SEM_FPCG2D(1) SEM_FPCG2D(2) SEM_FPCG2D(3) SEM_FPCG2D(4)
    SEM_FPCG2D(5) SEM_FPCG2D(6) SEM_FPCG2D(7) SEM_FPCG2D(8)
#undef SEM_FPCG2D
    default: return hipErrorInvalidValue;
  }
}

// the FPCG update after k_fpcg2d: p = z + beta p (first: p = z, beta from k_fpcg2d, the same
// fused multiply-add), alpha = (r.z) / (p.q) from prz_new and ppq_new; x += alpha p,
// r -= alpha q, partials of r.r into prr; block 0 moves the partial sets for the next
// iteration (prz_new -> prz_old, ppq_new -> ppq_old)
__global__ __launch_bounds__(RED_THREADS) void k_update_xrp(
    double* __restrict__ x, double* __restrict__ r, double* __restrict__ p,
    const double* __restrict__ z, const double* __restrict__ q, const double* __restrict__ beta_in,
    int first, const double* prz_new, const double* ppq_new, double* prz_old, double* ppq_old,
    double* prr, unsigned N) {
  __shared__ double sh[16];
  // the partial sums and the first batch of vector values are loaded together; elements are
  // visited in the grid-stride order (U per batch), so every sum keeps its order
  constexpr int U = 8, NP = NRED / RED_THREADS;
  double hz[NP], hq[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    hz[k] = prz_new[threadIdx.x + k * RED_THREADS];
    hq[k] = ppq_new[threadIdx.x + k * RED_THREADS];
  }
  const double beta = *beta_in;
  const unsigned stride = gridDim.x * blockDim.x;
  double alpha = 0.0, a = 0.0;
  for (size_t g0 = 0; g0 < N; g0 += (size_t)U * stride) {  // uniform trip count
    double zv[U], pv[U], xv[U], rv[U], qv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t g = g0 + blockIdx.x * blockDim.x + threadIdx.x + (size_t)u * stride;
      const bool ok = g < N;
      zv[u] = ok ? z[g] : 0.0;
      pv[u] = (ok && !first) ? p[g] : 0.0;
      xv[u] = ok ? x[g] : 0.0;
      rv[u] = ok ? r[g] : 0.0;
      qv[u] = ok ? q[g] : 0.0;
    }
    if (g0 == 0) {
      double sz = 0.0, sq = 0.0;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        sz += hz[k];
        sq += hq[k];
      }
      const double rz = block_sum(sz, sh);
      const double pq = block_sum(sq, sh);
      alpha = rz / pq;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t g = g0 + blockIdx.x * blockDim.x + threadIdx.x + (size_t)u * stride;
      if (g < N) {
        const double pn = first ? zv[u] : fma(beta, pv[u], zv[u]);
        p[g] = pn;
        x[g] = xv[u] + alpha * pn;
        const double rn = rv[u] - alpha * qv[u];
        r[g] = rn;
        a += rn * rn;
      }
    }
  }
  a = block_sum(a, sh);
  if (threadIdx.x == 0) prr[blockIdx.x] = a;
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < NRED; k += blockDim.x) {
      prz_old[k] = prz_new[k];
      ppq_old[k] = ppq_new[k];
    }
}

hipError_t update_xrp(double* x, double* r, double* p, const double* z, const double* q,
                      const double* beta, int first, const double* prz_new,
                      const double* ppq_new, double* prz_old, double* ppq_old, double* prr,
                      unsigned N, hipStream_t st) {
  acct_add(64.0 * N);
  hipLaunchKernelGGL(k_update_xrp, dim3(NRED), dim3(RED_THREADS), 0, st, x, r, p, z, q, beta,
                     first, prz_new, ppq_new, prz_old, ppq_old, prr, N);
  return hipGetLastError();
}

template <typename T>
__global__ void k_resid_fix(const T* __restrict__ b, const T* __restrict__ y,
                            const T* __restrict__ S, T* __restrict__ r, unsigned N, unsigned nzn,
                            unsigned P) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    r[g] = b[g] - ax_at(y, S, g, nzn, P);
}

template <int P, typename T, typename TG>
static hipError_t launch_cheb2d_first(void* x, void* d, void* b, const double* r64,
                                      const void* dinv, const void* G, int Nx, int Nz,
                                      int masked, double cr0, double cd, double cr, int store_d,
                                      hipStream_t st) {
  const bool dbl = sizeof(T) == 8;
  const int cpb = cheb2d_cpb(P, Nx, Nz, dbl);
  if (cpb <= 0) return hipErrorInvalidValue;
  const int nthr = (P + 1) * Nz;
  const int threads = (((cpb + 1) * nthr + 63) / 64) * 64;
  const int blocks = (Nx + cpb - 1) / cpb;
  const size_t smem = apply2d_smem(P, Nz, dbl) * (cpb + 1);
  if (threads > 1024 || smem > 160 * 1024) return hipErrorInvalidValue;
  const int remap = (blocks % 8 == 0) ? 1 : 0;
  hipError_t e = allow_lds(k_cheb2d_first<P, T, TG>, smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_cheb2d_first<P, T, TG>), dim3(blocks), dim3(threads), smem, st, (T*)x,
                     (T*)d, (T*)b, r64, (const T*)dinv, (const TG*)G, Nx, Nz, masked, cpb,
                     remap, (T)cr0, (T)cd, (T)cr, store_d);
  return hipGetLastError();
}

template <int P>
static hipError_t cheb2d_first_p(bool dbl, GType gt, void* x, void* d, void* b,
                                 const double* r64, const void* dinv, const void* G, int Nx,
                                 int Nz, int masked, double cr0, double cd, double cr,
                                 int store_d, hipStream_t st) {
  if (gt == G_COL64)
    return dbl ? launch_cheb2d_first<P, double, ColGeo64>(x, d, b, r64, dinv, G, Nx, Nz, masked,
                                                          cr0, cd, cr, store_d, st)
               : launch_cheb2d_first<P, float, ColGeo64>(x, d, b, r64, dinv, G, Nx, Nz, masked,
                                                         cr0, cd, cr, store_d, st);
  if (dbl)
    return launch_cheb2d_first<P, double, double>(x, d, b, r64, dinv, G, Nx, Nz, masked, cr0,
                                                  cd, cr, store_d, st);
  if (gt == G_BF16)
    return launch_cheb2d_first<P, float, uint16_t>(x, d, b, r64, dinv, G, Nx, Nz, masked, cr0,
                                                   cd, cr, store_d, st);
  return launch_cheb2d_first<P, float, float>(x, d, b, r64, dinv, G, Nx, Nz, masked, cr0, cd,
                                              cr, store_d, st);
}

hipError_t cheb2d_first(int P, bool dbl, GType gt, void* x, void* d, void* b, const double* r64,
                        const void* dinv, const void* G, int Nx, int Nz, int masked, double cr0,
                        double cd, double cr, int store_d, hipStream_t st) {
  acct_add(nodes2(P, Nx, Nz) * ((r64 ? 8.0 + vsz(dbl) : vsz(dbl)) + vsz(dbl) * (2 + (store_d ? 1 : 0))) + gbytes2(gt, P, Nx, Nz));
  switch (P) {
#define SEM_CHEB_FIRST(PP)                                                                  \
  case PP:                                                                                  \
    return cheb2d_first_p<PP>(dbl, gt, x, d, b, r64, dinv, G, Nx, Nz, masked, cr0, cd, cr, \
                              store_d, st);
    SEM_CHEB_FIRST(1) SEM_CHEB_FIRST(2) SEM_CHEB_FIRST(3) SEM_CHEB_FIRST(4)
    SEM_CHEB_FIRST(5) SEM_CHEB_FIRST(6) SEM_CHEB_FIRST(7) SEM_CHEB_FIRST(8)
#undef SEM_CHEB_FIRST
    default: return hipErrorInvalidValue;
  }
}

template <int P>
static hipError_t resid2d_p(bool dbl, GType gt, const void* x, void* r, const void* b,
                            const void* G, int Nx, int Nz, int masked, int cpb, hipStream_t st) {
  if (gt == G_COL64)
    return dbl ? launch_cheb2d<P, double, ColGeo64, 1>(x, r, nullptr, b, nullptr, G, Nx, Nz,
                                                       masked, 0.0, 0.0, 0, cpb, st)
               : launch_cheb2d<P, float, ColGeo64, 1>(x, r, nullptr, b, nullptr, G, Nx, Nz,
                                                      masked, 0.0, 0.0, 0, cpb, st);
  if (dbl)
    return launch_cheb2d<P, double, double, 1>(x, r, nullptr, b, nullptr, G, Nx, Nz, masked, 0.0,
                                               0.0, 0, cpb, st);
  if (gt == G_BF16)
    return launch_cheb2d<P, float, uint16_t, 1>(x, r, nullptr, b, nullptr, G, Nx, Nz, masked, 0.0,
                                                0.0, 0, cpb, st);
  return launch_cheb2d<P, float, float, 1>(x, r, nullptr, b, nullptr, G, Nx, Nz, masked, 0.0, 0.0,
                                           0, cpb, st);
}

hipError_t apply2d(int P, bool dbl, GType gt, const void* x, void* y, void* S, const void* G,
                   int Nx, int Nz, int masked, hipStream_t st);

hipError_t resid2d(int P, bool dbl, GType gt, const void* x, void* r, const void* b,
                   const void* G, int Nx, int Nz, int masked, void* y, void* S, hipStream_t st) {
  if (x == r) return hipErrorInvalidValue;
  const int cpb = P <= 8 ? cheb2d_cpb(P, Nx, Nz, dbl) : 0;
  acct_add(cpb > 0 ? 3 * vsz(dbl) * nodes2(P, Nx, Nz) + gbytes2(gt, P, Nx, Nz)
                   : vsz(dbl) * nodes2(P, Nx, Nz));
  if (cpb > 0) {
    switch (P) {
      case 1: return resid2d_p<1>(dbl, gt, x, r, b, G, Nx, Nz, masked, cpb, st);
      case 2: return resid2d_p<2>(dbl, gt, x, r, b, G, Nx, Nz, masked, cpb, st);
      case 3: return resid2d_p<3>(dbl, gt, x, r, b, G, Nx, Nz, masked, cpb, st);
      case 4: return resid2d_p<4>(dbl, gt, x, r, b, G, Nx, Nz, masked, cpb, st);
      case 5: return resid2d_p<5>(dbl, gt, x, r, b, G, Nx, Nz, masked, cpb, st);
      case 6: return resid2d_p<6>(dbl, gt, x, r, b, G, Nx, Nz, masked, cpb, st);
      case 7: return resid2d_p<7>(dbl, gt, x, r, b, G, Nx, Nz, masked, cpb, st);
      case 8: return resid2d_p<8>(dbl, gt, x, r, b, G, Nx, Nz, masked, cpb, st);
      default: return hipErrorInvalidValue;
    }
  }
  // columns too tall for the fused form: operator with side buffer, then r = b - (y + S)
  hipError_t e = apply2d(P, dbl, gt, x, y, S, G, Nx, Nz, masked, st);
  if (e != hipSuccess) return e;
  const unsigned N = (unsigned)((size_t)(Nx * P + 1) * (Nz * P + 1));
  const unsigned blocks = std::min(nblk(N, 256), 8192u);
  if (dbl)
    hipLaunchKernelGGL(k_resid_fix<double>, dim3(blocks), dim3(256), 0, st, (const double*)b,
                       (const double*)y, (const double*)S, (double*)r, N, (unsigned)(Nz * P + 1),
                       (unsigned)P);
  else
    hipLaunchKernelGGL(k_resid_fix<float>, dim3(blocks), dim3(256), 0, st, (const float*)b,
                       (const float*)y, (const float*)S, (float*)r, N, (unsigned)(Nz * P + 1),
                       (unsigned)P);
  return hipGetLastError();
}

template <int P, typename T, typename TG, bool DOT = false>
static hipError_t launch_apply2d(const void* x, void* y, void* S, const void* G, int Nx, int Nz,
                                 int masked, double* dotp, hipStream_t st) {
  const bool dbl = sizeof(T) == 8;
  const int nthr = (P + 1) * Nz;
  const int cpb = apply2d_cpb(P, Nx, Nz, dbl);
  const int threads = ((cpb * nthr + 63) / 64) * 64;
  const int blocks = (Nx + cpb - 1) / cpb;
  const size_t smem = apply2d_smem(P, Nz, dbl) * cpb;
  const int remap = (blocks % 8 == 0) ? 1 : 0;
  hipError_t e = allow_lds(k_apply2d<P, T, TG, DOT>, smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_apply2d<P, T, TG, DOT>), dim3(blocks), dim3(threads), smem, st,
                     (const T*)x, (T*)y, (T*)S, (const TG*)G, Nx, Nz, masked, cpb, remap, dotp);
  return hipGetLastError();
}

template <int P>
static hipError_t apply2d_p(bool dbl, GType gt, const void* x, void* y, void* S, const void* G,
                            int Nx, int Nz, int masked, hipStream_t st) {
  if (gt == G_COL64)
    return dbl ? launch_apply2d<P, double, ColGeo64>(x, y, S, G, Nx, Nz, masked, nullptr, st)
               : launch_apply2d<P, float, ColGeo64>(x, y, S, G, Nx, Nz, masked, nullptr, st);
  if (dbl) return launch_apply2d<P, double, double>(x, y, S, G, Nx, Nz, masked, nullptr, st);
  if (gt == G_BF16)
    return launch_apply2d<P, float, uint16_t>(x, y, S, G, Nx, Nz, masked, nullptr, st);
  return launch_apply2d<P, float, float>(x, y, S, G, Nx, Nz, masked, nullptr, st);
}

hipError_t apply2d(int P, bool dbl, GType gt, const void* x, void* y, void* S, const void* G,
                   int Nx, int Nz, int masked, hipStream_t st) {
  acct_add(2 * vsz(dbl) * nodes2(P, Nx, Nz) +
           gbytes2(gt, P, Nx, Nz));
  switch (P) {
    case 1: return apply2d_p<1>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 2: return apply2d_p<2>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 3: return apply2d_p<3>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 4: return apply2d_p<4>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 5: return apply2d_p<5>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 6: return apply2d_p<6>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 7: return apply2d_p<7>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 8: return apply2d_p<8>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 9: return apply2d_p<9>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 10: return apply2d_p<10>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 11: return apply2d_p<11>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    case 12: return apply2d_p<12>(dbl, gt, x, y, S, G, Nx, Nz, masked, st);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
static hipError_t apply2d_dot_p(bool dbl, GType gt, const void* x, void* y, void* S,
                                const void* G, int Nx, int Nz, int masked, double* dotp,
                                hipStream_t st) {
  if (gt == G_COL64)
    return dbl ? launch_apply2d<P, double, ColGeo64, true>(x, y, S, G, Nx, Nz, masked, dotp, st)
               : launch_apply2d<P, float, ColGeo64, true>(x, y, S, G, Nx, Nz, masked, dotp, st);
  if (dbl) return launch_apply2d<P, double, double, true>(x, y, S, G, Nx, Nz, masked, dotp, st);
  if (gt == G_BF16)
    return launch_apply2d<P, float, uint16_t, true>(x, y, S, G, Nx, Nz, masked, dotp, st);
  return launch_apply2d<P, float, float, true>(x, y, S, G, Nx, Nz, masked, dotp, st);
}

hipError_t apply2d_dot(int P, bool dbl, GType gt, const void* x, void* y, void* S, const void* G,
                       int Nx, int Nz, int masked, double* dotp, hipStream_t st) {
  acct_add(2 * vsz(dbl) * nodes2(P, Nx, Nz) + gbytes2(gt, P, Nx, Nz));
  switch (P) {
    case 1: return apply2d_dot_p<1>(dbl, gt, x, y, S, G, Nx, Nz, masked, dotp, st);
    case 2: return apply2d_dot_p<2>(dbl, gt, x, y, S, G, Nx, Nz, masked, dotp, st);
    case 3: return apply2d_dot_p<3>(dbl, gt, x, y, S, G, Nx, Nz, masked, dotp, st);
    case 4: return apply2d_dot_p<4>(dbl, gt, x, y, S, G, Nx, Nz, masked, dotp, st);
    case 5: return apply2d_dot_p<5>(dbl, gt, x, y, S, G, Nx, Nz, masked, dotp, st);
    case 6: return apply2d_dot_p<6>(dbl, gt, x, y, S, G, Nx, Nz, masked, dotp, st);
    case 7: return apply2d_dot_p<7>(dbl, gt, x, y, S, G, Nx, Nz, masked, dotp, st);
    case 8: return apply2d_dot_p<8>(dbl, gt, x, y, S, G, Nx, Nz, masked, dotp, st);
    default: return hipErrorInvalidValue;
  }
}

int apply2d_blocks(int P, int Nx, int Nz, bool dbl) {
  const int cpb = apply2d_cpb(P, Nx, Nz, dbl);
  return (Nx + cpb - 1) / cpb;
}

// ------------------------------------------------------------------------------------------
// 3D operator apply (sigma-mapped hexahedra; element matrices as in 2D with the five factors
// G_rr, G_tt, G_rs, G_ts, G_ss; G_rt = 0 because x and y are affine and independent)
// ------------------------------------------------------------------------------------------
// LDS per element column: four exchange arrays [Nz][NP][NP][NPp]; the space of the last two
// also holds the input/output column [NP(i)][NP(m)][nzp] and the element-top values
// [Nz][NP][NP] in the phases where they are dead
static size_t apply3d_slot(int P, int Nz, bool dbl) {
  const int NP = P + 1, V = dbl ? 2 : 4, NPp = (NP + V - 1) / V * V;
  const int nzp = (Nz * P + 1 + V - 1) / V * V;
  const size_t ex = (size_t)Nz * NP * NP * NPp;  // one exchange array
  const size_t col = (size_t)NP * NP * nzp + (size_t)Nz * NP * NP;
  const size_t n = 2 * ex + std::max(2 * ex, col);
  return (n + V - 1) / V * V;
}

size_t apply3d_smem(int P, int Nz, bool dbl) { return apply3d_slot(P, Nz, dbl) * (dbl ? 8 : 4); }

// G_COL64 in 3D: the factors of thread t = (ez NP + i) NP + m (vertical line (i, m) of element
// ez) formed from the record of column c, node (i, m): {W K d r_x^2, W K s_s^2 / d, h_x, d_x,
// h_y, d_y, W K r_x s_s, dx/dy} with W = w_i w_m, K = dx dy dsig / 8, r_x = 2/dx, s_s = 2/dsig.
// With a_x = h_x - sigma_j d_x and a_y = h_y - sigma_j d_y (d sigma_x, d sigma_y):
// G_rr = w_j c_rr, G_tt = w_j c_rr (dx/dy)^2, G_rs = w_j c_rs a_x, G_ts = w_j c_rs (dx/dy) a_y,
// G_ss = w_j c_ss (a_x^2 + a_y^2 + 1): the products w_i w_m w_j |J| J^-1 J^-T of the mapping
template <int P, typename T>
__device__ __forceinline__ void colgeo_g3d(const double* __restrict__ CG, int c, int Nz, int t,
                                           T (&g)[5][P + 1]) {
  constexpr int NP = P + 1, NL = NP * NP;
  const int ez = t / NL, ab = t - ez * NL;
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2* rc = reinterpret_cast<const d2*>(CG + ((size_t)c * NL + ab) * COLGEO3_N);
  const d2 q0 = rc[0], q1 = rc[1], q2 = rc[2], q3 = rc[3];
  const double inz = 1.0 / Nz, ezn = (double)ez * inz;
  const T crr = (T)q0[0], css = (T)q0[1], crs = (T)q3[0], rat = (T)q3[1];
  const T ctt = crr * rat * rat, cts = crs * rat;
  const T Ax = (T)fma(-ezn, q1[1], q1[0]), Bx = (T)(q1[1] * inz);
  const T Ay = (T)fma(-ezn, q2[1], q2[0]), By = (T)(q2[1] * inz);
  gllc::sfor<NP>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    constexpr T wj = (T)gllc::tab<P>.w[j];
    constexpr T hr = (T)(0.5 * (gllc::tab<P>.x[j] + 1.0));
    const T ax = fma(-hr, Bx, Ax), ay = fma(-hr, By, Ay);
    g[0][j] = wj * crr;
    g[1][j] = wj * ctt;
    g[2][j] = (wj * crs) * ax;
    g[3][j] = (wj * cts) * ay;
    g[4][j] = (wj * css) * fma(ax, ax, fma(ay, ay, (T)1));
  });
}

// this thread's 5 (P+1) factors (f, j) of element column c (3D layout: GLayout with K = 5 (P+1))
template <int P, typename T, typename TG>
__device__ __forceinline__ void load_g3d_stored(const TG* __restrict__ G, int c, int nthr, int t,
                                                T (&g)[5][P + 1]) {
  constexpr int NP = P + 1, K = 5 * NP, W = 16 / (int)sizeof(TG), H = W / 2 > 0 ? W / 2 : 1;
  constexpr int Kp = (K + H - 1) / H * H, NC = Kp / W, REM = Kp - NC * W;
  typedef TG vW __attribute__((ext_vector_type(W)));
  const size_t cstride = ((size_t)nthr * Kp + W - 1) / W * W;
  const TG* Gc = G + (size_t)c * cstride;
  TG raw[Kp];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const vW a = *reinterpret_cast<const vW*>(Gc + ((size_t)q * nthr + t) * W);
#pragma unroll
    for (int w = 0; w < W; ++w) raw[q * W + w] = a[w];
  }
  if constexpr (REM == 1) {
    raw[NC * W] = Gc[(size_t)NC * nthr * W + t];
  } else if constexpr (REM > 1) {
    typedef TG vR __attribute__((ext_vector_type(REM)));
    const vR a = *reinterpret_cast<const vR*>(Gc + (size_t)NC * nthr * W + (size_t)t * REM);
#pragma unroll
    for (int w = 0; w < REM; ++w) raw[NC * W + w] = a[w];
  }
#pragma unroll
  for (int f = 0; f < 5; ++f)
#pragma unroll
    for (int j = 0; j < NP; ++j) g[f][j] = gload<T, TG>(&raw[f * NP + j]);
}

// this thread's factors from the level's factor data: stored layout or column records
template <int P, typename T, typename TG>
__device__ __forceinline__ void load_g3d(const TG* __restrict__ G, int c, int nthr, int t,
                                         T (&g)[5][P + 1]) {
  if constexpr (std::is_same<TG, ColGeo64>::value) {
    colgeo_g3d<P, T>(reinterpret_cast<const double*>(G), c, nthr / ((P + 1) * (P + 1)), t, g);
  } else {
    load_g3d_stored<P, T, TG>(G, c, nthr, t, g);
  }
}

GLayout g3d_layout(int P, int Nz, size_t tgsize) {
  GLayout L;
  L.W = 16 / (int)tgsize;
  const int H = L.W / 2 > 0 ? L.W / 2 : 1, K = 5 * (P + 1);
  L.Kp = (K + H - 1) / H * H;
  L.NC = L.Kp / L.W;
  L.REM = L.Kp - L.NC * L.W;
  const size_t nk = (size_t)(P + 1) * (P + 1) * Nz * L.Kp;
  L.cstride = (nk + L.W - 1) / L.W * L.W;
  return L;
}

// One workgroup per element column (ex, ey) of Nz hexahedra; thread t = (ez NP + a) NP + b has
// three roles in element ez: the vertical line (i, m) = (a, b) (sigma contractions, factors),
// the x-row (m, j) = (a, b) and the y-row (i, j) = (a, b).  u_r and u_t go row -> line through
// LDS, w_r and w_t line -> row, D^T w back row -> line.  Outputs: nodes the column owns (its
// i < P, m < P lines, and the last lines of the domain) into y; its parts of lines shared with
// the next column in x, in y or in both into Sx, Sy, Sxy (full-size arrays indexed like y),
// which k_fix3d adds afterwards.  Deterministic, no atomics.
template <int P, typename T, typename TG>
__global__ __launch_bounds__(1024) void k_apply3d(const T* __restrict__ x, T* __restrict__ y,
                                                  T* __restrict__ Sx, T* __restrict__ Sy,
                                                  T* __restrict__ Sxy, const TG* __restrict__ G,
                                                  int Nx, int Ny, int Nz, int masked,
                                                  Step3 st3) {
  constexpr int NP = P + 1, NL = NP * NP;
  constexpr int V = lds_vec<T>();
  constexpr int NPp = (NP + V - 1) / V * V;
  constexpr int AL = line_align<P, T>();
  const int nzn = Nz * P + 1, nyn = Ny * P + 1;
  const int nzp = (nzn + V - 1) / V * V;
  const int nthr = NL * Nz;
  const int col = blockIdx.x;
  const int ex = col / Ny, ey = col - ex * Ny;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // A1, A2 live through phases 2-5; the space after them holds B1, B2 in phases 3-4 and, in the
  // other phases, the column su (input in 1-2, output in 6) and the element-top values stp (5-6)
  T* A1 = reinterpret_cast<T*>(smem_raw);  // [Nz][i][m][j]: u_r, later D_r^T w_r
  T* A2 = A1 + Nz * NL * NPp;               // [Nz][i][m][j]: u_t, later D_t^T w_t
  T* B1 = A2 + Nz * NL * NPp;               // [Nz][m][j][i]: w_r
  T* B2 = B1 + Nz * NL * NPp;               // [Nz][i][j][m]: w_t
  T* su = B1;                               // [NP(i)][NP(m)][nzp]
  T* stp = su + NL * nzp;                   // [Nz][i][m] element-top values
  const int t = threadIdx.x;
  const bool act = t < nthr;
  const int ez = t / NL, ab = t - (t / NL) * NL;
  const int a = ab / NP, b = ab - (ab / NP) * NP;
  const size_t gx0 = (size_t)ex * P, gy0 = (size_t)ey * P;

  T g[5][NP];
  if (act) load_g3d<P, T, TG>(G, col, nthr, t, g);
  // the column: NP*NP lines of nzn values, one coalesced pass per (line group).  Node k = t + r B
  // of the column is (line, iz) = divmod(k, nzn), stepped from one pass to the next by
  // divmod(B, nzn) (one division per thread instead of one per pass); offsets are 32-bit from
  // the column's first node
  const size_t cbase = ((size_t)gx0 * nyn + gy0) * nzn;
  const unsigned B = blockDim.x, qB = B / nzn, rB = B - qB * nzn;
  const unsigned line0 = t / nzn, iz0 = t - line0 * nzn;
  {
    const T* xc = x + cbase;
    T xin[NP + 1];
    unsigned line = line0, iz = iz0;
#pragma unroll
    for (int r = 0; r <= NP; ++r) {
      if (line < (unsigned)NL) {
        const unsigned i = line / NP, m = line - i * NP;
        xin[r] = xc[(i * nyn + m) * nzn + iz];
      }
      iz += rB;
      line += qB;
      if (iz >= (unsigned)nzn) {
        iz -= nzn;
        ++line;
      }
    }
    line = line0;
    iz = iz0;
#pragma unroll
    for (int r = 0; r <= NP; ++r) {
      if (line < (unsigned)NL) su[line * nzp + iz] = xin[r];
      iz += rB;
      line += qB;
      if (iz >= (unsigned)nzn) {
        iz -= nzn;
        ++line;
      }
    }
  }
  __syncthreads();

  const bool topel = (ez == Nz - 1);
  const bool mtop = masked && topel;
  T v[NP], us[NP];
  T xtop = 0;
  if (act) {
    const int zo = ez * P;
    {  // x-row role (m, j) = (a, b): u_r(i, m, j) = sum_k D_ik u(k, m, j)
      T r[NP], o[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) r[i] = (mtop && b == P) ? (T)0 : su[(i * NP + a) * nzp + zo + b];
      contract_eo<P, false>(r, o);
#pragma unroll
      for (int i = 0; i < NP; ++i) A1[((ez * NP + i) * NP + a) * NPp + b] = o[i];
    }
    {  // y-row role (i, j) = (a, b): u_t(i, m, j) = sum_k D_mk u(i, k, j)
      T r[NP], o[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) r[m] = (mtop && b == P) ? (T)0 : su[(a * NP + m) * nzp + zo + b];
      contract_eo<P, false>(r, o);
#pragma unroll
      for (int m = 0; m < NP; ++m) A2[((ez * NP + a) * NP + m) * NPp + b] = o[m];
    }
    // line role (i, m) = (a, b): u_s
    T u[NP];
    lds_get<NP, AL>(su + ab * nzp + zo, u);
    if (topel) xtop = u[P];
    if (mtop) u[P] = 0;
    contract_eo<P, false>(u, us);
  }
  __syncthreads();
  if (act) {
    T ur[NP], ut[NP], ws[NP];
    lds_get<NP, V>(A1 + (ez * NL + ab) * NPp, ur);
    lds_get<NP, V>(A2 + (ez * NL + ab) * NPp, ut);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      B1[((ez * NP + b) * NP + j) * NPp + a] = g[0][j] * ur[j] + g[2][j] * us[j];
      B2[((ez * NP + a) * NP + j) * NPp + b] = g[1][j] * ut[j] + g[3][j] * us[j];
      ws[j] = g[2][j] * ur[j] + g[3][j] * ut[j] + g[4][j] * us[j];
    }
    contract_eo<P, true>(ws, v);
  }
  __syncthreads();
  if (act) {
    {  // x-row (m, j) = (a, b): (D_r^T w_r)(i, m, j)
      T w[NP], o[NP];
      lds_get<NP, V>(B1 + ((ez * NP + a) * NP + b) * NPp, w);
      contract_eo<P, true>(w, o);
#pragma unroll
      for (int i = 0; i < NP; ++i) A1[((ez * NP + i) * NP + a) * NPp + b] = o[i];
    }
    {  // y-row (i, j) = (a, b): (D_t^T w_t)(i, m, j)
      T w[NP], o[NP];
      lds_get<NP, V>(B2 + ((ez * NP + a) * NP + b) * NPp, w);
      contract_eo<P, true>(w, o);
#pragma unroll
      for (int m = 0; m < NP; ++m) A2[((ez * NP + a) * NP + m) * NPp + b] = o[m];
    }
  }
  __syncthreads();
  if (act) {
    T o1[NP], o2[NP];
    lds_get<NP, V>(A1 + (ez * NL + ab) * NPp, o1);
    lds_get<NP, V>(A2 + (ez * NL + ab) * NPp, o2);
#pragma unroll
    for (int j = 0; j < NP; ++j) v[j] += o1[j] + o2[j];
    stp[ez * NL + ab] = v[P];
  }
  __syncthreads();
  if (act) {
    if (ez > 0) v[0] += stp[(ez - 1) * NL + ab];
    T* ocol = su + ab * nzp + ez * P;
#pragma unroll
    for (int j = 0; j < P; ++j) ocol[j] = v[j];
    if (topel) ocol[P] = masked ? xtop : v[P];
  }
  __syncthreads();
  {
    // outputs, node by node (line, iz) as in the load, offsets from the column's first node
    unsigned line = line0, iz = iz0;
    for (; line < (unsigned)NL;) {
      const unsigned i = line / NP, m = line - i * NP;
      const size_t gg = cbase + (size_t)((i * nyn + m) * nzn + iz);
      const bool dx = i == P && ex < Nx - 1, dy = m == P && ey < Ny - 1;
      T val = su[line * nzp + iz];
      if (!dx && !dy) {
        // smoother step (st3.b set): lines read by this column only are complete here and are
        // updated in place; the lines shared with the left / front column wait for k_fix3d
        if (st3.b && !(i == 0 && ex > 0) && !(m == 0 && ey > 0)) {
          T* xs = const_cast<T*>(x);
          T* d = static_cast<T*>(st3.d);
          const T r = static_cast<const T*>(st3.b)[gg] - val;
          T dn = (T)st3.cr * static_cast<const T*>(st3.dinv)[gg] * r;
          if (st3.cd != 0.0) dn += (T)st3.cd * d[gg];
          if (st3.store_d) d[gg] = dn;
          xs[gg] = xs[gg] + dn;
        } else {
          y[gg] = val;
        }
      } else {
        if (masked && iz == (unsigned)(nzn - 1)) val = (T)0;
        T* dst = dx ? (dy ? Sxy : Sx) : Sy;
        dst[gg] = val;
      }
      iz += rB;
      line += qB;
      if (iz >= (unsigned)nzn) {
        iz -= nzn;
        ++line;
      }
    }
  }
}

// y += the side-buffer parts on lines shared between columns: every node of an interior x-plane
// (Sx, plus Sy and Sxy where it also lies on an interior y-plane), then the nodes of interior
// y-planes that are not on an x-plane (Sy).  Each node is written by one thread.  I is the
// index type: 32-bit whenever the grid fits, which keeps the per-node divisions 32-bit.
template <typename T, typename I>
__global__ void k_fix3d(T* __restrict__ y, const T* __restrict__ Sx, const T* __restrict__ Sy,
                        const T* __restrict__ Sxy, int Nx, int Ny, int P, unsigned nyn,
                        unsigned nzn, Step3 st3, T* __restrict__ x) {
  const I nxn = (I)Nx * P + 1;
  const I nxp = (I)(Nx - 1) * nyn * nzn;
  const I nyp = (I)(Ny - 1) * nxn * nzn;
  // complete node g with its side-buffer part v: y, or (smoother step) the update of x, d
  auto finish = [&](I g, T v) {
    const T ax = y[g] + v;
    if (!st3.b) {
      y[g] = ax;
      return;
    }
    T* d = static_cast<T*>(st3.d);
    const T r = static_cast<const T*>(st3.b)[g] - ax;
    T dn = (T)st3.cr * static_cast<const T*>(st3.dinv)[g] * r;
    if (st3.cd != 0.0) dn += (T)st3.cd * d[g];
    if (st3.store_d) d[g] = dn;
    x[g] = x[g] + dn;
  };
  const I pyz = (I)nyn * nzn, pxz = nxn * (I)nzn;
  for (I k = blockIdx.x * (I)blockDim.x + threadIdx.x; k < nxp + nyp;
       k += (I)gridDim.x * blockDim.x) {
    if (k < nxp) {
      const I q = k / pyz, rem = k - q * pyz;
      const unsigned iy = (unsigned)(rem / nzn), iz = (unsigned)(rem - (I)iy * nzn);
      const I g = (((q + 1) * P) * nyn + iy) * nzn + iz;
      T v = Sx[g];
      const unsigned qy = iy / P;
      if (qy * P == iy && qy > 0 && qy < (unsigned)Ny) v += Sy[g] + Sxy[g];
      finish(g, v);
    } else {
      const I k2 = k - nxp;
      const I q = k2 / pxz, rem = k2 - q * pxz;
      const unsigned ix = (unsigned)(rem / nzn), iz = (unsigned)(rem - (I)ix * nzn);
      const unsigned qx = ix / P;
      if (qx * P == ix && qx > 0 && qx < (unsigned)Nx) continue;  // done by the x-plane pass
      const I g = ((I)ix * nyn + (q + 1) * P) * nzn + iz;
      finish(g, Sy[g]);
    }
  }
}

template <int P, typename T, typename TG>
static hipError_t launch_apply3d(const void* x, void* y, void* Sx, void* Sy, void* Sxy,
                                 const void* G, int Nx, int Ny, int Nz, int masked,
                                 hipStream_t st, Step3 st3) {
  const bool dbl = sizeof(T) == 8;
  const int nthr = (P + 1) * (P + 1) * Nz;
  const int threads = ((nthr + 63) / 64) * 64;
  hipError_t e = allow_lds(k_apply3d<P, T, TG>, apply3d_smem(P, Nz, dbl));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_apply3d<P, T, TG>), dim3(Nx * Ny), dim3(threads), apply3d_smem(P, Nz, dbl),
                     st, (const T*)x, (T*)y, (T*)Sx, (T*)Sy, (T*)Sxy, (const TG*)G, Nx, Ny, Nz,
                     masked, st3);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (Nx > 1 || Ny > 1) {
    const unsigned nyn = Ny * P + 1, nzn = Nz * P + 1;
    const size_t tot = (size_t)(Nx - 1) * nyn * nzn + (size_t)(Ny - 1) * (Nx * P + 1) * nzn;
    const unsigned blocks = (unsigned)std::min<size_t>((tot + 255) / 256, 16384);
    const size_t nodes = ((size_t)Nx * P + 1) * nyn * nzn;
    if (nodes < (1ull << 32) && tot + (size_t)blocks * 256 < (1ull << 32))
      hipLaunchKernelGGL((k_fix3d<T, unsigned>), dim3(blocks), dim3(256), 0, st, (T*)y,
                         (const T*)Sx, (const T*)Sy, (const T*)Sxy, Nx, Ny, P, nyn, nzn, st3,
                         (T*)x);
    else
      hipLaunchKernelGGL((k_fix3d<T, size_t>), dim3(blocks), dim3(256), 0, st, (T*)y,
                         (const T*)Sx, (const T*)Sy, (const T*)Sxy, Nx, Ny, P, nyn, nzn, st3,
                         (T*)x);
  }
  return hipGetLastError();
}

template <int P>
static hipError_t apply3d_p(bool dbl, GType gt, const void* x, void* y, void* Sx, void* Sy,
                            void* Sxy, const void* G, int Nx, int Ny, int Nz, int masked,
                            hipStream_t st, Step3 st3) {
  if (gt == G_COL64)
    return dbl ? launch_apply3d<P, double, ColGeo64>(x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st,
                                                     st3)
               : launch_apply3d<P, float, ColGeo64>(x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st,
                                                    st3);
  if (dbl)
    return launch_apply3d<P, double, double>(x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
  if (gt == G_BF16)
    return launch_apply3d<P, float, uint16_t>(x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
  return launch_apply3d<P, float, float>(x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
}

hipError_t apply3d(int P, bool dbl, GType gt, const void* x, void* y, void* Sx, void* Sy,
                   void* Sxy, const void* G, int Nx, int Ny, int Nz, int masked, hipStream_t st,
                   Step3 st3) {
  {
    const double N3 = (double)(Nx * P + 1) * (Ny * P + 1) * (Nz * P + 1);
    const double L3 = (double)Nx * Ny * Nz * (P + 1) * (P + 1) * (P + 1);
    const double nv = st3.b ? 4 + (st3.cd != 0.0) + (st3.store_d ? 1 : 0) : 2;
    acct_add(vsz(dbl) * N3 * nv +
             (gt == G_COL64 ? 8.0 * COLGEO3_N * Nx * Ny * (P + 1) * (P + 1) : 5 * gsz(gt) * L3));
  }
  switch (P) {
    case 1: return apply3d_p<1>(dbl, gt, x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
    case 2: return apply3d_p<2>(dbl, gt, x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
    case 3: return apply3d_p<3>(dbl, gt, x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
    case 4: return apply3d_p<4>(dbl, gt, x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
    case 5: return apply3d_p<5>(dbl, gt, x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
    case 6: return apply3d_p<6>(dbl, gt, x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
    case 7: return apply3d_p<7>(dbl, gt, x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
    case 8: return apply3d_p<8>(dbl, gt, x, y, Sx, Sy, Sxy, G, Nx, Ny, Nz, masked, st, st3);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------------------------------
// 3D transfers as three 1D passes: out[o][k][i] (+)= sum_e w_e (in[o][col_e][i] - in2[...])
// over the CSR row k of a 1D operator along the middle axis (outer o, inner i)
// ------------------------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ void k_axis(const TI* __restrict__ in, const TI* __restrict__ in2,
                       TO* __restrict__ out, int accumulate, unsigned n_outer, unsigned nin,
                       unsigned nout, unsigned n_inner, const int* __restrict__ rowptr,
                       const int* __restrict__ cols, const double* __restrict__ w,
                       unsigned mask_nzn) {
  const size_t total = (size_t)n_outer * nout * n_inner;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x) {
    const size_t ii = k % n_inner, rest = k / n_inner;
    const unsigned ko = (unsigned)(rest % nout);
    const size_t o = rest / nout;
    double s = 0.0;
    for (int e = rowptr[ko]; e < rowptr[ko + 1]; ++e) {
      const size_t src = (o * nin + cols[e]) * n_inner + ii;
      double v = (double)in[src];
      if (in2) v -= (double)in2[src];
      s += w[e] * v;
    }
    if (mask_nzn && (k % mask_nzn) == mask_nzn - 1) s = 0.0;  // Dirichlet surface rows
    out[k] = accumulate ? (TO)((double)out[k] + s) : (TO)s;
  }
}

// Stride-1 axis (n_inner == 1): B whole lines per block are staged in LDS (as FP64, with in2
// already subtracted) together with the 1D operator, then every output of those lines is a dot
// product out of LDS.  Reads and writes are contiguous spans of B*nin and B*nout values; the
// per-thread gathers with their dependent index loads stay on chip.  Same sums, same order, as
// k_axis.
template <typename TI, typename TO, bool SUB>
__global__ __launch_bounds__(256) void k_axis_lines(const TI* __restrict__ in,
                                                    const TI* __restrict__ in2,
                                                    TO* __restrict__ out, int accumulate,
                                                    unsigned n_outer, unsigned nin, unsigned nout,
                                                    const int* __restrict__ rowptr,
                                                    const int* __restrict__ cols,
                                                    const double* __restrict__ w, unsigned nnz,
                                                    unsigned B, unsigned mask_nzn) {
  extern __shared__ double lds_axis[];
  double* xs = lds_axis;              // B * nin line values
  double* ws = xs + (size_t)B * nin;  // nnz weights
  int* cs = (int*)(ws + nnz);         // nnz columns
  int* rs = cs + nnz;                 // nout + 1 row offsets
  const unsigned o0 = blockIdx.x * B;
  const unsigned nb = min(B, n_outer - o0);
  const unsigned nvin = nb * nin, g0 = o0 * nin;
  for (unsigned i = threadIdx.x; i < nvin; i += 1024u) {
    TI a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const unsigned q = i + 256u * u;
      a[u] = (TI)0;
      b[u] = (TI)0;
      if (q < nvin) {
        a[u] = in[g0 + q];
        if (SUB) b[u] = in2[g0 + q];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const unsigned q = i + 256u * u;
      if (q < nvin) xs[q] = SUB ? (double)a[u] - (double)b[u] : (double)a[u];
    }
  }
  for (unsigned i = threadIdx.x; i < nnz; i += 256u) {
    ws[i] = w[i];
    cs[i] = cols[i];
  }
  for (unsigned i = threadIdx.x; i <= nout; i += 256u) rs[i] = rowptr[i];
  __syncthreads();
  const unsigned nvout = nb * nout, h0 = o0 * nout;
  for (unsigned i = threadIdx.x; i < nvout; i += 256u) {
    const unsigned oo = i / nout, ko = i - oo * nout;
    const double* xl = xs + oo * nin;
    double s = 0.0;
    for (int e = rs[ko]; e < rs[ko + 1]; ++e) s += ws[e] * xl[cs[e]];
    const unsigned k = h0 + i;
    if (mask_nzn && (k % mask_nzn) == mask_nzn - 1) s = 0.0;
    out[k] = accumulate ? (TO)((double)out[k] + s) : (TO)s;
  }
}

// Strided axes: one output per thread as in k_axis, with 32-bit indices and the row as a band:
// one int4 {first column, length, offset into wband, 0} per row and the weights dense over the
// band (zeros where the CSR row has no entry), unrolled to R >= the longest band.  The data
// addresses then depend on one index load instead of two, and every gather of the row is issued
// before the sum (ascending columns).
template <typename TI, typename TO, int R, bool SUB>
__global__ __launch_bounds__(256) void k_axis_band(const TI* __restrict__ in,
                                                   const TI* __restrict__ in2,
                                                   TO* __restrict__ out, int accumulate,
                                                   unsigned total, unsigned nin, unsigned nout,
                                                   unsigned n_inner,
                                                   const int4* __restrict__ band,
                                                   const double* __restrict__ wband,
                                                   unsigned mask_nzn) {
  const unsigned k = blockIdx.x * 256u + threadIdx.x;
  if (k >= total) return;
  const unsigned ii = k % n_inner, rest = k / n_inner;
  const unsigned ko = rest % nout, o = rest / nout;
  const int4 bd = band[ko];
  const unsigned base = (o * nin + (unsigned)bd.x) * n_inner + ii;
  double v[R], ww[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    v[j] = 0.0;
    ww[j] = 0.0;
    if (j < bd.y) {
      const unsigned src = base + (unsigned)j * n_inner;
      ww[j] = wband[bd.z + j];
      v[j] = (double)in[src];
      if (SUB) v[j] -= (double)in2[src];
    }
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (j < bd.y) s += ww[j] * v[j];
  if (mask_nzn && (k % mask_nzn) == mask_nzn - 1) s = 0.0;
  out[k] = accumulate ? (TO)((double)out[k] + s) : (TO)s;
}

template <typename TI, typename TO, int R>
static void axis_band_launch(const void* in, const void* in2, void* out, int accumulate,
                             unsigned total, unsigned nin, unsigned nout, unsigned n_inner,
                             const int* band, const double* wband, unsigned mask_nzn,
                             hipStream_t st) {
  const unsigned blocks = (total + 255u) / 256u;
  if (in2)
    hipLaunchKernelGGL((k_axis_band<TI, TO, R, true>), dim3(blocks), dim3(256), 0, st,
                       (const TI*)in, (const TI*)in2, (TO*)out, accumulate, total, nin, nout,
                       n_inner, (const int4*)band, wband, mask_nzn);
  else
    hipLaunchKernelGGL((k_axis_band<TI, TO, R, false>), dim3(blocks), dim3(256), 0, st,
                       (const TI*)in, (const TI*)in2, (TO*)out, accumulate, total, nin, nout,
                       n_inner, (const int4*)band, wband, mask_nzn);
}

constexpr unsigned AXIS_LINES = 32;           // lines per block of k_axis_lines
constexpr size_t AXIS_LINES_SMEM = 64 * 1024;  // its LDS limit

template <typename TI, typename TO>
static hipError_t axis_t(const void* in, const void* in2, void* out, int accumulate,
                         unsigned n_outer, unsigned nin, unsigned nout, unsigned n_inner,
                         const int* rowptr, const int* cols, const double* w, unsigned nnz,
                         const int* band, const double* wband, int bandmax, unsigned mask_nzn,
                         hipStream_t st) {
  const size_t total = (size_t)n_outer * nout * n_inner;
  if (total == 0) return hipSuccess;
  const bool small = total < (1ull << 32) && (size_t)n_outer * nin * n_inner < (1ull << 32);
  if (small && n_inner == 1) {
    const unsigned B = AXIS_LINES;
    const size_t smem = (size_t)B * nin * 8 + (size_t)nnz * 12 + (size_t)(nout + 1) * 4;
    if (smem <= AXIS_LINES_SMEM) {
      const unsigned blocks = (n_outer + B - 1) / B;
      if (in2)
        hipLaunchKernelGGL((k_axis_lines<TI, TO, true>), dim3(blocks), dim3(256), smem, st,
                           (const TI*)in, (const TI*)in2, (TO*)out, accumulate, n_outer, nin,
                           nout, rowptr, cols, w, nnz, B, mask_nzn);
      else
        hipLaunchKernelGGL((k_axis_lines<TI, TO, false>), dim3(blocks), dim3(256), smem, st,
                           (const TI*)in, (const TI*)in2, (TO*)out, accumulate, n_outer, nin,
                           nout, rowptr, cols, w, nnz, B, mask_nzn);
      return hipGetLastError();
    }
  }
  if (small && band && wband && bandmax >= 0 && bandmax <= 16) {
    const unsigned t = (unsigned)total;
    if (bandmax <= 4)
      axis_band_launch<TI, TO, 4>(in, in2, out, accumulate, t, nin, nout, n_inner, band, wband,
                                  mask_nzn, st);
    else if (bandmax <= 8)
      axis_band_launch<TI, TO, 8>(in, in2, out, accumulate, t, nin, nout, n_inner, band, wband,
                                  mask_nzn, st);
    else
      axis_band_launch<TI, TO, 16>(in, in2, out, accumulate, t, nin, nout, n_inner, band, wband,
                                   mask_nzn, st);
    return hipGetLastError();
  }
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 65535);
  hipLaunchKernelGGL((k_axis<TI, TO>), dim3(blocks), dim3(256), 0, st, (const TI*)in,
                     (const TI*)in2, (TO*)out, accumulate, n_outer, nin, nout, n_inner, rowptr,
                     cols, w, mask_nzn);
  return hipGetLastError();
}

hipError_t axis_apply(int in_dbl, int out_dbl, const void* in, const void* in2, void* out,
                      int accumulate, unsigned n_outer, unsigned nin, unsigned nout,
                      unsigned n_inner, const int* rowptr, const int* cols, const double* w,
                      unsigned nnz, const int* band, const double* wband, int bandmax,
                      unsigned mask_nzn, hipStream_t st) {
  acct_add((in_dbl ? 8.0 : 4.0) * n_outer * nin * n_inner * (in2 ? 2 : 1) +
           (out_dbl ? 8.0 : 4.0) * n_outer * nout * n_inner * (accumulate ? 2 : 1) + 12.0 * nnz);
  if (in_dbl && out_dbl)
    return axis_t<double, double>(in, in2, out, accumulate, n_outer, nin, nout, n_inner, rowptr,
                                  cols, w, nnz, band, wband, bandmax, mask_nzn, st);
  if (in_dbl)
    return axis_t<double, float>(in, in2, out, accumulate, n_outer, nin, nout, n_inner, rowptr,
                                 cols, w, nnz, band, wband, bandmax, mask_nzn, st);
  if (out_dbl)
    return axis_t<float, double>(in, in2, out, accumulate, n_outer, nin, nout, n_inner, rowptr,
                                 cols, w, nnz, band, wband, bandmax, mask_nzn, st);
  return axis_t<float, float>(in, in2, out, accumulate, n_outer, nin, nout, n_inner, rowptr,
                              cols, w, nnz, band, wband, bandmax, mask_nzn, st);
}

// coarsest level: x = Ainv b (dense FP64 inverse of the masked operator), one wave per row
__global__ __launch_bounds__(256) void k_dense_gemv(const double* __restrict__ Ainv,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ x, int n) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;  // wave-uniform; no barrier below
  const double* a = Ainv + (size_t)row * n;
  double s = 0.0;
  for (int k = lane; k < n; k += 64) s += a[k] * b[k];
  s = wave_sum(s);
  if (lane == 0) x[row] = s;
}

hipError_t dense_gemv(const double* Ainv, const double* b, double* x, int n, hipStream_t st) {
  acct_add(8.0 * ((double)n * n + 2.0 * n));
  hipLaunchKernelGGL(k_dense_gemv, dim3((n + 3) / 4), dim3(256), 0, st, Ainv, b, x, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Surface update (sigma mapping moves with eta): fine-level FP64 factors and lumped mass of the
// outer operator from the column samples h, eta at the fine horizontal GLL nodes
// ------------------------------------------------------------------------------------------
// One thread per (column, ez, i, m) vertical line segment of the fine level; writes its 5 (P+1)
// factors in the operator's chunked layout (g3d_layout).  Formulas as the set-up's: d = h + eta,
// h_x, h_y, d_x, d_y by spectral differentiation within the element, sigma_x = (h_x - sigma
// d_x) / d, and G = w_i w_m w_j |J| (metric products).
template <int P>
__global__ void k_geom3d(const double* __restrict__ hf, const double* __restrict__ ef,
                         const double* __restrict__ r, const double* __restrict__ w,
                         double* __restrict__ G, int Nx, int Ny, int Nz, double dx, double dy) {
  constexpr int NP = P + 1, K = 5 * NP, W = 2, Kp = K, NC = Kp / W, REM = Kp - NC * W;
  const int nthr = NP * NP * Nz;
  const size_t cstride = ((size_t)nthr * Kp + W - 1) / W * W;
  const int nyf = Ny * P + 1;
  const double dsig = 1.0 / Nz, rx = 2.0 / dx, ty = 2.0 / dy, ss = 2.0 / dsig;
  const size_t total = (size_t)Nx * Ny * nthr;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(k % nthr);
    const size_t col = k / nthr;
    const int ex = (int)(col / Ny), ey = (int)(col - (size_t)ex * Ny);
    const int ez = t / (NP * NP), i = (t / NP) % NP, m = t % NP;
    auto H = [&](int a, int b) { return hf[(size_t)(ex * P + a) * nyf + ey * P + b]; };
    auto Dd = [&](int a, int b) { return H(a, b) + ef[(size_t)(ex * P + a) * nyf + ey * P + b]; };
    double hx = 0, dxd = 0, hy = 0, dyd = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const double Di = gllc::tab<P>.D[i][q], Dm = gllc::tab<P>.D[m][q];
      hx += Di * H(q, m);
      dxd += Di * Dd(q, m);
      hy += Dm * H(i, q);
      dyd += Dm * Dd(i, q);
    }
    hx *= rx;
    dxd *= rx;
    hy *= ty;
    dyd *= ty;
    const double d = Dd(i, m);
    double* Gc = G + col * cstride;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const double sig = (ez + (r[j] + 1.0) / 2.0) / Nz;
      const double sx = (hx - sig * dxd) / d, sy = (hy - sig * dyd) / d;
      const double wj = w[i] * w[m] * w[j] * (dx / 2.0) * (dy / 2.0) * (d * dsig / 2.0);
      const double v[5] = {wj * rx * rx, wj * ty * ty, wj * rx * ss * sx, wj * ty * ss * sy,
                           wj * ss * ss * (sx * sx + sy * sy + 1.0 / (d * d))};
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const int kk = f * NP + j, q = kk / W, ww = kk - q * W;
        const size_t off = q < NC ? ((size_t)q * nthr + t) * W + ww
                                  : (size_t)NC * nthr * W + (size_t)t * REM + (kk - NC * W);
        Gc[off] = v[f];
      }
    }
  }
}

hipError_t geom3d(int P, const double* hf, const double* ef, const double* r, const double* w,
                  double* G, int Nx, int Ny, int Nz, double dx, double dy, hipStream_t st) {
  const size_t total = (size_t)Nx * Ny * (P + 1) * (P + 1) * Nz;
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 65535);
#define SEM_GEOM(PP) \
  case PP:           \
    hipLaunchKernelGGL(k_geom3d<PP>, dim3(blocks), dim3(256), 0, st, hf, ef, r, w, G, Nx, Ny, Nz, dx, dy); \
    break;
  switch (P) {
    SEM_GEOM(1) SEM_GEOM(2) SEM_GEOM(3) SEM_GEOM(4) SEM_GEOM(5) SEM_GEOM(6) SEM_GEOM(7) SEM_GEOM(8)
    default:
      return hipErrorInvalidValue;
  }
#undef SEM_GEOM
  return hipGetLastError();
}

// the G_COL64 records of the fine level (layout above) from the column samples, one thread per
// column node (c, i, m); slopes by spectral differentiation within the element as in k_geom3d
template <int P>
__global__ void k_colrec3d(const double* __restrict__ hf, const double* __restrict__ ef,
                           double* __restrict__ CG, int Nx, int Ny, int Nz, double dx, double dy) {
  constexpr int NP = P + 1, NL = NP * NP;
  const int nyf = Ny * P + 1;
  const double dsig = 1.0 / Nz, rx = 2.0 / dx, ty = 2.0 / dy, ss = 2.0 / dsig;
  const double K = dx * dy * dsig / 8.0;
  const size_t total = (size_t)Nx * Ny * NL;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x) {
    const size_t col = k / NL;
    const int ab = (int)(k - col * NL), i = ab / NP, m = ab - (ab / NP) * NP;
    const int ex = (int)(col / Ny), ey = (int)(col - (size_t)ex * Ny);
    auto H = [&](int a, int b) { return hf[(size_t)(ex * P + a) * nyf + ey * P + b]; };
    auto Dd = [&](int a, int b) { return H(a, b) + ef[(size_t)(ex * P + a) * nyf + ey * P + b]; };
    double hx = 0, dxd = 0, hy = 0, dyd = 0, wi = 0, wm = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const double Di = gllc::tab<P>.D[i][q], Dm = gllc::tab<P>.D[m][q];
      hx += Di * H(q, m);
      dxd += Di * Dd(q, m);
      hy += Dm * H(i, q);
      dyd += Dm * Dd(i, q);
      if (q == i) wi = gllc::tab<P>.w[q];
      if (q == m) wm = gllc::tab<P>.w[q];
    }
    const double d = Dd(i, m), W = wi * wm;
    double* r = CG + k * COLGEO3_N;
    r[0] = W * K * d * rx * rx;
    r[1] = W * K * ss * ss / d;
    r[2] = rx * hx;
    r[3] = rx * dxd;
    r[4] = ty * hy;
    r[5] = ty * dyd;
    r[6] = W * K * rx * ss;
    r[7] = dx / dy;
  }
}

hipError_t colrec3d(int P, const double* hf, const double* ef, double* CG, int Nx, int Ny, int Nz,
                    double dx, double dy, hipStream_t st) {
  const size_t total = (size_t)Nx * Ny * (P + 1) * (P + 1);
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 65535);
#define SEM_COLREC(PP) \
  case PP:             \
    hipLaunchKernelGGL(k_colrec3d<PP>, dim3(blocks), dim3(256), 0, st, hf, ef, CG, Nx, Ny, Nz, dx, dy); \
    break;
  switch (P) {
    SEM_COLREC(1) SEM_COLREC(2) SEM_COLREC(3) SEM_COLREC(4) SEM_COLREC(5) SEM_COLREC(6)
    SEM_COLREC(7) SEM_COLREC(8)
    default:
      return hipErrorInvalidValue;
  }
#undef SEM_COLREC
  return hipGetLastError();
}

// ---- stage loop pieces ---------------------------------------------------------------------
// d phi / dz at the surface node of every vertical node line s: (2 / dsig) (D_{P j} phi_j over the
// top element's nodes of the line) / d_s, with D the GLL differentiation matrix of the sigma order
template <int P>
__global__ void k_surface_dz(const double* __restrict__ phi, const double* __restrict__ dsurf,
                             double* __restrict__ w, size_t ns, unsigned nzn, double scale) {
  for (size_t s = blockIdx.x * (size_t)blockDim.x + threadIdx.x; s < ns;
       s += (size_t)gridDim.x * blockDim.x) {
    const double* line = phi + s * nzn + (nzn - 1 - P);
    double a = 0.0;
#pragma unroll
    for (int j = 0; j <= P; ++j) a += gllc::tab<P>.D[P][j] * line[j];
    w[s] = scale * a / dsurf[s];
  }
}

hipError_t surface_dz(int P, const double* phi, const double* dsurf, double* w, size_t ns,
                      unsigned nzn, double dsig, hipStream_t st) {
  acct_add(8.0 * ns * (P + 3));
  const unsigned blocks = (unsigned)std::min<size_t>((ns + 255) / 256, 4096);
  const double scale = 2.0 / dsig;
#define SEM_SDZ(PP) \
  case PP:          \
    hipLaunchKernelGGL(k_surface_dz<PP>, dim3(blocks), dim3(256), 0, st, phi, dsurf, w, ns, nzn, scale); \
    break;
  switch (P) {
    SEM_SDZ(1) SEM_SDZ(2) SEM_SDZ(3) SEM_SDZ(4) SEM_SDZ(5) SEM_SDZ(6) SEM_SDZ(7) SEM_SDZ(8)
    SEM_SDZ(9) SEM_SDZ(10) SEM_SDZ(11) SEM_SDZ(12)
    default:
      return hipErrorInvalidValue;
  }
#undef SEM_SDZ
  return hipGetLastError();
}

// low-storage Runge-Kutta stage update: K = a K + dt F, y += b K
__global__ void k_lserk_update(const double* __restrict__ F, double* __restrict__ K,
                               double* __restrict__ y, size_t n, double a, double dt, double b) {
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
       g += (size_t)gridDim.x * blockDim.x) {
    const double k = fma(a, K[g], dt * F[g]);
    K[g] = k;
    y[g] = fma(b, k, y[g]);
  }
}

hipError_t lserk_update(const double* F, double* K, double* y, size_t n, double a, double dt,
                        double b, hipStream_t st) {
  acct_add(8.0 * n * 5);
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_lserk_update, dim3(blocks), dim3(256), 0, st, F, K, y, n, a, dt, b);
  return hipGetLastError();
}

// assembled lumped mass: m_g = (dx dy dsig / 8) d(ix, iy) Wx[ix] Wy[iy] Wz[iz], W the sum of the
// GLL weights of the elements sharing the 1D node (the mass is separable on sigma meshes)
__global__ void k_mass3d(const double* __restrict__ hf, const double* __restrict__ ef,
                         const double* __restrict__ Wx, const double* __restrict__ Wy,
                         const double* __restrict__ Wz, double* __restrict__ mass, unsigned nyn,
                         unsigned nzn, size_t N, double scale) {
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < N;
       g += (size_t)gridDim.x * blockDim.x) {
    const size_t col = g / nzn;
    const unsigned iz = (unsigned)(g - col * nzn);
    const unsigned ix = (unsigned)(col / nyn), iy = (unsigned)(col - (size_t)ix * nyn);
    mass[g] = scale * (hf[col] + ef[col]) * Wx[ix] * Wy[iy] * Wz[iz];
  }
}

hipError_t mass3d(const double* hf, const double* ef, const double* Wx, const double* Wy,
                  const double* Wz, double* mass, unsigned nyn, unsigned nzn, size_t N,
                  double scale, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<size_t>((N + 255) / 256, 65535);
  hipLaunchKernelGGL(k_mass3d, dim3(blocks), dim3(256), 0, st, hf, ef, Wx, Wy, Wz, mass, nyn, nzn,
                     N, scale);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// element-wise kernels
// ------------------------------------------------------------------------------------------
// mode SU_AX: r = b - (y + S); SU_ZERO: x starts at zero, r = b; SU_RESID: r = b is the residual
// of the current x (given by the caller)
template <typename T>
__global__ void k_smooth_update(T* __restrict__ x, T* __restrict__ d, const T* __restrict__ b,
                                const T* __restrict__ dinv, const T* __restrict__ y,
                                const T* __restrict__ S, unsigned N, unsigned nzn, unsigned P,
                                T cd, T cr, int mode, int store_d) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    const T r = mode == SU_AX ? b[g] - ax_at(y, S, g, nzn, P) : b[g];
    T dn = cr * dinv[g] * r;
    if (cd != (T)0) dn += cd * d[g];
    if (store_d) d[g] = dn;
    x[g] = mode == SU_ZERO ? dn : x[g] + dn;
  }
}

hipError_t smooth_update(bool dbl, void* x, void* d, const void* b, const void* dinv,
                         const void* y, const void* S, unsigned N, unsigned nzn, unsigned P,
                         double cd, double cr, int mode, int store_d, hipStream_t st) {
  acct_add(vsz(dbl) * N * ((mode == SU_ZERO ? 3 : mode == SU_AX ? 5 : 4) + (cd != 0.0 && mode != SU_ZERO) + (store_d ? 1 : 0)));
  const unsigned blocks = nblk(N, 256);
  if (dbl)
    hipLaunchKernelGGL(k_smooth_update<double>, dim3(blocks), dim3(256), 0, st, (double*)x,
                       (double*)d, (const double*)b, (const double*)dinv, (const double*)y,
                       (const double*)S, N, nzn, P, cd, cr, mode, store_d);
  else
    hipLaunchKernelGGL(k_smooth_update<float>, dim3(blocks), dim3(256), 0, st, (float*)x,
                       (float*)d, (const float*)b, (const float*)dinv, (const float*)y,
                       (const float*)S, N, nzn, P, (float)cd, (float)cr, mode, store_d);
  return hipGetLastError();
}

// first smoothing step of a V-cycle from x = 0 with the right-hand side given in FP64:
// b = (T) r64;  d = cr dinv b;  x = d
template <typename T>
__global__ void k_smooth_first64(T* __restrict__ x, T* __restrict__ d, T* __restrict__ b,
                                 const double* __restrict__ r64, const T* __restrict__ dinv,
                                 unsigned N, T cr, int store_d) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    const T bv = (T)r64[g];
    b[g] = bv;
    const T dn = cr * dinv[g] * bv;
    if (store_d) d[g] = dn;
    x[g] = dn;
  }
}

hipError_t smooth_first64(bool dbl, void* x, void* d, void* b, const double* r64,
                          const void* dinv, unsigned N, double cr, int store_d, hipStream_t st) {
  acct_add(8.0 * N + vsz(dbl) * N * (3 + (store_d ? 1 : 0)));
  const unsigned blocks = nblk(N, 256);
  if (dbl)
    hipLaunchKernelGGL(k_smooth_first64<double>, dim3(blocks), dim3(256), 0, st, (double*)x,
                       (double*)d, (double*)b, r64, (const double*)dinv, N, cr, store_d);
  else
    hipLaunchKernelGGL(k_smooth_first64<float>, dim3(blocks), dim3(256), 0, st, (float*)x,
                       (float*)d, (float*)b, r64, (const float*)dinv, N, (float)cr, store_d);
  return hipGetLastError();
}

template <typename T, typename TO>
__global__ void k_fix_ax(const T* __restrict__ y, const T* __restrict__ S, TO* __restrict__ out,
                         unsigned N, unsigned nzn, unsigned P) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    out[g] = (TO)ax_at(y, S, g, nzn, P);
}

hipError_t fix_ax(bool dbl, const void* y, const void* S, void* out, int out64, unsigned N,
                  unsigned nzn, unsigned P, hipStream_t st) {
  acct_add((vsz(dbl) + (out64 ? 8.0 : vsz(dbl))) * N);
  const unsigned blocks = nblk(N, 256);
  if (dbl)
    hipLaunchKernelGGL((k_fix_ax<double, double>), dim3(blocks), dim3(256), 0, st,
                       (const double*)y, (const double*)S, (double*)out, N, nzn, P);
  else if (out64)
    hipLaunchKernelGGL((k_fix_ax<float, double>), dim3(blocks), dim3(256), 0, st,
                       (const float*)y, (const float*)S, (double*)out, N, nzn, P);
  else
    hipLaunchKernelGGL((k_fix_ax<float, float>), dim3(blocks), dim3(256), 0, st,
                       (const float*)y, (const float*)S, (float*)out, N, nzn, P);
  return hipGetLastError();
}

template <typename TS, typename TD>
__global__ void k_cast(const TS* __restrict__ s, TD* __restrict__ d, unsigned N) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    d[g] = (TD)s[g];
}

hipError_t cast_to(bool dbl_dst, const double* src, void* dst, unsigned N, hipStream_t st) {
  acct_add((8.0 + vsz(dbl_dst)) * N);
  if (dbl_dst)
    hipLaunchKernelGGL((k_cast<double, double>), dim3(nblk(N, 256)), dim3(256), 0, st, src,
                       (double*)dst, N);
  else
    hipLaunchKernelGGL((k_cast<double, float>), dim3(nblk(N, 256)), dim3(256), 0, st, src,
                       (float*)dst, N);
  return hipGetLastError();
}

hipError_t cast_from(bool dbl_src, const void* src, double* dst, unsigned N, hipStream_t st) {
  acct_add((8.0 + vsz(dbl_src)) * N);
  if (dbl_src)
    hipLaunchKernelGGL((k_cast<double, double>), dim3(nblk(N, 256)), dim3(256), 0, st,
                       (const double*)src, dst, N);
  else
    hipLaunchKernelGGL((k_cast<float, double>), dim3(nblk(N, 256)), dim3(256), 0, st,
                       (const float*)src, dst, N);
  return hipGetLastError();
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, T v, size_t n) {
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
       g += (size_t)gridDim.x * blockDim.x)
    p[g] = v;
}

hipError_t fill(bool dbl, void* p, double v, size_t n, hipStream_t st) {
  acct_add(vsz(dbl) * (double)n);
  const unsigned blocks = (unsigned)(n < (1u << 20) * 256ull ? nblk(n, 256) : (1u << 20));
  if (n == 0) return hipSuccess;
  if (dbl)
    hipLaunchKernelGGL(k_fill<double>, dim3(blocks), dim3(256), 0, st, (double*)p, v, n);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(256), 0, st, (float*)p, (float)v, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// p-transfers (paper Sec. 5.2): prolongation = coarse Lagrange basis at fine GLL nodes
// (I_Pp = Phi V^{-1}) per direction; restriction = its transpose on assembled vectors.
// Both in pull form: every output node sums its own inputs, each shared input counted once.
// ------------------------------------------------------------------------------------------
template <typename T, int PF = 0, int PC = 0>
__device__ __forceinline__ T pull1d(const T* __restrict__ v, int vstride, int c, int Ne, int Pf_rt,
                                    int Pc_rt, const T* __restrict__ J) {
  // coarse node c of a 1D line (Ne elements): sum_f P1[f][c] v[f]; PF, PC > 0 fix the orders
  // at compile time (loops unrolled, every LDS read of a node issued together)
  const int Pf = PF > 0 ? PF : Pf_rt, Pc = PC > 0 ? PC : Pc_rt;
  int ea = c / Pc;
  if (ea > Ne - 1) ea = Ne - 1;
  const int ka = c - ea * Pc;
  T s = 0;
#pragma unroll
  for (int jf = 0; jf <= Pf; ++jf) s += J[jf * (Pc + 1) + ka] * v[(ea * Pf + jf) * vstride];
  if (ka == 0 && ea > 0) {
#pragma unroll
    for (int jf = 0; jf < Pf; ++jf) s += J[jf * (Pc + 1) + Pc] * v[((ea - 1) * Pf + jf) * vstride];
  }
  return s;
}

template <typename T, typename TC, int PF = 0, int PC = 0>
__global__ void k_restrict2d(const T* __restrict__ b, const T* __restrict__ y,
                             const T* __restrict__ S, int use_ax, TC* __restrict__ rc,
                             const double* __restrict__ Jg, int Nx, int Nz, int Pf_rt, int Pc_rt,
                             int masked, StageFold f) {
  const int Pf = PF > 0 ? PF : Pf_rt, Pc = PC > 0 ? PC : Pc_rt;
  const int ex = blockIdx.x;
  // learned-stage fold: the fine residual is b - alpha q (the stage's updated residual); alpha
  // is formed while the first batch of loads is in flight
  T al = 0;
  const T* fq = static_cast<const T*>(f.q);
  __shared__ double sh[8];
  const int nzf = Nz * Pf + 1, nzc = Nz * Pc + 1;
  const int L0 = ex > 0 ? (ex - 1) * Pf : 0;
  const int L1 = ex * Pf + Pf;
  const int nl = L1 - L0 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sJ = reinterpret_cast<T*>(smem_raw);  // (Pf+1)(Pc+1)
  T* rf = sJ + (Pf + 1) * (Pc + 1);        // [nl][nzf]
  T* tv = rf + nl * nzf;                   // [nl][nzc]
  for (int k = threadIdx.x; k < (Pf + 1) * (Pc + 1); k += blockDim.x) sJ[k] = (T)Jg[k];
  // TU values per thread loaded together before any is stored (one memory latency per batch)
  constexpr int TU = 8;
  const int nrf = nl * nzf;
  for (int k0 = 0; k0 < nrf; k0 += TU * (int)blockDim.x) {  // uniform trip count
    T v[TU], w[TU];
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      const int k = k0 + (int)threadIdx.x + u * (int)blockDim.x;
      v[u] = 0;
      w[u] = 0;
      if (k < nrf) {
        const unsigned g = (unsigned)L0 * nzf + k;
        v[u] = b[g];
        if (fq) w[u] = fq[g];
        else if (use_ax) v[u] -= ax_at(y, S, g, (unsigned)nzf, (unsigned)Pf);
      }
    }
    if (fq && k0 == 0) {
      bool ok;
      al = (T)stage_alpha(f.pcr, f.ncr, f.pcq, f.ncq, sh, &ok);
      if (blockIdx.x == 0 && threadIdx.x == 0 && !ok) f.skips[0] += 1;
    }
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      const int k = k0 + (int)threadIdx.x + u * (int)blockDim.x;
      if (k < nrf) rf[k] = (masked && k % nzf == nzf - 1) ? (T)0 : v[u] - al * w[u];
    }
  }
  __syncthreads();
  // along x first, onto the owned coarse lines only (the left neighbour's fine lines feed the
  // shared coarse line alone), then along z; tv holds the x-contracted lines [kc][nzf]
  const int nown = (ex == Nx - 1) ? Pc + 1 : Pc;
  for (int k = threadIdx.x; k < nown * nzf; k += blockDim.x) {
    const int kc = k / nzf, izf = k - kc * nzf;
    const int ic = ex * Pc + kc;
    int ea = ic / Pc;
    if (ea > Nx - 1) ea = Nx - 1;
    const int ka = ic - ea * Pc;
    // rf holds the fine lines from L0 (local index = fine line - L0)
    T s = 0;
#pragma unroll
    for (int i = 0; i <= Pf; ++i) s += sJ[i * (Pc + 1) + ka] * rf[(ea * Pf + i - L0) * nzf + izf];
    if (ka == 0 && ea > 0) {
#pragma unroll
      for (int i = 0; i < Pf; ++i)
        s += sJ[i * (Pc + 1) + Pc] * rf[((ea - 1) * Pf + i - L0) * nzf + izf];
    }
    tv[k] = s;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nown * nzc; k += blockDim.x) {
    const int kc = k / nzc, izc = k - kc * nzc;
    T s = pull1d<T, PF, PC>(tv + kc * nzf, 1, izc, Nz, Pf, Pc, sJ);
    if (masked && izc == nzc - 1) s = 0;
    rc[(size_t)(ex * Pc + kc) * nzc + izc] = (TC)s;
  }
}

size_t restrict2d_smem(int Pf, int Pc, int Nz, bool dbl) {
  const int nl = 2 * Pf + 1;
  const size_t n = (size_t)(Pf + 1) * (Pc + 1) + (size_t)nl * (Nz * Pf + 1) +
                   (size_t)(Pc + 1) * (Nz * Pf + 1);
  return n * (dbl ? 8 : 4);
}

template <typename T, typename TC, int PF, int PC>
static hipError_t restrict2d_t(const void* b, const void* y, const void* S, int use_ax, void* rc,
                               const double* J, int Nx, int Nz, int Pf, int Pc, int masked,
                               size_t smem, hipStream_t st, StageFold f) {
  const hipError_t e = allow_lds(k_restrict2d<T, TC, PF, PC>, smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_restrict2d<T, TC, PF, PC>), dim3(Nx), dim3(256), smem, st, (const T*)b,
                     (const T*)y, (const T*)S, use_ax, (TC*)rc, J, Nx, Nz, Pf, Pc, masked, f);
  return hipGetLastError();
}

// the level pairs of the usual order sequences get unrolled kernels; others the generic one
template <typename T, typename TC>
static hipError_t restrict2d_p(const void* b, const void* y, const void* S, int use_ax, void* rc,
                               const double* J, int Nx, int Nz, int Pf, int Pc, int masked,
                               size_t smem, hipStream_t st, StageFold f) {
#define SEM_R2(a, c)                                                                           \
  if (Pf == a && Pc == c)                                                                      \
    return restrict2d_t<T, TC, a, c>(b, y, S, use_ax, rc, J, Nx, Nz, Pf, Pc, masked, smem, st, f);
  SEM_R2(8, 4) SEM_R2(4, 2) SEM_R2(2, 1) SEM_R2(6, 3) SEM_R2(3, 1)
#undef SEM_R2
  return restrict2d_t<T, TC, 0, 0>(b, y, S, use_ax, rc, J, Nx, Nz, Pf, Pc, masked, smem, st, f);
}

hipError_t restrict2d(bool dbl, bool dbl_c, const void* b, const void* y, const void* S,
                      int use_ax, void* rc, const double* J, int Nx, int Nz, int Pf, int Pc,
                      int masked, hipStream_t st, StageFold f) {
  acct_add(vsz(dbl) * nodes2(Pf, Nx, Nz) * ((use_ax || f.q) ? 2 : 1) + vsz(dbl_c) * nodes2(Pc, Nx, Nz));
  const size_t smem = restrict2d_smem(Pf, Pc, Nz, dbl);
  if (dbl)
    return restrict2d_p<double, double>(b, y, S, use_ax, rc, J, Nx, Nz, Pf, Pc, masked, smem, st, f);
  if (dbl_c)
    return restrict2d_p<float, double>(b, y, S, use_ax, rc, J, Nx, Nz, Pf, Pc, masked, smem, st, f);
  return restrict2d_p<float, float>(b, y, S, use_ax, rc, J, Nx, Nz, Pf, Pc, masked, smem, st, f);
}

template <typename T, typename TC, int PF = 0, int PC = 0>
__global__ void k_prolong2d(const TC* __restrict__ ec, T* __restrict__ xf,
                            const double* __restrict__ Jg, int Nx, int Nz, int Pf_rt, int Pc_rt,
                            StageFold f) {
  const int Pf = PF > 0 ? PF : Pf_rt, Pc = PC > 0 ? PC : Pc_rt;
  const int ex = blockIdx.x;
  // learned-stage fold: the stage's step alpha c is added together with the correction
  T al = 0;
  const T* fc = static_cast<const T*>(f.c);
  __shared__ double sh[8];
  const int nzf = Nz * Pf + 1, nzc = Nz * Pc + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sJ = reinterpret_cast<T*>(smem_raw);  // (Pf+1)(Pc+1)
  T* ce = sJ + (Pf + 1) * (Pc + 1);        // [Pc+1][nzc]
  T* tv = ce + (Pc + 1) * nzc;             // [Pc+1][nzf]
  // the first batch of fine values (TU per thread) is requested before anything else
  const int nown = (ex == Nx - 1) ? Pf + 1 : Pf;
  const size_t fb = (size_t)ex * Pf * nzf;
  constexpr int TU = 5;
  const int nout = nown * nzf;
  T xv[TU], cv[TU];
  auto load_batch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      const int k = k0 + (int)threadIdx.x + u * (int)blockDim.x;
      xv[u] = k < nout ? xf[fb + k] : (T)0;
      cv[u] = (k < nout && fc) ? fc[fb + k] : (T)0;
    }
  };
  load_batch(0);
  for (int k = threadIdx.x; k < (Pf + 1) * (Pc + 1); k += blockDim.x) sJ[k] = (T)Jg[k];
  const size_t cb = (size_t)ex * Pc * nzc;
  for (int k = threadIdx.x; k < (Pc + 1) * nzc; k += blockDim.x) ce[k] = (T)ec[cb + k];
  __syncthreads();
  for (int k = threadIdx.x; k < (Pc + 1) * nzf; k += blockDim.x) {
    const int kc = k / nzf, izf = k - kc * nzf;
    int e = izf / Pf;
    if (e > Nz - 1) e = Nz - 1;
    const int jf = izf - e * Pf;
    T s = 0;
#pragma unroll
    for (int q = 0; q <= Pc; ++q) s += sJ[jf * (Pc + 1) + q] * ce[kc * nzc + e * Pc + q];
    tv[k] = s;
  }
  __syncthreads();
  if (fc) {
    bool ok;
    al = (T)stage_alpha(f.pcr, f.ncr, f.pcq, f.ncq, sh, &ok);
  }
  for (int k0 = 0; k0 < nout; k0 += TU * (int)blockDim.x) {  // uniform trip count
    if (k0 > 0) load_batch(k0);
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      const int k = k0 + (int)threadIdx.x + u * (int)blockDim.x;
      if (k < nout) {
        xv[u] += al * cv[u];
        const int i = k / nzf, izf = k - i * nzf;
        T s = 0;
#pragma unroll
        for (int q = 0; q <= Pc; ++q) s += sJ[i * (Pc + 1) + q] * tv[q * nzf + izf];
        xf[fb + k] = xv[u] + s;
      }
    }
  }
}

size_t prolong2d_smem(int Pf, int Pc, int Nz, bool dbl) {
  const size_t n = (size_t)(Pf + 1) * (Pc + 1) + (size_t)(Pc + 1) * (Nz * Pc + 1) +
                   (size_t)(Pc + 1) * (Nz * Pf + 1);
  return n * (dbl ? 8 : 4);
}

template <typename T, typename TC, int PF, int PC>
static hipError_t prolong2d_t(const void* ec, void* xf, const double* J, int Nx, int Nz, int Pf,
                              int Pc, size_t smem, hipStream_t st, StageFold f) {
  const hipError_t e = allow_lds(k_prolong2d<T, TC, PF, PC>, smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_prolong2d<T, TC, PF, PC>), dim3(Nx), dim3(256), smem, st, (const TC*)ec,
                     (T*)xf, J, Nx, Nz, Pf, Pc, f);
  return hipGetLastError();
}

template <typename T, typename TC>
static hipError_t prolong2d_p(const void* ec, void* xf, const double* J, int Nx, int Nz, int Pf,
                              int Pc, size_t smem, hipStream_t st, StageFold f) {
#define SEM_P2(a, c) \
  if (Pf == a && Pc == c) return prolong2d_t<T, TC, a, c>(ec, xf, J, Nx, Nz, Pf, Pc, smem, st, f);
  SEM_P2(8, 4) SEM_P2(4, 2) SEM_P2(2, 1) SEM_P2(6, 3) SEM_P2(3, 1)
#undef SEM_P2
  return prolong2d_t<T, TC, 0, 0>(ec, xf, J, Nx, Nz, Pf, Pc, smem, st, f);
}

hipError_t prolong2d(bool dbl, bool dbl_c, const void* ec, void* xf, const double* J, int Nx,
                     int Nz, int Pf, int Pc, hipStream_t st, StageFold f) {
  acct_add(vsz(dbl) * nodes2(Pf, Nx, Nz) * (f.c ? 3 : 2) + vsz(dbl_c) * nodes2(Pc, Nx, Nz));
  const size_t smem = prolong2d_smem(Pf, Pc, Nz, dbl);
  if (dbl) return prolong2d_p<double, double>(ec, xf, J, Nx, Nz, Pf, Pc, smem, st, f);
  if (dbl_c) return prolong2d_p<float, double>(ec, xf, J, Nx, Nz, Pf, Pc, smem, st, f);
  return prolong2d_p<float, float>(ec, xf, J, Nx, Nz, Pf, Pc, smem, st, f);
}

// ------------------------------------------------------------------------------------------
// A coarse level's whole smoothing sequence in one kernel (2D)
// ------------------------------------------------------------------------------------------
// PRE: the pre-smoothing from x = 0, the residual and its restriction to the next level (rc);
// POST: the prolongation of the next level's correction (ec) into x and the post-smoothing.
// Workgroup w owns the element columns [w W, (w+1) W) and holds nslot column slots: the owned
// columns and HL columns to their left, the rest to their right.  Values stay exact only where
// every element they depend on is in the window, which moves in by one column per operator
// apply on either side; the margins (the number of applies, PRE one more on the left, whose
// fine lines feed the shared coarse line of the first owned column) keep the owned columns
// exact, and everything outside them is computed but never stored.  A thread keeps its nodes'
// x, d, b and dinv in registers for the whole sequence and the factors of its element too;
// each apply exchanges x through the window array WX and runs the column operator per slot.
// POST reads x and writes xo (another vector: other workgroups still read x).
template <int P, int PC, typename T, typename TG, typename TC, bool PRE>
__global__ __launch_bounds__(1024) void k_coarse2d(const T* __restrict__ x, T* __restrict__ xo,
                                                   const T* __restrict__ b,
                                                   const T* __restrict__ dinv,
                                                   const TG* __restrict__ G,
                                                   const TC* __restrict__ ec, TC* __restrict__ rc,
                                                   const double* __restrict__ Jg, int Nx, int Nz,
                                                   int masked, int W, int HL, int nslot,
                                                   CoarseSeq sq, CoarseIO io) {
  constexpr int NP = P + 1, NPC = PC + 1;
  constexpr int V = lds_vec<T>();
  constexpr int JP = (NP * NPC + V - 1) / V * V;
  const int nzn = Nz * P + 1, nzc = Nz * PC + 1;
  const int nzp = (nzn + V - 1) / V * V;
  const int nthr = NP * Nz;
  const int cs = threadIdx.x / nthr;
  const int t = threadIdx.x - cs * nthr;
  const int c0 = (int)blockIdx.x * W;
  const int ex = c0 - HL + cs;
  const bool valid = cs < nslot && ex >= 0 && ex < Nx;
  const bool nodes = valid && t < nzn;
  const bool owned = valid && cs >= HL && cs < HL + W;
  const int nl = (ex == Nx - 1) ? NP : P;  // lines of this column (the last one also line P)
  const int slot = slot2d_elems<int>(NP, Nz, nzp, V);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sJ = reinterpret_cast<T*>(smem_raw);              // [NP][NPC]
  T* WX = sJ + JP;                                     // window lines [nslot P + 1][nzp]
  T* slots = WX + (size_t)(nslot * P + 1) * nzp;
  T* base = slots + (size_t)(valid ? cs : 0) * slot;   // this column's apply space
  const size_t g0 = (size_t)(valid ? ex : 0) * P * nzn + t;
  const bool from_x = !PRE || (io.flags & CO_FROM_X);
  const bool do_restrict = PRE && (io.flags & CO_RESTRICT);
  const bool do_prolong = !PRE && (io.flags & CO_PROLONG);
  const T* din = static_cast<const T*>(io.din);
  T* dout = static_cast<T*>(io.dout);

  // every global load first: factors, b, dinv (and x, d, the coarse correction when used)
  T g[3][NP], xr[NP], dr[NP], br[NP], di[NP];
  if (valid) load_g2d<P, T, TG>(G, ex, nthr, t, g);
#pragma unroll
  for (int l = 0; l < NP; ++l) {
    xr[l] = 0;
    dr[l] = 0;
    br[l] = 0;
    di[l] = 0;
    if (nodes && l < nl) {
      br[l] = b[g0 + (size_t)l * nzn];
      di[l] = dinv[g0 + (size_t)l * nzn];
      if (from_x) xr[l] = x[g0 + (size_t)l * nzn];
      if (din) dr[l] = din[g0 + (size_t)l * nzn];
    }
  }
  for (int k = threadIdx.x; k < NP * NPC; k += blockDim.x) sJ[k] = (T)Jg[k];
  for (int k = threadIdx.x; k < (nslot * P + 1) * nzp; k += blockDim.x) WX[k] = (T)0;
  T* sce = base;                 // POST: coarse lines of the column [NPC][nzc]
  T* stv = base + NPC * nzc;     // POST: interpolated along z [NPC][nzn]
  if (do_prolong) {
    if (valid) {
      const size_t cb = (size_t)ex * PC * nzc;
      for (int k = t; k < NPC * nzc; k += nthr) sce[k] = (T)ec[cb + k];
    }
  }
  __syncthreads();
  if (do_prolong) {  // x += P ec on the window: along z, then along x (uniform branch)
    if (valid) {
      for (int k = t; k < NPC * nzn; k += nthr) {
        const int kc = k / nzn, izf = k - kc * nzn;
        int e = izf / P;
        if (e > Nz - 1) e = Nz - 1;
        const int jf = izf - e * P;
        T s = 0;
#pragma unroll
        for (int q = 0; q < NPC; ++q) s += sJ[jf * NPC + q] * sce[kc * nzc + e * PC + q];
        stv[k] = s;
      }
    }
    __syncthreads();
    if (nodes) {
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        if (l < nl) {
          T s = 0;
#pragma unroll
          for (int q = 0; q < NPC; ++q) s += sJ[l * NPC + q] * stv[q * nzn + t];
          xr[l] += s;
        }
      }
    }
    __syncthreads();  // the apply space is reused below
  }

  const bool mtop = masked && t == nzn - 1;  // Dirichlet node: its residual is zero
  // one operator apply of the window's x: ax[l] = (A x)(line l of this column, node t)
  auto apply = [&](T (&ax)[NP]) {
    if (nodes) {
#pragma unroll
      for (int l = 0; l < NP; ++l)
        if (l < nl) WX[(size_t)(cs * P + l) * nzp + t] = xr[l];
    }
    __syncthreads();
    T xin[NP];
    column_apply_g<P, T>(
        g,
        [&](T(&v)[NP]) {
#pragma unroll
          for (int l = 0; l < NP; ++l) v[l] = WX[(size_t)(cs * P + l) * nzp + t];
        },
        t, valid, Nz, nzn, nzp, masked, base, xin, [] {});
    if (nodes) {
      const T* su = base + Nz * NP * ((NP + V - 1) / V * V);
      const T* sl = su - slot;
      const bool left = ex > 0 && cs > 0 && !mtop;
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        T a = 0;
        if (l < nl) {
          a = su[l * nzp + t];
          if (l == 0 && left) a += sl[P * nzp + t];
        }
        ax[l] = a;
      }
    }
    __syncthreads();  // the apply space is written again by the next apply
  };

  for (int st = 0; st < sq.ns; ++st) {
    const T cd = (T)sq.cd[st], cr = (T)sq.cr[st];
    T ax[NP];
#pragma unroll
    for (int l = 0; l < NP; ++l) ax[l] = 0;
    if (!(st == 0 && !from_x)) apply(ax);  // from x = 0: A x = 0
    if (nodes) {
#pragma unroll
      for (int l = 0; l < NP; ++l) {
        if (l < nl) {
          const T r = mtop ? (T)0 : br[l] - ax[l];
          const T dn = cr * di[l] * r + cd * dr[l];
          dr[l] = dn;
          xr[l] += dn;
        }
      }
    }
  }

  if (do_restrict) {
    // residual of the smoothed x, into WX (lines of each column), then its restriction onto
    // the owned coarse lines: along x first, then along z
    T ax[NP];
    apply(ax);
    if (nodes) {
#pragma unroll
      for (int l = 0; l < NP; ++l)
        if (l < nl) WX[(size_t)(cs * P + l) * nzp + t] = mtop ? (T)0 : br[l] - ax[l];
    }
    __syncthreads();
    const int nown = (ex == Nx - 1) ? NPC : PC;
    T* sxs = base;  // [NPC][nzn]
    if (owned) {
      for (int k = t; k < nown * nzn; k += nthr) {
        const int kc = k / nzn, izf = k - kc * nzn;
        const int ka = (kc == PC) ? PC : kc;  // kc == PC only for the last column
        T s = 0;
#pragma unroll
        for (int i = 0; i < NP; ++i) s += sJ[i * NPC + ka] * WX[(size_t)(cs * P + i) * nzp + izf];
        if (ka == 0 && ex > 0) {
#pragma unroll
          for (int i = 0; i < P; ++i)
            s += sJ[i * NPC + PC] * WX[(size_t)((cs - 1) * P + i) * nzp + izf];
        }
        sxs[k] = s;
      }
    }
    __syncthreads();
    if (owned) {
      for (int k = t; k < nown * nzc; k += nthr) {
        const int kc = k / nzc, izc = k - kc * nzc;
        T s = pull1d<T, P, PC>(sxs + kc * nzn, 1, izc, Nz, P, PC, sJ);
        if (masked && izc == nzc - 1) s = 0;
        rc[(size_t)(ex * PC + kc) * nzc + izc] = (TC)s;
      }
    }
  }
  if (owned && t < nzn) {
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      if (l < nl) {
        xo[g0 + (size_t)l * nzn] = xr[l];
        if (dout) dout[g0 + (size_t)l * nzn] = dr[l];
      }
    }
  }
}

// window shape of a coarse-level kernel: columns per workgroup and margins, 0 when it does not
// fit one workgroup (1024 threads) or its LDS
CoarsePlan coarse2d_plan(int P, int PC, int Nz, bool dbl, int flags, int applies) {
  CoarsePlan pl;
  const int nthr = (P + 1) * Nz;
  const int V = dbl ? 2 : 4;
  const int nzn = Nz * P + 1, nzc = Nz * PC + 1;
  const int nzp = (nzn + V - 1) / V * V;
  const bool rs = (flags & CO_RESTRICT) != 0, pr = (flags & CO_PROLONG) != 0;
  const int HL = applies + (rs ? 1 : 0), HR = applies;
  const int maxs = 1024 / nthr;
  const int W = maxs - HL - HR;
  if (W < 1) return pl;
  const size_t slot = slot2d_elems<size_t>(P + 1, Nz, nzp, V);
  const size_t scratch = std::max(rs ? (size_t)(PC + 1) * nzn : 0,
                                  pr ? (size_t)(PC + 1) * (nzc + nzn) : 0);
  if (scratch > slot) return pl;
  const int nslot = W + HL + HR;
  const size_t JP = ((size_t)(P + 1) * (PC + 1) + V - 1) / V * V;
  const size_t elems = JP + (size_t)(nslot * P + 1) * nzp + (size_t)nslot * slot;
  const size_t bytes = elems * (dbl ? 8 : 4);
  if (bytes > 160 * 1024) return pl;
  pl.W = W;
  pl.HL = HL;
  pl.nslot = nslot;
  pl.smem = bytes;
  return pl;
}

template <int P, int PC, typename T, typename TG, typename TC, bool PRE>
static hipError_t coarse2d_t(const CoarsePlan& pl, const void* x, void* xo, const void* b,
                             const void* dinv, const void* G, const void* ec, void* rc,
                             const double* J, int Nx, int Nz, int masked, const CoarseSeq& sq,
                             hipStream_t st, CoarseIO io) {
  const hipError_t e = allow_lds(k_coarse2d<P, PC, T, TG, TC, PRE>, pl.smem);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)((Nx + pl.W - 1) / pl.W);
  const int nthr = (P + 1) * Nz;
  hipLaunchKernelGGL((k_coarse2d<P, PC, T, TG, TC, PRE>), dim3(blocks), dim3(pl.nslot * nthr),
                     pl.smem, st, (const T*)x, (T*)xo, (const T*)b, (const T*)dinv,
                     (const TG*)G, (const TC*)ec, (TC*)rc, J, Nx, Nz, masked, pl.W, pl.HL,
                     pl.nslot, sq, io);
  return hipGetLastError();
}

template <int P, int PC, bool PRE>
static hipError_t coarse2d_ty(const CoarsePlan& pl, bool dbl, GType gt, bool dbl_c, const void* x,
                              void* xo, const void* b, const void* dinv, const void* G,
                              const void* ec, void* rc, const double* J, int Nx, int Nz,
                              int masked, const CoarseSeq& sq, hipStream_t st, CoarseIO io) {
  if (gt == G_COL64) {
    if (dbl)
      return coarse2d_t<P, PC, double, ColGeo64, double, PRE>(pl, x, xo, b, dinv, G, ec, rc, J,
                                                              Nx, Nz, masked, sq, st, io);
    if (dbl_c)
      return coarse2d_t<P, PC, float, ColGeo64, double, PRE>(pl, x, xo, b, dinv, G, ec, rc, J,
                                                             Nx, Nz, masked, sq, st, io);
    return coarse2d_t<P, PC, float, ColGeo64, float, PRE>(pl, x, xo, b, dinv, G, ec, rc, J, Nx,
                                                          Nz, masked, sq, st, io);
  }
  if (dbl)
    return coarse2d_t<P, PC, double, double, double, PRE>(pl, x, xo, b, dinv, G, ec, rc, J, Nx,
                                                          Nz, masked, sq, st, io);
  if (gt == G_BF16) {
    if (dbl_c)
      return coarse2d_t<P, PC, float, uint16_t, double, PRE>(pl, x, xo, b, dinv, G, ec, rc, J,
                                                             Nx, Nz, masked, sq, st, io);
    return coarse2d_t<P, PC, float, uint16_t, float, PRE>(pl, x, xo, b, dinv, G, ec, rc, J, Nx,
                                                          Nz, masked, sq, st, io);
  }
  if (dbl_c)
    return coarse2d_t<P, PC, float, float, double, PRE>(pl, x, xo, b, dinv, G, ec, rc, J, Nx, Nz,
                                                        masked, sq, st, io);
  return coarse2d_t<P, PC, float, float, float, PRE>(pl, x, xo, b, dinv, G, ec, rc, J, Nx, Nz,
                                                     masked, sq, st, io);
}

bool coarse2d_supported(int P, int PC) {
  return (P == 4 && (PC == 2 || PC == 1)) || (P == 3 && (PC == 2 || PC == 1)) ||
         (P == 2 && PC == 1);
}

hipError_t coarse2d(bool pre, const CoarsePlan& pl, int P, int PC, bool dbl, GType gt, bool dbl_c,
                    const void* x, void* xo, const void* b, const void* dinv, const void* G,
                    const void* ec, void* rc, const double* J, int Nx, int Nz, int masked,
                    const CoarseSeq& sq, hipStream_t st, CoarseIO io) {
  {
    const bool from_x = !pre || (io.flags & CO_FROM_X);
    const bool coarse = pre ? (io.flags & CO_RESTRICT) : (io.flags & CO_PROLONG);
    const double nv = 3 + (from_x ? 1 : 0) + (io.din ? 1 : 0) + (io.dout ? 1 : 0);
    acct_add(vsz(dbl) * nodes2(P, Nx, Nz) * nv + (coarse ? vsz(dbl_c) * nodes2(PC, Nx, Nz) : 0) +
             gbytes2(gt, P, Nx, Nz));
  }
  if (pl.W < 1 || sq.ns < 1 || sq.ns > CO_MAXS) return hipErrorInvalidValue;
#define SEM_CO(a, c)                                                                            \
  if (P == a && PC == c)                                                                        \
    return pre ? coarse2d_ty<a, c, true>(pl, dbl, gt, dbl_c, x, xo, b, dinv, G, ec, rc, J, Nx,  \
                                         Nz, masked, sq, st, io)                                \
               : coarse2d_ty<a, c, false>(pl, dbl, gt, dbl_c, x, xo, b, dinv, G, ec, rc, J, Nx, \
                                          Nz, masked, sq, st, io);
  SEM_CO(4, 2) SEM_CO(4, 1) SEM_CO(3, 2) SEM_CO(3, 1) SEM_CO(2, 1)
#undef SEM_CO
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------------
// exact coarse solve by block cyclic reduction (FP64)
// ------------------------------------------------------------------------------------------
// Level-vector position of unknown r of a block: the free rows of a block skip the top
// (Dirichlet) node of every vertical line, so r -> r + r / (nzn - 1).
__device__ __forceinline__ size_t bpos(size_t blk, int bstride, int r, int nzf) {
  return blk * bstride + r + r / nzf;
}

// 4 lanes per (block, row): lane q sums columns q, q+4, ...; fixed-order 4-lane reduction
__global__ __launch_bounds__(256) void k_bcr_fwd(double* __restrict__ b,
                                                 const double* __restrict__ F, int n, int stride,
                                                 int total, int bstride, int nzf, int nb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int idx = t >> 2, q = t & 3;
  const bool act = idx < total;
  double s = 0.0;
  size_t self = 0;
  if (act) {
    const int kk = idx / nb, row = idx - kk * nb;
    const int k = 2 * kk;
    const size_t i = (size_t)k * stride;
    const size_t nn = (size_t)nb * nb;
    const double* Mm = F + (size_t)kk * 2 * nn + row;
    const double* Mp = Mm + nn;
    self = bpos(i, bstride, row, nzf);
    if (k > 0)
      for (int c = q; c < nb; c += 4) s += Mm[(size_t)c * nb] * b[bpos(i - stride, bstride, c, nzf)];
    if (k + 1 < n)
      for (int c = q; c < nb; c += 4) s += Mp[(size_t)c * nb] * b[bpos(i + stride, bstride, c, nzf)];
  }
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  if (act && q == 0) b[self] -= s;
}

__global__ __launch_bounds__(256) void k_bcr_bwd(const double* __restrict__ b,
                                                 double* __restrict__ x,
                                                 const double* __restrict__ Bk, int n, int stride,
                                                 int total, int bstride, int nzf, int nb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int idx = t >> 2, q = t & 3;
  const bool act = idx < total;
  double s = 0.0;
  size_t self = 0;
  if (act) {
    const int kk = idx / nb, row = idx - kk * nb;
    const int k = 2 * kk + 1;
    const size_t i = (size_t)k * stride;
    const size_t nn = (size_t)nb * nb;
    const double* DO = Bk + (size_t)kk * 3 * nn + row;
    const double* DL = DO + nn;
    const double* DU = DL + nn;
    self = bpos(i, bstride, row, nzf);
    for (int c = q; c < nb; c += 4)
      s += DO[(size_t)c * nb] * b[bpos(i, bstride, c, nzf)] -
           DL[(size_t)c * nb] * x[bpos(i - stride, bstride, c, nzf)];
    if (k + 1 < n)
      for (int c = q; c < nb; c += 4) s -= DU[(size_t)c * nb] * x[bpos(i + stride, bstride, c, nzf)];
  }
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  if (act && q == 0) x[self] = s;
}

// x at the reduced positions = Ainv b: the block gathers b into LDS, then one wave per row
// (lanes stride the row, 8 loads in flight each; fixed-order wave reduction)
__global__ __launch_bounds__(256) void k_bcr_dense(const double* __restrict__ Ainv,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ x, int nd, int nb,
                                                   int stride, int bstride, int nzf) {
  extern __shared__ double sbv[];  // [nd]
  constexpr int UG = 4, UR = 8;
  for (int c0 = 0; c0 < nd; c0 += UG * (int)blockDim.x) {
    double v[UG];
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      const int c = c0 + (int)threadIdx.x + u * (int)blockDim.x;
      if (c < nd) {
        const int k = c / nb, r = c - k * nb;
        v[u] = b[bpos((size_t)k * stride, bstride, r, nzf)];
      } else {
        v[u] = 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      const int c = c0 + (int)threadIdx.x + u * (int)blockDim.x;
      if (c < nd) sbv[c] = v[u];
    }
  }
  __syncthreads();
  const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nd) return;
  const double* a = Ainv + (size_t)row * nd;
  double s = 0.0;
  for (int c0 = 0; c0 < nd; c0 += UR * 64) {
    double av[UR];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int c = c0 + lane + u * 64;
      av[u] = c < nd ? a[c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int c = c0 + lane + u * 64;
      if (c < nd) s += av[u] * sbv[c];
    }
  }
  s = wave_sum(s);
  if (lane == 0) {
    const int k = row / nb, r = row - k * nb;
    x[bpos((size_t)k * stride, bstride, r, nzf)] = s;
  }
}

hipError_t bcr_dense(const double* Ainv, const double* b, double* x, int nd, int nb, int stride,
                     int bstride, int nzf, hipStream_t st) {
  const size_t smem = (size_t)nd * sizeof(double);
  const hipError_t e = allow_lds(k_bcr_dense, smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bcr_dense, dim3(nblk(nd, 4)), dim3(256), smem, st, Ainv, b, x, nd, nb,
                     stride, bstride, nzf);
  return hipGetLastError();
}

// Every level of the forward reduction in one launch.  Workgroup w owns the level-0 blocks
// [w C, (w+1) C) and keeps in LDS a window that extends S - 1 = 2^nl - 1 blocks to either side:
// a block's value after nl levels depends on the original right-hand side within that distance
// only, so each workgroup recomputes the reductions of its margin instead of waiting for its
// neighbours (values the window cannot complete are computed too but never leave it).  The
// reduced right-hand side goes to bred, so no workgroup reads a value another one has updated.
// Tasks (block, row) of all levels are numbered level after level and task k goes to thread
// k mod blockDim: every thread requests the factor row of its first task at the start, so the
// levels wait for one memory latency in all (tasks beyond blockDim load theirs when they run).
// The rows of one task read consecutive entries of the column-major factor columns.  NB > 0
// fixes the block size at compile time (NB = 0: any size).
template <int NB>
__global__ __launch_bounds__(512) void k_bcr_fwd_all(const double* __restrict__ b,
                                                     double* __restrict__ bred,
                                                     const double* __restrict__ F, BcrLevels lv,
                                                     int nblocks, int C, int bstride, int nzf,
                                                     int nb_rt) {
  extern __shared__ double sb[];  // [window][nb]
  const int nb = NB > 0 ? NB : nb_rt;
  constexpr int NBR = NB > 0 ? NB : 1;
  const int S = 1 << lv.nl;
  const int ws = (int)blockIdx.x * C - (S - 1);
  const int Wn = C + 2 * (S - 1);
  const int we = ws + Wn;  // exclusive
  const int gl = (we - 1 < nblocks - 1 ? we - 1 : nblocks - 1);
  const size_t nn = (size_t)nb * nb;
  // blocks reduced at level l: multiples of 2s in the window (their neighbours checked below)
  auto level_range = [&](int l, int* g0, int* ncand) {
    const int s = 1 << l, s2 = 2 * s;
    int g = ws + s > 0 ? ws + s : 0;
    g = (g + s2 - 1) / s2 * s2;
    *g0 = g;
    *ncand = gl >= g ? (gl - g) / s2 + 1 : 0;
  };
  // task number k (over all levels, level 0 first) -> level, block, row; false past the end
  auto task_of = [&](int k, int* tl, int* tg, int* trow) {
    int tb = 0;
    for (int l = 0; l < lv.nl; ++l) {
      int g0, nc;
      level_range(l, &g0, &nc);
      const int j = k - tb;
      if (j >= 0 && j < nc * nb) {
        *tl = l;
        *tg = g0 + (j / nb) * (2 << l);
        *trow = j - (j / nb) * nb;
        return true;
      }
      tb += nc * nb;
    }
    return false;
  };
  // one task: sb[g][row] -= Mm row . sb[g - s] + Mp row . sb[g + s]; fm, fp: its factor rows
  auto task_rows = [&](int l, int g, int row, double* fm, double* fp) {
    const int s = 1 << l;
    const double* Mm = F + lv.offM[l] + (size_t)(g >> (l + 1)) * 2 * nn + row;
    const double* Mp = Mm + nn;
    const bool left = g > 0, right = g + s < nblocks;
    for (int c = 0; c < nb; ++c) {
      fm[c] = left ? Mm[(size_t)c * nb] : 0.0;
      fp[c] = right ? Mp[(size_t)c * nb] : 0.0;
    }
  };
  auto task_apply = [&](int l, int g, int row, const double* fm, const double* fp) {
    const int s = 1 << l;
    const bool left = g > 0, right = g + s < nblocks;
    if (right && g + s >= we) return;  // right neighbour outside the window: not needed
    const double* vl = sb + (size_t)(g - s - ws) * nb;
    const double* vr = sb + (size_t)(g + s - ws) * nb;
    double acc = 0.0;
    for (int c = 0; c < nb; ++c) {
      if (left) acc += fm[c] * vl[c];
      if (right) acc += fp[c] * vr[c];
    }
    sb[(size_t)(g - ws) * nb + row] -= acc;
  };
  // this thread's first two tasks (k = tid, tid + blockDim): their factor rows are requested
  // before anything else
  double fmA[NBR], fpA[NBR], fmB[NBR], fpB[NBR];
  if constexpr (NB > 0) {
    int l, g, row;
    if (task_of((int)threadIdx.x, &l, &g, &row)) task_rows(l, g, row, fmA, fpA);
    if (task_of((int)(threadIdx.x + blockDim.x), &l, &g, &row)) task_rows(l, g, row, fmB, fpB);
  }
  for (int t = threadIdx.x; t < Wn * nb; t += blockDim.x) {
    const int p = t / nb, r = t - p * nb;
    const int g = ws + p;
    sb[t] = (g >= 0 && g < nblocks) ? b[bpos(g, bstride, r, nzf)] : 0.0;
  }
  __syncthreads();
  int tb = 0;
  for (int l = 0; l < lv.nl; ++l) {
    int g0, nc;
    level_range(l, &g0, &nc);
    const int s2 = 2 << l;
    for (int k = (int)threadIdx.x - tb; k < nc * nb; k += blockDim.x) {
      if (k < 0) continue;
      const int g = g0 + (k / nb) * s2, row = k - (k / nb) * nb;
      if constexpr (NB > 0) {
        const int kk = k + tb;  // task number
        if (kk == (int)threadIdx.x) {
          task_apply(l, g, row, fmA, fpA);
        } else {
          // the second task was prefetched; later ones (after it) reuse its registers
          if (kk != (int)(threadIdx.x + blockDim.x)) task_rows(l, g, row, fmB, fpB);
          task_apply(l, g, row, fmB, fpB);
        }
      } else {
        double fm[64], fp[64];  // nb <= 64 on this path (host check)
        task_rows(l, g, row, fm, fp);
        task_apply(l, g, row, fm, fp);
      }
    }
    tb += nc * nb;
    __syncthreads();
  }
  const int o0 = (int)blockIdx.x * C;
  for (int t = threadIdx.x; t < C * nb; t += blockDim.x) {
    const int p = t / nb, r = t - p * nb;
    const int g = o0 + p;
    if (g < nblocks) bred[bpos(g, bstride, r, nzf)] = sb[(size_t)(g - ws) * nb + r];
  }
}

// Every level of the back substitution in one launch.  Workgroup w owns the blocks
// [w C, (w+1) C) with C a multiple of S = 2^nl: the blocks that are multiples of S (solved by
// the dense step) bound the chunk, and every other block of it follows from them and from the
// chunk's reduced right-hand side alone.  As in the forward kernel, the tasks of all levels are
// numbered level after level (coarsest first) and every thread prefetches its first task's rows.
template <int NB>
__global__ __launch_bounds__(256) void k_bcr_bwd_all(const double* __restrict__ bred,
                                                     double* __restrict__ x,
                                                     const double* __restrict__ Bk, BcrLevels lv,
                                                     int nblocks, int C, int bstride, int nzf,
                                                     int nb_rt) {
  extern __shared__ double sm[];
  const int nb = NB > 0 ? NB : nb_rt;
  constexpr int NBR = NB > 0 ? NB : 1;
  double* sx = sm;                         // [C + 1][nb]
  double* sv = sm + (size_t)(C + 1) * nb;  // [C][nb]
  const int S = 1 << lv.nl;
  const int g0 = (int)blockIdx.x * C;
  const size_t nn = (size_t)nb * nb;
  auto task_rows = [&](int l, int g, int row, double* fo, double* fl, double* fu) {
    const int s = 1 << l;
    const double* DO = Bk + lv.offB[l] + (size_t)(g >> (l + 1)) * 3 * nn + row;
    const double* DL = DO + nn;
    const double* DU = DL + nn;
    const bool ok = g < nblocks, right = g + s < nblocks;
    for (int c = 0; c < nb; ++c) {
      fo[c] = ok ? DO[(size_t)c * nb] : 0.0;
      fl[c] = ok ? DL[(size_t)c * nb] : 0.0;
      fu[c] = (ok && right) ? DU[(size_t)c * nb] : 0.0;
    }
  };
  auto task_apply = [&](int l, int g, int row, const double* fo, const double* fl,
                        const double* fu) {
    const int s = 1 << l;
    if (g >= nblocks) return;
    const bool right = g + s < nblocks;
    const double* vb = sv + (size_t)(g - g0) * nb;
    const double* xl = sx + (size_t)(g - s - g0) * nb;
    const double* xr = sx + (size_t)(g + s - g0) * nb;
    double acc = 0.0;
    for (int c = 0; c < nb; ++c) {
      acc += fo[c] * vb[c] - fl[c] * xl[c];
      if (right) acc -= fu[c] * xr[c];
    }
    sx[(size_t)(g - g0) * nb + row] = acc;
  };
  // this thread's first task (levels nl - 1 down to 0; level l has C / 2^(l+1) blocks)
  int my_l = -1, my_g = 0, my_row = 0;
  {
    int tb = 0;
    for (int l = lv.nl - 1; l >= 0; --l) {
      const int nc = C >> (l + 1);
      const int k = (int)threadIdx.x - tb;
      if (my_l < 0 && k >= 0 && k < nc * nb) {
        my_l = l;
        my_g = g0 + (1 << l) + (k / nb) * (2 << l);
        my_row = k - (k / nb) * nb;
      }
      tb += nc * nb;
    }
  }
  double fo0[NBR], fl0[NBR], fu0[NBR];
  if constexpr (NB > 0) {
    if (my_l >= 0) {
      const int s = 1 << my_l;
      const double* DO = Bk + lv.offB[my_l] + (size_t)(my_g >> (my_l + 1)) * 3 * nn + my_row;
      const bool ok = my_g < nblocks, right = my_g + s < nblocks;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        fo0[c] = ok ? DO[c * NB] : 0.0;
        fl0[c] = ok ? DO[nn + c * NB] : 0.0;
        fu0[c] = (ok && right) ? DO[2 * nn + c * NB] : 0.0;
      }
    }
  }
  for (int t = threadIdx.x; t < C * nb; t += blockDim.x) {
    const int p = t / nb, r = t - p * nb;
    const int g = g0 + p;
    sv[t] = g < nblocks ? bred[bpos(g, bstride, r, nzf)] : 0.0;
  }
  const int nd = C / S + 1;
  for (int t = threadIdx.x; t < nd * nb; t += blockDim.x) {
    const int m = t / nb, r = t - m * nb;
    const int g = g0 + m * S;
    sx[(size_t)m * S * nb + r] = g < nblocks ? x[bpos(g, bstride, r, nzf)] : 0.0;
  }
  __syncthreads();
  int tb = 0;
  for (int l = lv.nl - 1; l >= 0; --l) {
    const int nc = C >> (l + 1);
    const int s = 1 << l, s2 = 2 * s;
    for (int k = (int)threadIdx.x - tb; k < nc * nb; k += blockDim.x) {
      if (k < 0) continue;
      const int g = g0 + s + (k / nb) * s2, row = k - (k / nb) * nb;
      if constexpr (NB > 0) {
        if (k + tb != (int)threadIdx.x) task_rows(l, g, row, fo0, fl0, fu0);
        task_apply(l, g, row, fo0, fl0, fu0);
      } else {
        double fo[64], fl[64], fu[64];
        task_rows(l, g, row, fo, fl, fu);
        task_apply(l, g, row, fo, fl, fu);
      }
    }
    tb += nc * nb;
    __syncthreads();
  }
  for (int t = threadIdx.x; t < C * nb; t += blockDim.x) {
    const int p = t / nb, r = t - p * nb;
    const int g = g0 + p;
    if (g < nblocks && (p & (S - 1)) != 0) x[bpos(g, bstride, r, nzf)] = sx[t];
  }
}


static int bcr_chunk(int nl) { return (1 << nl) > 16 ? (1 << nl) : 16; }
size_t bcr_fwd_all_smem(int nl, int nb) {
  return (size_t)(bcr_chunk(nl) + 2 * ((1 << nl) - 1)) * nb * sizeof(double);
}
size_t bcr_bwd_all_smem(int nl, int nb) {
  return (size_t)(2 * bcr_chunk(nl) + 1) * nb * sizeof(double);
}

template <int NB>
static hipError_t bcr_all_launch(bool fwd, const double* in, double* out, const double* M,
                                 const BcrLevels& lv, int nblocks, int bstride, int nzf, int nb,
                                 hipStream_t st) {
  const int C = bcr_chunk(lv.nl);
  if (fwd) {
    const size_t smem = bcr_fwd_all_smem(lv.nl, nb);
    const hipError_t e = allow_lds(k_bcr_fwd_all<NB>, smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_bcr_fwd_all<NB>), dim3(nblk(nblocks, C)), dim3(512), smem, st, in, out,
                       M, lv, nblocks, C, bstride, nzf, nb);
  } else {
    const size_t smem = bcr_bwd_all_smem(lv.nl, nb);
    const hipError_t e = allow_lds(k_bcr_bwd_all<NB>, smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_bcr_bwd_all<NB>), dim3(nblk(nblocks, C)), dim3(256), smem, st, in, out,
                       M, lv, nblocks, C, bstride, nzf, nb);
  }
  return hipGetLastError();
}

static hipError_t bcr_all(bool fwd, const double* in, double* out, const double* M,
                          const BcrLevels& lv, int nblocks, int bstride, int nzf, int nb,
                          hipStream_t st) {
  switch (nb) {
    case 4: return bcr_all_launch<4>(fwd, in, out, M, lv, nblocks, bstride, nzf, nb, st);
    case 8: return bcr_all_launch<8>(fwd, in, out, M, lv, nblocks, bstride, nzf, nb, st);
    case 16: return bcr_all_launch<16>(fwd, in, out, M, lv, nblocks, bstride, nzf, nb, st);
    default:
      if (nb > 64) return hipErrorInvalidValue;
      return bcr_all_launch<0>(fwd, in, out, M, lv, nblocks, bstride, nzf, nb, st);
  }
}

hipError_t bcr_fwd_all(const double* b, double* bred, const double* F, const BcrLevels& lv,
                       int nblocks, int bstride, int nzf, int nb, hipStream_t st) {
  return bcr_all(true, b, bred, F, lv, nblocks, bstride, nzf, nb, st);
}

hipError_t bcr_bwd_all(const double* bred, double* x, const double* Bk, const BcrLevels& lv,
                       int nblocks, int bstride, int nzf, int nb, hipStream_t st) {
  return bcr_all(false, bred, x, Bk, lv, nblocks, bstride, nzf, nb, st);
}

hipError_t bcr_fwd(double* b, const double* F, int n, int stride, int neven, int bstride,
                   int nzf, int nb, hipStream_t st) {
  const int total = neven * nb;
  hipLaunchKernelGGL(k_bcr_fwd, dim3(nblk((size_t)total * 4, 256)), dim3(256), 0, st, b, F, n,
                     stride, total, bstride, nzf, nb);
  return hipGetLastError();
}

hipError_t bcr_bwd(const double* b, double* x, const double* Bk, int n, int stride, int nodd,
                   int bstride, int nzf, int nb, hipStream_t st) {
  const int total = nodd * nb;
  hipLaunchKernelGGL(k_bcr_bwd, dim3(nblk((size_t)total * 4, 256)), dim3(256), 0, st, b, x, Bk,
                     n, stride, total, bstride, nzf, nb);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// FP64 outer-loop kernels.  Every reduction writes NRED block partials in a fixed layout;
// consumers sum them in a fixed order, so results are bitwise reproducible.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(RED_THREADS) void k_resid64(const double* __restrict__ b,
                                                         const double* __restrict__ y,
                                                         const double* __restrict__ S,
                                                         double* __restrict__ r, double* prr,
                                                         double* pbb, unsigned N, unsigned nzn,
                                                         unsigned P) {
  __shared__ double sh[16];
  double a = 0, c = 0;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    const double bv = b[g];
    const double rv = bv - ax_at(y, S, g, nzn, P);
    r[g] = rv;
    a += rv * rv;
    c += bv * bv;
  }
  a = block_sum(a, sh);
  if (pbb) c = block_sum(c, sh);
  if (threadIdx.x == 0) {
    prr[blockIdx.x] = a;
    if (pbb) pbb[blockIdx.x] = c;
  }
}

hipError_t resid64(const double* b, const double* y, const double* S, double* r, double* prr,
                   double* pbb, unsigned N, unsigned nzn, unsigned P, hipStream_t st) {
  acct_add(24.0 * N);
  hipLaunchKernelGGL(k_resid64, dim3(NRED), dim3(RED_THREADS), 0, st, b, y, S, r, prr, pbb, N,
                     nzn, P);
  return hipGetLastError();
}

__global__ __launch_bounds__(RED_THREADS) void k_fixdot64(const double* __restrict__ y,
                                                          const double* __restrict__ S,
                                                          double* __restrict__ q,
                                                          const double* __restrict__ p,
                                                          double* ppq, const double* rz_from,
                                                          double* rz_to, unsigned N,
                                                          unsigned nzn, unsigned P) {
  __shared__ double sh[16];
  double a = 0;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    const double qv = ax_at(y, S, g, nzn, P);
    q[g] = qv;
    a += p[g] * qv;
  }
  a = block_sum(a, sh);
  if (threadIdx.x == 0) ppq[blockIdx.x] = a;
  if (rz_from && blockIdx.x == 0)
    for (int k = threadIdx.x; k < NRED; k += blockDim.x) rz_to[k] = rz_from[k];
}

hipError_t fixdot64(const double* y, const double* S, double* q, const double* p, double* ppq,
                    const double* rz_from, double* rz_to, unsigned N, unsigned nzn, unsigned P,
                    hipStream_t st) {
  acct_add(24.0 * N);
  hipLaunchKernelGGL(k_fixdot64, dim3(NRED), dim3(RED_THREADS), 0, st, y, S, q, p, ppq, rz_from,
                     rz_to, N, nzn, P);
  return hipGetLastError();
}

__global__ __launch_bounds__(RED_THREADS) void k_update_xr(double* __restrict__ x,
                                                           double* __restrict__ r,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ q,
                                                           const double* prz, const double* ppq,
                                                           double* prr, unsigned N) {
  __shared__ double sh[16];
  const double rz = sum_partials(prz, sh);
  const double pq = sum_partials(ppq, sh);
  const double alpha = rz / pq;
  double a = 0;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    x[g] += alpha * p[g];
    const double rv = r[g] - alpha * q[g];
    r[g] = rv;
    a += rv * rv;
  }
  a = block_sum(a, sh);
  if (threadIdx.x == 0) prr[blockIdx.x] = a;
}

hipError_t update_xr(double* x, double* r, const double* p, const double* q, const double* prz,
                     const double* ppq, double* prr, unsigned N, hipStream_t st) {
  acct_add(48.0 * N);
  hipLaunchKernelGGL(k_update_xr, dim3(NRED), dim3(RED_THREADS), 0, st, x, r, p, q, prz, ppq,
                     prr, N);
  return hipGetLastError();
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce_sets(const double* parts, int nsets,
                                                             double* out) {
  __shared__ double sh[16];
  for (int s = 0; s < nsets; ++s) {
    const double v = sum_partials(parts + (size_t)s * NRED, sh);
    if (threadIdx.x == 0) out[s] = v;
    __syncthreads();
  }
}

hipError_t reduce_sets(const double* parts, int nsets, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_sets, dim3(1), dim3(RED_THREADS), 0, st, parts, nsets, out);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_castdot(const T* __restrict__ x0,
                                                         double* __restrict__ z,
                                                         const double* __restrict__ q,
                                                         const double* __restrict__ r,
                                                         double* pzq, double* prz, unsigned N) {
  __shared__ double sh[16];
  double a = 0, c = 0;
  // U elements per batch, all loads issued before the stores (grid-stride order kept)
  constexpr int U = 8;
  const unsigned stride = gridDim.x * blockDim.x;
  for (size_t g0 = 0; g0 < N; g0 += (size_t)U * stride) {
    double zv[U], qv[U], rv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t g = g0 + blockIdx.x * blockDim.x + threadIdx.x + (size_t)u * stride;
      const bool ok = g < N;
      zv[u] = ok ? (double)x0[g] : 0.0;
      qv[u] = (ok && q) ? q[g] : 0.0;
      rv[u] = ok ? r[g] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t g = g0 + blockIdx.x * blockDim.x + threadIdx.x + (size_t)u * stride;
      if (g < N) {
        z[g] = zv[u];
        if (q) a += zv[u] * qv[u];
        c += rv[u] * zv[u];
      }
    }
  }
  if (q) a = block_sum(a, sh);
  c = block_sum(c, sh);
  if (threadIdx.x == 0) {
    if (q) pzq[blockIdx.x] = a;
    prz[blockIdx.x] = c;
  }
}

hipError_t castdot(bool dbl_src, const void* x0, double* z, const double* q, const double* r,
                   double* pzq, double* prz, unsigned N, hipStream_t st) {
  acct_add(vsz(dbl_src) * N + 8.0 * N * (q ? 3 : 2));
  if (dbl_src)
    hipLaunchKernelGGL(k_castdot<double>, dim3(NRED), dim3(RED_THREADS), 0, st,
                       (const double*)x0, z, q, r, pzq, prz, N);
  else
    hipLaunchKernelGGL(k_castdot<float>, dim3(NRED), dim3(RED_THREADS), 0, st, (const float*)x0,
                       z, q, r, pzq, prz, N);
  return hipGetLastError();
}

__global__ __launch_bounds__(RED_THREADS) void k_pupdate(double* __restrict__ p,
                                                         const double* __restrict__ z,
                                                         const double* prz_old,
                                                         const double* ppq, const double* pzq,
                                                         int first, unsigned N) {
  __shared__ double sh[16];
  double beta = 0.0;
  if (!first) {
    const double rz = sum_partials(prz_old, sh);
    const double pq = sum_partials(ppq, sh);
    const double zq = sum_partials(pzq, sh);
    const double alpha = rz / pq;
    beta = -alpha * zq / rz;
  }
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    p[g] = first ? z[g] : z[g] + beta * p[g];
}

hipError_t pupdate(double* p, const double* z, const double* prz_old, const double* ppq,
                   const double* pzq, int first, unsigned N, hipStream_t st) {
  acct_add(8.0 * N * (first ? 2 : 3));
  hipLaunchKernelGGL(k_pupdate, dim3(NRED), dim3(RED_THREADS), 0, st, p, z, prz_old, ppq, pzq,
                     first, N);
  return hipGetLastError();
}

__global__ void k_axpy64(double* __restrict__ x, const double* __restrict__ z, double a,
                         unsigned N) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    x[g] += a * z[g];
}

hipError_t axpy64(double* x, const double* z, double a, unsigned N, hipStream_t st) {
  acct_add(24.0 * N);
  hipLaunchKernelGGL(k_axpy64, dim3(nblk(N, 256)), dim3(256), 0, st, x, z, a, N);
  return hipGetLastError();
}

__global__ void k_copy_top(double* __restrict__ x, const double* __restrict__ src, unsigned ncols,
                           unsigned nzn) {
  const unsigned c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncols) x[(size_t)c * nzn + nzn - 1] = src[(size_t)c * nzn + nzn - 1];
}

hipError_t copy_top(double* x, const double* src, unsigned ncols, unsigned nzn, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_top, dim3(nblk(ncols, 256)), dim3(256), 0, st, x, src, ncols, nzn);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_dot_partial(const T* __restrict__ a,
                                                             const T* __restrict__ b,
                                                             double* part, unsigned N) {
  __shared__ double sh[16];
  double s = 0;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    s += (double)a[g] * (double)b[g];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

hipError_t dot_partial(bool dbl, const void* a, const void* b, double* part, unsigned N,
                       hipStream_t st) {
  acct_add(2 * vsz(dbl) * N);
  if (dbl)
    hipLaunchKernelGGL(k_dot_partial<double>, dim3(NRED), dim3(RED_THREADS), 0, st,
                       (const double*)a, (const double*)b, part, N);
  else
    hipLaunchKernelGGL(k_dot_partial<float>, dim3(NRED), dim3(RED_THREADS), 0, st,
                       (const float*)a, (const float*)b, part, N);
  return hipGetLastError();
}

template <typename T>
__global__ void k_vmul(const T* __restrict__ a, const T* __restrict__ s, T* __restrict__ o,
                       unsigned N) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    o[g] = a[g] * s[g];
}

hipError_t vmul(bool dbl, const void* a, const void* s, void* out, unsigned N, hipStream_t st) {
  acct_add(3 * vsz(dbl) * N);
  if (dbl)
    hipLaunchKernelGGL(k_vmul<double>, dim3(nblk(N, 256)), dim3(256), 0, st, (const double*)a,
                       (const double*)s, (double*)out, N);
  else
    hipLaunchKernelGGL(k_vmul<float>, dim3(nblk(N, 256)), dim3(256), 0, st, (const float*)a,
                       (const float*)s, (float*)out, N);
  return hipGetLastError();
}

template <typename T>
__global__ void k_vaxpby(T alpha, const T* a, T beta, const T* b, T* o, unsigned N) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    o[g] = alpha * a[g] + beta * b[g];
}

hipError_t vaxpby(bool dbl, double alpha, const void* a, double beta, const void* b, void* out,
                  unsigned N, hipStream_t st) {
  acct_add(3 * vsz(dbl) * N);
  if (dbl)
    hipLaunchKernelGGL(k_vaxpby<double>, dim3(nblk(N, 256)), dim3(256), 0, st, alpha,
                       (const double*)a, beta, (const double*)b, (double*)out, N);
  else
    hipLaunchKernelGGL(k_vaxpby<float>, dim3(nblk(N, 256)), dim3(256), 0, st, (float)alpha,
                       (const float*)a, (float)beta, (const float*)b, (float*)out, N);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// right-hand side
// ------------------------------------------------------------------------------------------
__global__ void k_rhs_mass(const double* __restrict__ m, const double* __restrict__ f,
                           double* __restrict__ rhs, unsigned N) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    rhs[g] = f ? m[g] * f[g] : 0.0;
}

hipError_t rhs_mass(const double* mass, const double* f, double* rhs, unsigned N, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs_mass, dim3(nblk(N, 256)), dim3(256), 0, st, mass, f, rhs, N);
  return hipGetLastError();
}

__global__ void k_rhs_face(const long long* __restrict__ idx, const double* __restrict__ w,
                           const double* __restrict__ g, double* __restrict__ rhs, unsigned n) {
  const unsigned k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) rhs[idx[k]] += w[k] * g[k];
}

hipError_t rhs_face(const long long* idx, const double* w, const double* g, double* rhs,
                    unsigned n, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs_face, dim3(nblk(n, 256)), dim3(256), 0, st, idx, w, g, rhs, n);
  return hipGetLastError();
}

__global__ void k_rhs_lift(double* __restrict__ rhs, const double* __restrict__ y,
                           const double* __restrict__ S, const double* __restrict__ gD,
                           unsigned N, unsigned nzn, unsigned P) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    const unsigned col = g / nzn;
    if (g - col * nzn == nzn - 1) rhs[g] = gD ? gD[col] : 0.0;
    else rhs[g] -= ax_at(y, S, g, nzn, P);
  }
}

hipError_t rhs_lift(double* rhs, const double* y, const double* S, const double* gD, unsigned N,
                    unsigned nzn, unsigned P, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs_lift, dim3(nblk(N, 256)), dim3(256), 0, st, rhs, y, S, gD, N, nzn, P);
  return hipGetLastError();
}

__global__ void k_scatter_top(double* __restrict__ v, const double* __restrict__ gD,
                              unsigned ncols, unsigned nzn) {
  const unsigned c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncols) v[(size_t)c * nzn + nzn - 1] = gD ? gD[c] : 0.0;
}

hipError_t scatter_top(double* v, const double* gD, unsigned ncols, unsigned nzn, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_top, dim3(nblk(ncols, 256)), dim3(256), 0, st, v, gD, ncols, nzn);
  return hipGetLastError();
}

}  // namespace semk
