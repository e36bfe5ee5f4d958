// Element-local MLP of the learned smoothing stage on gfx950: BF16 MFMA (16x16x16, FP32
// accumulate) GEMMs, exact-erf GELU, MSE loss, Adam, and the fused per-wave inference kernel
// used inside the V-cycle.  The stage itself (features, output scaling, weighted assembly,
// energy-optimal step and its acceptance test) is described in mlp.h / sem.h.
#include "mlp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "host_math.h"
#include "kernels.h"

namespace semm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

static inline unsigned nblk(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// float -> bfloat16 bits, IEEE round to nearest even (the gfx950 conversion instruction)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// erf by Abramowitz & Stegun, Handbook of Mathematical Functions, formula 7.1.26 (after Hastings):
// erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2), t = 1 / (1 + p x), x >= 0,
// absolute error <= 1.5e-7, far below the bfloat16 rounding (2^-9 relative) that every hidden
// activation goes through next
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  const float poly =
      t * fmaf(fmaf(fmaf(fmaf(1.061405429f, t, -1.453152027f), t, 1.421413741f), t, -0.284496736f), t,
               0.254829592f);
  return copysignf(1.0f - poly * __expf(-ax * ax), x);
}
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) +
         x * __expf(-0.5f * x * x) * 0.39894228040143268f;
}
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// MFMA 16x16x16 operand layout (wave64): lane l holds A[l%16][4(l/16)+v] and B[4(l/16)+v][l%16]
// for v = 0..3, and the result D[4(l/16)+v][l%16].

// ------------------------------------------------------------------------------------------
// generic GEMM (training and set-up): C = A B (+ C).  One workgroup owns a 16 x 64 block of C
// and its GEMM_W waves split the K range (wave w takes the 16-wide k-steps w, w + GEMM_W,
// ...).  A wave issues the loads of up to GEMM_CH k-steps before its first product, so one
// memory latency covers a whole chunk; the partial blocks are summed through LDS in wave order
// (the result does not depend on timing).  Operands whose k direction is contiguous (A and B
// with unit k stride) load a lane's four k values as one 8-byte word.
// ------------------------------------------------------------------------------------------
constexpr int GEMM_CH = 8, GEMM_W = 8;

template <bool VEC>
__device__ __forceinline__ bf16x4 frag_load(const uint16_t* p, long sk) {
  if constexpr (VEC) {
    return __builtin_bit_cast(bf16x4, *reinterpret_cast<const uint2*>(p));
  } else {
    bf16x4 r;
#pragma unroll
    for (int v = 0; v < 4; ++v) r[v] = (short)p[v * sk];
    return r;
  }
}

template <bool AV, bool BV, int EPI>
__global__ __launch_bounds__(64 * GEMM_W) void k_gemm_bf16(const uint16_t* __restrict__ A,
                                                          long sam, long sak,
                                                          const uint16_t* __restrict__ B, long sbk,
                                                          long sbn, float* __restrict__ C, int ldc,
                                                          int M, int N, int K, int accumulate,
                                                          GemmEpi ep) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.x * 16, n0 = blockIdx.y * 64;
  const int nt = min(4, (N - n0) >> 4);  // 16-column tiles of this block (uniform)
  const int li = lane & 15, kq = (lane >> 4) * 4;
  const int ks = K >> 4;
  const uint16_t* ap = A + (long)(m0 + li) * sam + (long)kq * sak;
  const uint16_t* bp = B + (long)kq * sbk + (long)(n0 + li) * sbn;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int s0 = wave; s0 < ks; s0 += GEMM_W * GEMM_CH) {
    bf16x4 a[GEMM_CH], b[GEMM_CH][4];
#pragma unroll
    for (int c = 0; c < GEMM_CH; ++c) {
      const int s = s0 + GEMM_W * c;
      if (s < ks) {
        a[c] = frag_load<AV>(ap + (long)s * 16 * sak, sak);
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t < nt) b[c][t] = frag_load<BV>(bp + (long)s * 16 * sbk + (long)t * 16 * sbn, sbk);
      }
    }
#pragma unroll
    for (int c = 0; c < GEMM_CH; ++c) {
      if (s0 + GEMM_W * c < ks) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t < nt) acc[t] = mfma16(a[c], b[c][t], acc[t]);
      }
    }
  }
  __shared__ f32x4 part[GEMM_W][4][64];  // [wave][tile][lane]
#pragma unroll
  for (int t = 0; t < 4; ++t) part[wave][t][lane] = acc[t];
  __syncthreads();
  const int t = wave;  // wave w < 4 sums and stores tile w
  if (t >= nt) return;
  f32x4 s = part[0][t][lane];
#pragma unroll
  for (int w = 1; w < GEMM_W; ++w) s += part[w][t][lane];
  const int n = n0 + 16 * t + li;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const long r = m0 + kq + v;
    float* cp = C + r * ldc + n;
    if constexpr (EPI == 0) {
      *cp = accumulate ? *cp + s[v] : s[v];
    } else {
      float o;
      uint16_t h;
      if constexpr (EPI == GemmEpi::BIAS_GELU) {
        o = s[v] + ep.bias[n];
        h = f2bf(gelu(o));
      } else {
        o = s[v] * gelu_grad(ep.Zin[r * ldc + n]);
        h = f2bf(o);
      }
      *cp = o;
      ep.Hb[r * ldc + n] = h;
      if (ep.HT) ep.HT[(long)n * ep.ldT + r] = h;
    }
  }
}

template <int EPI>
void launch_gemm(bool av, bool bv, dim3 grid, const uint16_t* A, long sam, long sak,
                 const uint16_t* B, long sbk, long sbn, float* C, int ldc, int M, int N, int K,
                 int accumulate, const GemmEpi& ep, hipStream_t st) {
  if (av && bv)
    hipLaunchKernelGGL((k_gemm_bf16<true, true, EPI>), grid, dim3(64 * GEMM_W), 0, st, A, sam,
                       sak, B, sbk, sbn, C, ldc, M, N, K, accumulate, ep);
  else if (av)
    hipLaunchKernelGGL((k_gemm_bf16<true, false, EPI>), grid, dim3(64 * GEMM_W), 0, st, A, sam,
                       sak, B, sbk, sbn, C, ldc, M, N, K, accumulate, ep);
  else  // (a k-contiguous B alone takes the element loads too: no such product in this library)
    hipLaunchKernelGGL((k_gemm_bf16<false, false, EPI>), grid, dim3(64 * GEMM_W), 0, st, A, sam,
                       sak, B, sbk, sbn, C, ldc, M, N, K, accumulate, ep);
}

hipError_t gemm_bf16(const uint16_t* A, long sam, long sak, const uint16_t* B, long sbk, long sbn,
                     float* C, int ldc, int M, int N, int K, int accumulate, hipStream_t st,
                     const GemmEpi* epi) {
  if (M % 16 || N % 16 || K % 16 || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
  if (epi && (accumulate || !epi->Hb || (epi->kind == GemmEpi::BIAS_GELU ? !epi->bias : !epi->Zin)))
    return hipErrorInvalidValue;
  // 8-byte fragment loads need a unit k stride, a row stride that keeps every row's start on
  // 8 bytes, and an 8-byte aligned base
  const bool av = sak == 1 && sam % 4 == 0 && ((uintptr_t)A & 7) == 0;
  const bool bv = sbk == 1 && sbn % 4 == 0 && ((uintptr_t)B & 7) == 0;
  const dim3 grid(M / 16, nblk(N, 64));
  const GemmEpi none{GemmEpi::BIAS_GELU, nullptr, nullptr, nullptr, nullptr, 0};
  if (!epi)
    launch_gemm<0>(av, bv, grid, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, accumulate, none, st);
  else if (epi->kind == GemmEpi::BIAS_GELU)
    launch_gemm<GemmEpi::BIAS_GELU>(av, bv, grid, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, 0,
                                    *epi, st);
  else
    launch_gemm<GemmEpi::GELU_BACK>(av, bv, grid, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, 0,
                                    *epi, st);
  return hipGetLastError();
}

__global__ void k_to_bf16_padded(const float* __restrict__ src, int rows, int cols, int lds,
                                 uint16_t* __restrict__ dst, int ldd, int dcols,
                                 const int* __restrict__ rowidx, uint16_t* __restrict__ dstT,
                                 int ldT) {
  const long total = (long)rows * dcols;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int r = (int)(t / dcols), c = (int)(t - (long)r * dcols);
    const int sr = rowidx ? rowidx[r] : r;
    const float v = (sr >= 0 && c < cols) ? src[(long)sr * lds + c] : 0.0f;
    dst[(long)r * ldd + c] = f2bf(v);
    if (dstT) dstT[(long)c * ldT + r] = f2bf(v);
  }
}

hipError_t to_bf16_padded(const float* src, int rows, int cols, int lds, uint16_t* dst, int ldd,
                          int dcols, const int* rowidx, hipStream_t st, uint16_t* dstT, int ldT) {
  const long total = (long)rows * dcols;
  hipLaunchKernelGGL(k_to_bf16_padded, dim3(std::min<long>(nblk(total, 256), 65535)), dim3(256), 0,
                     st, src, rows, cols, lds, dst, ldd, dcols, rowidx, dstT, ldT);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// training element-wise kernels
// ------------------------------------------------------------------------------------------
// y = Y + b3 on the first nout columns; d = y - t on valid rows (< nvalid; t = row idx[r] of T,
// read in place); dY = 2 d / (nvalid nout) (fp32 and bf16, padded columns and rows zero; the
// bf16 also transposed into dYbT [ldy x ldT]); Y is overwritten with y; per-block partial sums
// of d^2 into part[blockIdx.x]
__global__ __launch_bounds__(256) void k_loss_grad(float* __restrict__ Y, const float* __restrict__ b3,
                                                   const float* __restrict__ T, int ldt,
                                                   float* __restrict__ dYf,
                                                   uint16_t* __restrict__ dYb, int M, int ldy,
                                                   int nout, int nvalid, double* part,
                                                   uint16_t* __restrict__ dYbT, int ldT,
                                                   const int* __restrict__ idx) {
  __shared__ double sh[8];
  double acc = 0.0;
  const float scale = 2.0f / ((float)nvalid * (float)nout);
  const long total = (long)M * ldy;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int r = (int)(t / ldy), c = (int)(t - (long)r * ldy);
    float g = 0.0f;
    if (c < nout) {
      const float y = Y[t] + b3[c];
      Y[t] = y;
      if (r < nvalid) {
        const float d = y - T[(long)idx[r] * ldt + c];
        acc += (double)d * (double)d;
        g = scale * d;
      }
    }
    dYf[t] = g;
    dYb[t] = f2bf(g);
    dYbT[(long)c * ldT + r] = f2bf(g);
  }
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    part[blockIdx.x] = s;
  }
}

// out[c] = sum_r D[r][c], c < N: 64 columns per block (coalesced rows), 16 row groups summed in
// a fixed order
__global__ __launch_bounds__(1024) void k_colsum(const float* __restrict__ D, int M, int N, int ld,
                                                 float* __restrict__ out) {
  __shared__ float part[16][64];
  const int cl = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  float s = 0.0f;
  if (c < N) {
    // eight rows' loads issued before their sum (one memory latency per eight rows)
    int r = rg;
    for (; r + 7 * 16 < M; r += 8 * 16) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = D[(long)(r + 16 * u) * ld + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; r < M; r += 16) s += D[(long)r * ld + c];
  }
  part[rg][cl] = s;
  __syncthreads();
  if (rg == 0 && c < N) {
    float t = 0.0f;
    for (int k = 0; k < 16; ++k) t += part[k][cl];
    out[c] = t;
  }
}

static void colsum(const float* D, int M, int N, int ld, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3(nblk(N, 64)), dim3(1024), 0, st, D, M, N, ld, out);
}

// Adam on FP32 master weights of all six parameter tensors in one launch; g, m, v hold the
// tensors back to back (tensor i from off[i]), the weights sit in their own buffers, wb[i] is
// the bf16 copy and wbt[i] the transposed bf16 copy of a [rows x cols] tensor (either may be
// null)
struct AdamSlots {
  float* w[6];
  uint16_t* wb[6];
  uint16_t* wbt[6];
  int cols[6];
  long off[7];
};

__global__ void k_adam(AdamSlots sl, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr_t, float b1, float b2, float eps, float c1,
                       float c2) {
  const long n = sl.off[6];
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    int i = 0;
    while (t >= sl.off[i + 1]) ++i;
    const long j = t - sl.off[i];
    const float gi = g[t];
    const float mi = b1 * m[t] + (1.0f - b1) * gi;
    const float vi = b2 * v[t] + (1.0f - b2) * gi * gi;
    m[t] = mi;
    v[t] = vi;
    const float wi = sl.w[i][j] - lr_t * (mi / c1) / (sqrtf(vi / c2) + eps);
    sl.w[i][j] = wi;
    const uint16_t h = f2bf(wi);
    if (sl.wb[i]) sl.wb[i][j] = h;
    if (sl.wbt[i]) {
      const long r = j / sl.cols[i], c = j - r * sl.cols[i];
      sl.wbt[i][c * ((sl.off[i + 1] - sl.off[i]) / sl.cols[i]) + r] = h;
    }
  }
}

__global__ void k_out_bias(const float* __restrict__ Y, int ldy, const float* __restrict__ b,
                           int rows, int cols, float* __restrict__ out) {
  const long total = (long)rows * cols;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int r = (int)(t / cols), c = (int)(t - (long)r * cols);
    out[t] = Y[(long)r * ldy + c] + b[c];
  }
}

// Z[r][c] += b[c]
__global__ void k_add_bias(float* __restrict__ Z, const float* __restrict__ b, int rows, int cols) {
  const long total = (long)rows * cols;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x)
    Z[t] += b[t % cols];
}

hipError_t add_bias(float* Z, const float* b, int rows, int cols, hipStream_t st) {
  hipLaunchKernelGGL(k_add_bias, dim3(nblk((size_t)rows * cols, 256)), dim3(256), 0, st, Z, b,
                     rows, cols);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// host: network container, blob, init
// ------------------------------------------------------------------------------------------
struct BlobHeader {
  uint32_t magic, version, nin, nh, nout, epochs, steps, reserved;
  uint64_t seed;
  float train_loss, val_loss;
  uint32_t pad[4];
};
static_assert(sizeof(BlobHeader) == 64, "blob header is 64 bytes");
static const uint32_t kMagic = 0x4e4d4553u;  // "SEMN"

size_t blob_size(int nin, int nout) {
  const size_t np = (size_t)nin * NH + NH + (size_t)NH * NH + NH + (size_t)NH * nout + nout;
  return sizeof(BlobHeader) + np * sizeof(float);
}

bool net_from_blob(const void* blob, size_t nbytes, Net& net, std::string& err) {
  if (!blob || nbytes < sizeof(BlobHeader)) { err = "blob too small"; return false; }
  BlobHeader h;
  std::memcpy(&h, blob, sizeof h);
  if (h.magic != kMagic || h.version != 1 || h.nh != (uint32_t)NH) { err = "not a network blob"; return false; }
  if (h.nin == 0 || h.nout == 0 || h.nin > 4096 || h.nout > 4096) { err = "bad blob sizes"; return false; }
  if (nbytes != blob_size(h.nin, h.nout)) { err = "blob size mismatch"; return false; }
  net.nin = h.nin;
  net.nout = h.nout;
  net.seed = h.seed;
  net.train_loss = h.train_loss;
  net.val_loss = h.val_loss;
  net.epochs = h.epochs;
  net.steps = h.steps;
  const float* p = (const float*)((const char*)blob + sizeof h);
  auto take = [&](std::vector<float>& v, size_t n) { v.assign(p, p + n); p += n; };
  take(net.W1, (size_t)h.nin * NH);
  take(net.b1, NH);
  take(net.W2, (size_t)NH * NH);
  take(net.b2, NH);
  take(net.W3, (size_t)NH * h.nout);
  take(net.b3, h.nout);
  return true;
}

void net_to_blob(const Net& net, void* blob) {
  BlobHeader h{};
  h.magic = kMagic;
  h.version = 1;
  h.nin = net.nin;
  h.nh = NH;
  h.nout = net.nout;
  h.epochs = net.epochs;
  h.steps = net.steps;
  h.seed = net.seed;
  h.train_loss = net.train_loss;
  h.val_loss = net.val_loss;
  std::memcpy(blob, &h, sizeof h);
  float* p = (float*)((char*)blob + sizeof h);
  for (const auto* v : {&net.W1, &net.b1, &net.W2, &net.b2, &net.W3, &net.b3}) {
    std::memcpy(p, v->data(), v->size() * sizeof(float));
    p += v->size();
  }
}

void net_init(Net& net, int nin, int nout, uint64_t seed) {
  net.nin = nin;
  net.nout = nout;
  net.seed = seed;
  uint64_t ctr = 0;
  auto fill = [&](std::vector<float>& W, int fan_in, size_t n) {
    W.resize(n);
    const double lim = 1.0 / std::sqrt((double)fan_in);
    for (size_t i = 0; i < n; ++i) W[i] = (float)(lim * semh::splitmix64_uniform(seed, ctr++));
  };
  fill(net.W1, nin, (size_t)nin * NH);
  fill(net.W2, NH, (size_t)NH * NH);
  fill(net.W3, NH, (size_t)NH * nout);
  net.b1.assign(NH, 0.f);
  net.b2.assign(NH, 0.f);
  net.b3.assign(nout, 0.f);
}

// ------------------------------------------------------------------------------------------
// host: training driver
// ------------------------------------------------------------------------------------------
namespace {

struct Dev {
  std::vector<void*> ptrs;
  hipError_t e = hipSuccess;
  template <typename T>
  T* alloc(size_t n) {
    void* p = nullptr;
    hipError_t r = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
    if (r != hipSuccess) { e = r; return nullptr; }
    ptrs.push_back(p);
    return (T*)p;
  }
  ~Dev() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

#define CK(x)                                 \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) {                   \
      err = std::string(#x) + ": " + hipGetErrorString(e_); \
      return false;                           \
    }                                         \
  } while (0)

// padded parameter set on the device (fp32 masters + bf16 copies)
struct Params {
  int nin, nout, K1, N3;
  float *W1, *b1, *W2, *b2, *W3, *b3;      // padded: W1 [K1 x NH], W3 [NH x N3], b3 [N3]
  uint16_t *W1b, *W2b, *W3b;
  // transposed bf16 copies (W1bT [NH x K1], W2bT [NH x NH], W3bT [N3 x NH]), so that the forward
  // products read k-contiguous fragments; null where only the row-major copies are kept
  uint16_t *W1bT = nullptr, *W2bT = nullptr, *W3bT = nullptr;
  size_t n1() const { return (size_t)K1 * NH; }
  size_t n2() const { return (size_t)NH * NH; }
  size_t n3() const { return (size_t)NH * N3; }
};

bool alloc_params(Dev& d, Params& p, int nin, int nout) {
  p.nin = nin;
  p.nout = nout;
  p.K1 = pad16(nin);
  p.N3 = pad16(nout);
  p.W1 = d.alloc<float>(p.n1());
  p.b1 = d.alloc<float>(NH);
  p.W2 = d.alloc<float>(p.n2());
  p.b2 = d.alloc<float>(NH);
  p.W3 = d.alloc<float>(p.n3());
  p.b3 = d.alloc<float>(p.N3);
  p.W1b = d.alloc<uint16_t>(p.n1());
  p.W2b = d.alloc<uint16_t>(p.n2());
  p.W3b = d.alloc<uint16_t>(p.n3());
  p.W1bT = d.alloc<uint16_t>(p.n1());
  p.W2bT = d.alloc<uint16_t>(p.n2());
  p.W3bT = d.alloc<uint16_t>(p.n3());
  return d.e == hipSuccess;
}

bool upload_params(const Net& net, Params& p, hipStream_t st, std::string& err) {
  std::vector<float> W1((size_t)p.K1 * NH, 0.f), W3((size_t)NH * p.N3, 0.f), b3(p.N3, 0.f);
  for (int k = 0; k < net.nin; ++k)
    for (int n = 0; n < NH; ++n) W1[(size_t)k * NH + n] = net.W1[(size_t)k * NH + n];
  for (int k = 0; k < NH; ++k)
    for (int n = 0; n < net.nout; ++n) W3[(size_t)k * p.N3 + n] = net.W3[(size_t)k * net.nout + n];
  for (int n = 0; n < net.nout; ++n) b3[n] = net.b3[n];
  CK(hipMemcpyAsync(p.W1, W1.data(), W1.size() * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(p.W2, net.W2.data(), net.W2.size() * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(p.W3, W3.data(), W3.size() * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(p.b1, net.b1.data(), NH * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(p.b2, net.b2.data(), NH * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(p.b3, b3.data(), p.N3 * 4, hipMemcpyHostToDevice, st));
  CK(to_bf16_padded(p.W1, p.K1, NH, NH, p.W1b, NH, NH, nullptr, st, p.W1bT, p.K1));
  CK(to_bf16_padded(p.W2, NH, NH, NH, p.W2b, NH, NH, nullptr, st, p.W2bT, NH));
  CK(to_bf16_padded(p.W3, NH, p.N3, p.N3, p.W3b, p.N3, p.N3, nullptr, st, p.W3bT, NH));
  CK(hipStreamSynchronize(st));
  return true;
}

bool download_params(const Params& p, Net& net, hipStream_t st, std::string& err) {
  std::vector<float> W1((size_t)p.K1 * NH), W3((size_t)NH * p.N3), b3(p.N3);
  net.W2.resize((size_t)NH * NH);
  net.b1.resize(NH);
  net.b2.resize(NH);
  CK(hipMemcpyAsync(W1.data(), p.W1, W1.size() * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(net.W2.data(), p.W2, net.W2.size() * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(W3.data(), p.W3, W3.size() * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(net.b1.data(), p.b1, NH * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(net.b2.data(), p.b2, NH * 4, hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(b3.data(), p.b3, p.N3 * 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  net.W1.resize((size_t)p.nin * NH);
  net.W3.resize((size_t)NH * p.nout);
  net.b3.resize(p.nout);
  for (int k = 0; k < p.nin; ++k)
    for (int n = 0; n < NH; ++n) net.W1[(size_t)k * NH + n] = W1[(size_t)k * NH + n];
  for (int k = 0; k < NH; ++k)
    for (int n = 0; n < p.nout; ++n) net.W3[(size_t)k * p.nout + n] = W3[(size_t)k * p.N3 + n];
  for (int n = 0; n < p.nout; ++n) net.b3[n] = b3[n];
  return true;
}

// activations of one batch of at most Bmax rows
struct Acts {
  int Bmax, K1, N3;
  uint16_t *Xb, *H1b, *H2b, *dYb, *dZ2b, *dZ1b;
  // batch-major (transposed) bf16 copies [cols x Bmax] for the weight-gradient products, whose
  // k index is the batch row; null in the forward-only set
  uint16_t *XbT = nullptr, *H1bT = nullptr, *H2bT = nullptr, *dYbT = nullptr, *dZ2bT = nullptr,
           *dZ1bT = nullptr;
  float *Z1, *Z2, *Y, *dYf, *dZ2f, *dZ1f;
  int* idx;
  double* part;
};

bool alloc_acts(Dev& d, Acts& a, int Bmax, int K1, int N3) {
  a.Bmax = Bmax;
  a.K1 = K1;
  a.N3 = N3;
  const size_t B = Bmax;
  a.Xb = d.alloc<uint16_t>(B * K1);
  a.H1b = d.alloc<uint16_t>(B * NH);
  a.H2b = d.alloc<uint16_t>(B * NH);
  a.dYb = d.alloc<uint16_t>(B * N3);
  a.dZ2b = d.alloc<uint16_t>(B * NH);
  a.dZ1b = d.alloc<uint16_t>(B * NH);
  a.XbT = d.alloc<uint16_t>(B * K1);
  a.H1bT = d.alloc<uint16_t>(B * NH);
  a.H2bT = d.alloc<uint16_t>(B * NH);
  a.dYbT = d.alloc<uint16_t>(B * N3);
  a.dZ2bT = d.alloc<uint16_t>(B * NH);
  a.dZ1bT = d.alloc<uint16_t>(B * NH);
  a.Z1 = d.alloc<float>(B * NH);
  a.Z2 = d.alloc<float>(B * NH);
  a.Y = d.alloc<float>(B * N3);
  a.dYf = d.alloc<float>(B * N3);
  a.dZ2f = d.alloc<float>(B * NH);
  a.dZ1f = d.alloc<float>(B * NH);
  a.idx = d.alloc<int>(B);
  a.part = d.alloc<double>(256);
  return d.e == hipSuccess;
}

constexpr int LOSS_BLOCKS = 64;

// forward of rows idx[0..M) (M multiple of 16; idx < 0 = zero row); Y holds y on return
bool fwd(const Params& p, Acts& a, const float* X, int M, hipStream_t st, std::string& err) {
  const int lt = a.Bmax;
  CK(to_bf16_padded(X, M, p.nin, p.nin, a.Xb, p.K1, p.K1, a.idx, st, a.XbT, lt));
  // B = W (K x N): the transposed copy gives unit k stride
  const bool wt = p.W1bT != nullptr;
  // hidden layers: Z = X W + b and H = bf16(GELU(Z)) (and its batch-major copy) in the epilogue
  const GemmEpi e1{GemmEpi::BIAS_GELU, p.b1, nullptr, a.H1b, a.H1bT, lt};
  CK(gemm_bf16(a.Xb, p.K1, 1, wt ? p.W1bT : p.W1b, wt ? 1 : NH, wt ? p.K1 : 1, a.Z1, NH, M, NH,
               p.K1, 0, st, &e1));
  const GemmEpi e2{GemmEpi::BIAS_GELU, p.b2, nullptr, a.H2b, a.H2bT, lt};
  CK(gemm_bf16(a.H1b, NH, 1, wt ? p.W2bT : p.W2b, wt ? 1 : NH, wt ? NH : 1, a.Z2, NH, M, NH, NH, 0,
               st, &e2));
  CK(gemm_bf16(a.H2b, NH, 1, wt ? p.W3bT : p.W3b, wt ? 1 : p.N3, wt ? NH : 1, a.Y, p.N3, M, p.N3,
               NH, 0, st));
  return true;
}

// loss (sum of squares over valid rows) + gradients into padded g buffers
bool bwd(const Params& p, Acts& a, const float* Tsrc, int M, int nvalid, float* gW1, float* gb1,
         float* gW2, float* gb2, float* gW3, float* gb3, hipStream_t st, std::string& err) {
  if (!a.H1bT || !a.H2bT || !a.dYbT || !a.dZ2bT || !a.dZ1bT || !a.XbT) {
    err = "gradient pass without the batch-major activation copies";
    return false;
  }
  const int lt = a.Bmax;
  hipLaunchKernelGGL(k_loss_grad, dim3(LOSS_BLOCKS), dim3(256), 0, st, a.Y, p.b3, Tsrc, p.nout,
                     a.dYf, a.dYb, M, p.N3, p.nout, nvalid, a.part, a.dYbT, lt, a.idx);
  CK(hipGetLastError());
  // dW3 = H2^T dY, db3 = colsum dY
  CK(gemm_bf16(a.H2bT, lt, 1, a.dYbT, 1, lt, gW3, p.N3, NH, p.N3, M, 0, st));
  colsum(a.dYf, M, p.N3, p.N3, gb3, st);
  // dZ2 = (dY W3^T) * gelu'(Z2), the factor applied in the product's epilogue
  const GemmEpi g2{GemmEpi::GELU_BACK, nullptr, a.Z2, a.dZ2b, a.dZ2bT, lt};
  CK(gemm_bf16(a.dYb, p.N3, 1, p.W3b, 1, p.N3, a.dZ2f, NH, M, NH, p.N3, 0, st, &g2));
  // dW2 = H1^T dZ2, db2
  CK(gemm_bf16(a.H1bT, lt, 1, a.dZ2bT, 1, lt, gW2, NH, NH, NH, M, 0, st));
  colsum(a.dZ2f, M, NH, NH, gb2, st);
  // dZ1 = (dZ2 W2^T) * gelu'(Z1)
  const GemmEpi g1{GemmEpi::GELU_BACK, nullptr, a.Z1, a.dZ1b, a.dZ1bT, lt};
  CK(gemm_bf16(a.dZ2b, NH, 1, p.W2b, 1, NH, a.dZ1f, NH, M, NH, NH, 0, st, &g1));
  // dW1 = X^T dZ1, db1
  CK(gemm_bf16(a.XbT, lt, 1, a.dZ1bT, 1, lt, gW1, NH, p.K1, NH, M, 0, st));
  colsum(a.dZ1f, M, NH, NH, gb1, st);
  CK(hipGetLastError());
  return true;
}

double read_loss(Acts& a, hipStream_t st, std::string& err, bool& ok) {
  double h[LOSS_BLOCKS];
  ok = hipMemcpyAsync(h, a.part, sizeof h, hipMemcpyDeviceToHost, st) == hipSuccess &&
       hipStreamSynchronize(st) == hipSuccess;
  if (!ok) err = "loss read-back failed";
  double s = 0;
  for (double v : h) s += v;
  return s;
}

}  // namespace

bool train(const float* X, const float* T, int n, int nin, int nout, const TrainCfg& cfg, Net& net,
           std::vector<float>* losses, hipStream_t st, std::string& err, const Net* init) {
  if (n < 32 || nin < 1 || nout < 1 || cfg.batch < 16 || cfg.epochs < 1) {
    err = "bad training arguments";
    return false;
  }
  if (init && (init->nin != nin || init->nout != nout)) {
    err = "bad initial network (size mismatch)";
    return false;
  }
  const int B = (cfg.batch + 15) / 16 * 16;
  int nval = (int)std::floor(cfg.val_frac * n);
  if (nval < 0) nval = 0;
  const int ntr = n - nval;
  if (init) {
    net = *init;
    net.seed = cfg.seed;
  } else {
    net_init(net, nin, nout, cfg.seed);
  }
  Dev d;
  Params p;
  Acts a;
  if (!alloc_params(d, p, nin, nout) || !alloc_acts(d, a, B, pad16(nin), pad16(nout))) {
    err = "device allocation failed";
    return false;
  }
  const size_t np = p.n1() + NH + p.n2() + NH + p.n3() + p.N3;
  float* g = d.alloc<float>(np);
  float* m = d.alloc<float>(np);
  float* v = d.alloc<float>(np);
  if (d.e != hipSuccess) { err = "device allocation failed"; return false; }
  CK(hipMemsetAsync(m, 0, np * 4, st));
  CK(hipMemsetAsync(v, 0, np * 4, st));
  if (!upload_params(net, p, st, err)) return false;
  float* gW1 = g;
  float* gb1 = gW1 + p.n1();
  float* gW2 = gb1 + NH;
  float* gb2 = gW2 + p.n2();
  float* gW3 = gb2 + NH;
  float* gb3 = gW3 + p.n3();
  AdamSlots slots;
  {
    float* const w[6] = {p.W1, p.b1, p.W2, p.b2, p.W3, p.b3};
    uint16_t* const wb[6] = {p.W1b, nullptr, p.W2b, nullptr, p.W3b, nullptr};
    uint16_t* const wbt[6] = {p.W1bT, nullptr, p.W2bT, nullptr, p.W3bT, nullptr};
    const size_t sz[6] = {p.n1(), NH, p.n2(), NH, p.n3(), (size_t)p.N3};
    const int cols[6] = {NH, NH, NH, NH, p.N3, p.N3};
    slots.off[0] = 0;
    for (int i = 0; i < 6; ++i) {
      slots.w[i] = w[i];
      slots.wb[i] = wb[i];
      slots.wbt[i] = wbt[i];
      slots.cols[i] = cols[i];
      slots.off[i + 1] = slots.off[i] + (long)sz[i];
    }
  }
  const int steps_per_epoch = (ntr + B - 1) / B;
  const long total_steps = (long)steps_per_epoch * cfg.epochs;
  // the row indices of a whole epoch (batch k at k B, -1 pads a short batch to a multiple of 16)
  // go to the device in one copy, and the validation rows' once
  const int vsteps = (nval + B - 1) / B;
  int* eidx = d.alloc<int>((size_t)steps_per_epoch * B);
  int* vidx = vsteps ? d.alloc<int>((size_t)vsteps * B) : nullptr;
  if (d.e != hipSuccess) { err = "device allocation failed"; return false; }
  std::vector<int> perm(ntr), idx((size_t)std::max(steps_per_epoch, vsteps) * B, -1);
  for (int i = 0; i < ntr; ++i) perm[i] = i;
  if (vsteps) {
    for (int r = 0; r < vsteps * B; ++r) idx[r] = r < nval ? ntr + r : -1;
    CK(hipMemcpyAsync(vidx, idx.data(), (size_t)vsteps * B * sizeof(int), hipMemcpyHostToDevice, st));
  }
  uint64_t ctr = 0;
  long step = 0;
  for (int ep = 0; ep < cfg.epochs; ++ep) {
    // Fisher-Yates shuffle with SplitMix64 draws
    for (int i = ntr - 1; i > 0; --i) {
      const double u = 0.5 * (semh::splitmix64_uniform(cfg.seed ^ 0x5eedull, ctr++) + 1.0);
      int j = (int)(u * (i + 1));
      if (j > i) j = i;
      std::swap(perm[i], perm[j]);
    }
    for (int r = 0; r < steps_per_epoch * B; ++r) idx[r] = r < ntr ? perm[r] : -1;
    CK(hipMemcpyAsync(eidx, idx.data(), (size_t)steps_per_epoch * B * sizeof(int),
                      hipMemcpyHostToDevice, st));
    double ep_loss = 0.0;
    long ep_count = 0;
    for (int s0 = 0; s0 < ntr; s0 += B) {
      const int nv = std::min(B, ntr - s0);
      const int M = (nv + 15) / 16 * 16;
      a.idx = eidx + s0;
      if (!fwd(p, a, X, M, st, err)) return false;
      if (!bwd(p, a, T, M, nv, gW1, gb1, gW2, gb2, gW3, gb3, st, err)) return false;
      ++step;
      const double b1 = 0.9, b2 = 0.999;
      const float lr_t = (float)(cfg.lr * 0.5 * (1.0 + std::cos(M_PI * (double)(step - 1) / total_steps)));
      const float c1 = (float)(1.0 - std::pow(b1, (double)step));
      const float c2 = (float)(1.0 - std::pow(b2, (double)step));
      hipLaunchKernelGGL(k_adam, dim3(nblk(np, 256)), dim3(256), 0, st, slots, g, m, v, lr_t,
                         (float)b1, (float)b2, 1e-8f, c1, c2);
      CK(hipGetLastError());
      bool ok = true;
      if (s0 + B >= ntr) {  // epoch loss from the last batch only (cheap); full loss below
        ep_loss = read_loss(a, st, err, ok);
        ep_count = (long)nv * nout;
        if (!ok) return false;
      }
    }
    // validation loss over the held-out rows (full pass)
    double vl = 0.0;
    long vc = 0;
    for (int s0 = 0; s0 < nval; s0 += B) {
      const int nv = std::min(B, nval - s0);
      const int M = (nv + 15) / 16 * 16;
      a.idx = vidx + s0;
      if (!fwd(p, a, X, M, st, err)) return false;
      if (!bwd(p, a, T, M, nv, gW1, gb1, gW2, gb2, gW3, gb3, st, err)) return false;  // loss
      bool ok = true;
      vl += read_loss(a, st, err, ok);
      if (!ok) return false;
      vc += (long)nv * nout;
    }
    net.train_loss = (float)(ep_loss / std::max<long>(1, ep_count));
    net.val_loss = vc ? (float)(vl / vc) : 0.f;
    if (losses) {
      losses->push_back(net.train_loss);
      losses->push_back(net.val_loss);
    }
  }
  net.epochs = cfg.epochs;
  net.steps = (int)step;
  return download_params(p, net, st, err);
}

bool forward(const Net& net, const float* X, int n, float* Y, hipStream_t st, std::string& err) {
  const int B = 1024;
  Dev d;
  Params p;
  Acts a;
  if (!alloc_params(d, p, net.nin, net.nout) || !alloc_acts(d, a, B, pad16(net.nin), pad16(net.nout))) {
    err = "device allocation failed";
    return false;
  }
  if (!upload_params(net, p, st, err)) return false;
  std::vector<int> idx(B);
  for (int s0 = 0; s0 < n; s0 += B) {
    const int nv = std::min(B, n - s0);
    const int M = (nv + 15) / 16 * 16;
    for (int r = 0; r < M; ++r) idx[r] = r < nv ? s0 + r : -1;
    CK(hipMemcpyAsync(a.idx, idx.data(), M * sizeof(int), hipMemcpyHostToDevice, st));
    if (!fwd(p, a, X, M, st, err)) return false;
    // y = Y + b3 into the caller's rows s0 .. s0 + nv
    hipLaunchKernelGGL(k_out_bias, dim3(nblk((size_t)nv * net.nout, 256)), dim3(256), 0, st, a.Y,
                       p.N3, p.b3, nv, net.nout, Y + (size_t)s0 * net.nout);
    CK(hipGetLastError());
    CK(hipStreamSynchronize(st));
  }
  return true;
}

bool gradients(const Net& net, const float* X, const float* T, int n, float* grads, float* loss,
               hipStream_t st, std::string& err) {
  const int M = (n + 15) / 16 * 16;
  Dev d;
  Params p;
  Acts a;
  if (!alloc_params(d, p, net.nin, net.nout) || !alloc_acts(d, a, M, pad16(net.nin), pad16(net.nout))) {
    err = "device allocation failed";
    return false;
  }
  if (!upload_params(net, p, st, err)) return false;
  const size_t np = p.n1() + NH + p.n2() + NH + p.n3() + p.N3;
  float* g = d.alloc<float>(np);
  if (d.e != hipSuccess) { err = "device allocation failed"; return false; }
  std::vector<int> idx(M);
  for (int r = 0; r < M; ++r) idx[r] = r < n ? r : -1;
  CK(hipMemcpyAsync(a.idx, idx.data(), M * sizeof(int), hipMemcpyHostToDevice, st));
  if (!fwd(p, a, X, M, st, err)) return false;
  float* gW1 = g;
  float* gb1 = gW1 + p.n1();
  float* gW2 = gb1 + NH;
  float* gb2 = gW2 + p.n2();
  float* gW3 = gb2 + NH;
  float* gb3 = gW3 + p.n3();
  if (!bwd(p, a, T, M, n, gW1, gb1, gW2, gb2, gW3, gb3, st, err)) return false;
  bool ok = true;
  const double l = read_loss(a, st, err, ok);
  if (!ok) return false;
  if (loss) *loss = (float)(l / ((double)n * net.nout));
  std::vector<float> hg(np);
  CK(hipMemcpy(hg.data(), g, np * 4, hipMemcpyDeviceToHost));
  // pack like the blob (unpadded)
  float* o = grads;
  for (int k = 0; k < net.nin; ++k)
    for (int c = 0; c < NH; ++c) *o++ = hg[(size_t)k * NH + c];
  for (int c = 0; c < NH; ++c) *o++ = hg[p.n1() + c];
  for (size_t k = 0; k < p.n2(); ++k) *o++ = hg[p.n1() + NH + k];
  for (int c = 0; c < NH; ++c) *o++ = hg[p.n1() + NH + p.n2() + c];
  const size_t o3 = p.n1() + 2 * NH + p.n2();
  for (int k = 0; k < NH; ++k)
    for (int c = 0; c < net.nout; ++c) *o++ = hg[o3 + (size_t)k * p.N3 + c];
  for (int c = 0; c < net.nout; ++c) *o++ = hg[o3 + p.n3() + c];
  return true;
}

// ------------------------------------------------------------------------------------------
// inference: one wave = 16 elements; layer 1 split into the residual part (K = n, padded) and
// the precomputed geometric part Z1geo
// ------------------------------------------------------------------------------------------
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

// deterministic block sum (fixed shuffle pattern and LDS order)
__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ double bsum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wsum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < nw; ++k) s += sh[k];
  return s;
}

// acc[t] += W^T(tile t0 + t) . xb over KS k-steps, weights in fragment order (F[(tile KS + k) 64 +
// lane]): the fragments of k-step k + 1 are read from LDS while the MFMAs of k-step k run
template <int NTT, int KS>
__device__ __forceinline__ void layer_mfma(const bf16x4* __restrict__ F, int t0, int lane,
                                           const bf16x4 (&xb)[KS], f32x4 (&acc)[NTT]) {
  bf16x4 w[2][NTT];
#pragma unroll
  for (int t = 0; t < NTT; ++t) w[0][t] = F[((t0 + t) * KS) * 64 + lane];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    if (k + 1 < KS) {
#pragma unroll
      for (int t = 0; t < NTT; ++t) w[(k + 1) & 1][t] = F[((t0 + t) * KS + k + 1) * 64 + lane];
    }
#pragma unroll
    for (int t = 0; t < NTT; ++t) acc[t] = mfma16(w[k & 1][t], xb[k], acc[t]);
  }
}

// Two waves carry a 16-element tile through the network, each computing half of every layer's
// outputs.  Every layer is computed transposed, Z^T = W^T X^T: the weights (stored output-major,
// staged once per workgroup into LDS with padded rows while the residual is being gathered) are
// the MFMA A operand and the activations the B operand.  The result of a 16x16x16 MFMA (lane l
// holds rows 4(l/16)+v of column l%16) is exactly the B operand of the next layer's k-step for
// the same 16 rows, so a wave's half of the hidden activations goes to its partner through one
// 8-byte LDS slot per lane and k-step (double-buffered between the layers, one barrier each).
// Per lane: element le = l%16 of the tile and, in every 16-block of features, the slice
// kq..kq+3 (kq = 4 (l/16)); the residual gathered for layer 1 sits in the same slices as the
// layer-3 output, so each wave also forms its part of c . r for its output half:
// with c = W sum_e R_e^T c_e, c . r = sum_e sum_l c_e[l] r_g / m_g (g the global node of (e, l),
// m_g its multiplicity, weight 0 on the Dirichlet surface when masked).  The workgroup's sum
// goes to pcr[workgroup].
constexpr int MLP_TILES = 4;  // 16-element tiles per workgroup, two waves each
constexpr int MLP_THREADS = 128 * MLP_TILES;

template <int P, typename T>
__global__ __launch_bounds__(MLP_THREADS) void k_stage_mlp(
    const T* __restrict__ r, const uint16_t* __restrict__ W1r, const float* __restrict__ Z1geo,
    const uint16_t* __restrict__ W2, const float* __restrict__ b2,
    const uint16_t* __restrict__ W3, const float* __restrict__ b3,
    const float* __restrict__ abar, float* __restrict__ CE, int E, int Nx, int Nz, unsigned nzn,
    int masked, double* __restrict__ pcr) {
  constexpr int NP = P + 1, n = NP * NP, KR = (n + 15) / 16 * 16, KS = KR / 16, NT = NH / 16;
  constexpr int NTH = NT / 2;          // hidden tiles per wave
  constexpr int K3 = (KS + 1) / 2;     // output tiles per wave (the second may have fewer)
  // the network in LDS, in fragment order: every A-operand read is 64 lanes x 8 contiguous bytes
  __shared__ __align__(16) uint16_t sW[(NH * KR + NH * NH + KR * NH)];
  __shared__ bf16x4 sH[2][MLP_TILES][NT][64];  // exchanged hidden fragments (two buffers)
  const bf16x4* F1 = reinterpret_cast<const bf16x4*>(sW);
  const bf16x4* F2 = reinterpret_cast<const bf16x4*>(sW + NH * KR);
  const bf16x4* F3 = reinterpret_cast<const bf16x4*>(sW + NH * KR + NH * NH);
  __shared__ double sred[MLP_THREADS / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = wave >> 1, h = wave & 1;
  const int le = lane & 15, kq = (lane >> 4) * 4;
  const int e = (blockIdx.x * MLP_TILES + tile) * 16 + le;
  const bool ve = e < E;
  const int ex = ve ? e / Nz : 0, ez = ve ? e - ex * Nz : 0;
  const unsigned base = (unsigned)(ex * P) * nzn + ez * P;

  // residual of this lane's slices (fp32; both waves of a tile gather it), element norm over the
  // 4 lanes of the element
  float rv[KS][4];
  float ss = 0.f;
#pragma unroll
  for (int k = 0; k < KS; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int loc = 16 * k + kq + v;
      rv[k][v] = 0.f;
      if (ve && loc < n) {
        const int i = loc / NP, j = loc - (loc / NP) * NP;
        rv[k][v] = (float)r[base + i * nzn + j];
      }
      ss += rv[k][v] * rv[k][v];
    }
  // the network into LDS (straight 16-byte copies), issued behind the residual loads
  {
    constexpr int c1 = NH * KR / 8, c2 = NH * NH / 8, c3 = KR * NH / 8;
    uint4* d = reinterpret_cast<uint4*>(sW);
    for (int k = threadIdx.x; k < c1; k += MLP_THREADS) d[k] = reinterpret_cast<const uint4*>(W1r)[k];
    for (int k = threadIdx.x; k < c2; k += MLP_THREADS) d[c1 + k] = reinterpret_cast<const uint4*>(W2)[k];
    for (int k = threadIdx.x; k < c3; k += MLP_THREADS) d[c1 + c2 + k] = reinterpret_cast<const uint4*>(W3)[k];
  }
  ss += __shfl_xor(ss, 16, 64);
  ss += __shfl_xor(ss, 32, 64);
  const float sn = sqrtf(ss);
  const float sinv = sn > 0.f ? 1.0f / sn : 0.f;
  bf16x4 xb[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) xb[k][v] = (short)f2bf(rv[k][v] * sinv);

  // three phases per half, with the half index a compile-time constant inside each (register
  // arrays stay statically indexed); the barriers sit between the phases, outside any branch
  double part = 0.0;
  f32x4 acc[NTH];
  bf16x4 hb[NT];
  auto layer1 = [&](auto hc) {  // Z1 = Xr W1r + Z1geo on hidden tiles NTH H ..
    constexpr int H = decltype(hc)::value;
    layer_mfma<NTH, KS>(F1, NTH * H, lane, xb, acc);
#pragma unroll
    for (int t = 0; t < NTH; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) hb[NTH * H + t][v] = (short)f2bf(gelu(acc[t][v]));
      sH[0][tile][NTH * H + t][lane] = hb[NTH * H + t];
    }
  };
  auto layer2 = [&](auto hc) {  // Z2 = H1 W2 + b2
    constexpr int H = decltype(hc)::value;
#pragma unroll
    for (int t = 0; t < NTH; ++t) hb[NTH * (1 - H) + t] = sH[0][tile][NTH * (1 - H) + t][lane];
#pragma unroll
    for (int t = 0; t < NTH; ++t)
      acc[t] = *reinterpret_cast<const f32x4*>(b2 + 16 * (NTH * H + t) + kq);
    layer_mfma<NTH, NT>(F2, NTH * H, lane, hb, acc);
#pragma unroll
    for (int t = 0; t < NTH; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) hb[NTH * H + t][v] = (short)f2bf(gelu(acc[t][v]));
      sH[1][tile][NTH * H + t][lane] = hb[NTH * H + t];
    }
  };
  auto layer3 = [&](auto hc) {  // Y = H2 W3 + b3 on output tiles K3 H ..; c_e, c . r part
    constexpr int H = decltype(hc)::value;
    constexpr int T0 = K3 * H;
#pragma unroll
    for (int t = 0; t < NTH; ++t) hb[NTH * (1 - H) + t] = sH[1][tile][NTH * (1 - H) + t][lane];
    const float sc = ve ? sn / abar[e] : 0.f;
#pragma unroll
    for (int t = 0; t < K3; ++t) {
      const int t3 = T0 + t;
      if (T0 + t >= KS) break;
      f32x4 c[1] = {*reinterpret_cast<const f32x4*>(b3 + 16 * t3 + kq)};
      layer_mfma<1, NT>(F3, t3, lane, hb, c);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int loc = 16 * t3 + kq + v;
        if (ve && loc < n) {
          const float ce = sc * c[0][v];
          const int i = loc / NP, j = loc - (loc / NP) * NP;
          CE[semk::ce_index(ex, i, ez, j, Nz, NP)] = ce;
          // 1 / multiplicity, exact: 1, 1/2 or 1/4
          const double wx = ((i == 0 && ex > 0) || (i == P && ex < Nx - 1)) ? 0.5 : 1.0;
          const double wz = ((j == 0 && ez > 0) || (j == P && ez < Nz - 1)) ? 0.5 : 1.0;
          const bool top = masked && j == P && ez == Nz - 1;
          if (!top) part += (double)ce * (double)rv[t3][v] * (wx * wz);
        }
      }
    }
  };
  using H0 = std::integral_constant<int, 0>;
  using H1 = std::integral_constant<int, 1>;
#pragma unroll
  for (int t = 0; t < NTH; ++t)
    acc[t] = ve ? *reinterpret_cast<const f32x4*>(Z1geo + (long)e * NH + 16 * (NTH * h + t) + kq)
                : (f32x4){0.f, 0.f, 0.f, 0.f};
  __syncthreads();  // the network is in LDS
  if (h == 0) layer1(H0{}); else layer1(H1{});
  __syncthreads();
  if (h == 0) layer2(H0{}); else layer2(H1{});
  __syncthreads();
  if (h == 0) layer3(H0{}); else layer3(H1{});
  part = wsum(part);
  if (lane == 0) sred[wave] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < MLP_THREADS / 64; ++w) tot += sred[w];
    pcr[blockIdx.x] = tot;
  }
}


// 3D form (hexahedra of n = (P+1)^3 nodes, P <= 6): the same two-wave tile scheme, but the
// network (2 (128 KR + 128 128 + KR 128) bytes, up to 208 KB at P = 6) does not fit the LDS, so
// the MFMA A fragments are read from global memory in fragment order (the weights stay in L2);
// only the exchanged hidden fragments use LDS.  Element e = (ex Ny + ey) Nz + ez, local node
// (i NP + m) NP + j; c_e written element-major (CE[e n + l]).  The c . r part uses the exact
// multiplicity weights 1, 1/2, 1/4, 1/8 of nodes on shared faces, edges and corners.
template <int P, typename T>
__global__ __launch_bounds__(MLP_THREADS) void k_stage_mlp3d(
    const T* __restrict__ r, const uint16_t* __restrict__ W1r, const float* __restrict__ Z1geo,
    const uint16_t* __restrict__ W2, const float* __restrict__ b2,
    const uint16_t* __restrict__ W3, const float* __restrict__ b3,
    const float* __restrict__ abar, float* __restrict__ CE, int E, int Nx, int Ny, int Nz,
    unsigned nyn, unsigned nzn, int masked, double* __restrict__ pcr) {
  constexpr int NP = P + 1, n = NP * NP * NP, KR = (n + 15) / 16 * 16, KS = KR / 16,
                NT = NH / 16;
  constexpr int NTH = NT / 2, K3 = (KS + 1) / 2;
  __shared__ bf16x4 sH[2][MLP_TILES][NT][64];
  __shared__ double sred[MLP_THREADS / 64];
  const bf16x4* F1 = reinterpret_cast<const bf16x4*>(W1r);
  const bf16x4* F2 = reinterpret_cast<const bf16x4*>(W2);
  const bf16x4* F3 = reinterpret_cast<const bf16x4*>(W3);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = wave >> 1, h = wave & 1;
  const int le = lane & 15, kq = (lane >> 4) * 4;
  const int e = (blockIdx.x * MLP_TILES + tile) * 16 + le;
  const bool ve = e < E;
  const int ez = ve ? e % Nz : 0, exy = ve ? e / Nz : 0;
  const int ey = exy % Ny, ex = exy / Ny;
  const size_t base = ((size_t)(ex * P) * nyn + (size_t)ey * P) * nzn + (size_t)ez * P;
  float rv[KS][4];
  float ss = 0.f;
#pragma unroll
  for (int k = 0; k < KS; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int loc = 16 * k + kq + v;
      rv[k][v] = 0.f;
      if (ve && loc < n) {
        const int i = loc / (NP * NP), m = (loc / NP) % NP, j = loc % NP;
        rv[k][v] = (float)r[base + ((size_t)i * nyn + m) * nzn + j];
      }
      ss += rv[k][v] * rv[k][v];
    }
  ss += __shfl_xor(ss, 16, 64);
  ss += __shfl_xor(ss, 32, 64);
  const float sn = sqrtf(ss);
  const float sinv = sn > 0.f ? 1.0f / sn : 0.f;
  bf16x4 xb[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) xb[k][v] = (short)f2bf(rv[k][v] * sinv);
  double part = 0.0;
  f32x4 acc[NTH];
  bf16x4 hb[NT];
  auto layer1 = [&](auto hc) {
    constexpr int H = decltype(hc)::value;
    layer_mfma<NTH, KS>(F1, NTH * H, lane, xb, acc);
#pragma unroll
    for (int t = 0; t < NTH; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) hb[NTH * H + t][v] = (short)f2bf(gelu(acc[t][v]));
      sH[0][tile][NTH * H + t][lane] = hb[NTH * H + t];
    }
  };
  auto layer2 = [&](auto hc) {
    constexpr int H = decltype(hc)::value;
#pragma unroll
    for (int t = 0; t < NTH; ++t) hb[NTH * (1 - H) + t] = sH[0][tile][NTH * (1 - H) + t][lane];
#pragma unroll
    for (int t = 0; t < NTH; ++t)
      acc[t] = *reinterpret_cast<const f32x4*>(b2 + 16 * (NTH * H + t) + kq);
    layer_mfma<NTH, NT>(F2, NTH * H, lane, hb, acc);
#pragma unroll
    for (int t = 0; t < NTH; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) hb[NTH * H + t][v] = (short)f2bf(gelu(acc[t][v]));
      sH[1][tile][NTH * H + t][lane] = hb[NTH * H + t];
    }
  };
  auto layer3 = [&](auto hc) {
    constexpr int H = decltype(hc)::value;
    constexpr int T0 = K3 * H;
#pragma unroll
    for (int t = 0; t < NTH; ++t) hb[NTH * (1 - H) + t] = sH[1][tile][NTH * (1 - H) + t][lane];
    const float sc = ve ? sn / abar[e] : 0.f;
#pragma unroll
    for (int t = 0; t < K3; ++t) {
      const int t3 = T0 + t;
      if (T0 + t >= KS) break;
      f32x4 c[1] = {*reinterpret_cast<const f32x4*>(b3 + 16 * t3 + kq)};
      layer_mfma<1, NT>(F3, t3, lane, hb, c);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int loc = 16 * t3 + kq + v;
        if (ve && loc < n) {
          const float ce = sc * c[0][v];
          const int i = loc / (NP * NP), m = (loc / NP) % NP, j = loc % NP;
          CE[(size_t)e * n + loc] = ce;
          const double wx = ((i == 0 && ex > 0) || (i == P && ex < Nx - 1)) ? 0.5 : 1.0;
          const double wy = ((m == 0 && ey > 0) || (m == P && ey < Ny - 1)) ? 0.5 : 1.0;
          const double wz = ((j == 0 && ez > 0) || (j == P && ez < Nz - 1)) ? 0.5 : 1.0;
          const bool top = masked && j == P && ez == Nz - 1;
          if (!top) part += (double)ce * (double)rv[t3][v] * (wx * wy * wz);
        }
      }
    }
  };
  using H0 = std::integral_constant<int, 0>;
  using H1 = std::integral_constant<int, 1>;
#pragma unroll
  for (int t = 0; t < NTH; ++t)
    acc[t] = ve ? *reinterpret_cast<const f32x4*>(Z1geo + (long)e * NH + 16 * (NTH * h + t) + kq)
                : (f32x4){0.f, 0.f, 0.f, 0.f};
  if (h == 0) layer1(H0{}); else layer1(H1{});
  __syncthreads();
  if (h == 0) layer2(H0{}); else layer2(H1{});
  __syncthreads();
  if (h == 0) layer3(H0{}); else layer3(H1{});
  part = wsum(part);
  if (lane == 0) sred[wave] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < MLP_THREADS / 64; ++w) tot += sred[w];
    pcr[blockIdx.x] = tot;
  }
}

// c[g] = average of the element-local corrections of the (up to eight) hexahedra holding node
// g, zero on the Dirichlet surface when masked; contributions in a fixed order
template <int P, typename T>
__global__ __launch_bounds__(256) void k_stage_assemble3d(const float* __restrict__ CE,
                                                          T* __restrict__ c, int Nx, int Ny,
                                                          int Nz, unsigned nyn, unsigned nzn,
                                                          size_t N, int masked) {
  constexpr int NP = P + 1, n = NP * NP * NP;
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < N;
       g += (size_t)gridDim.x * blockDim.x) {
    const int iz = (int)(g % nzn);
    const size_t gxy = g / nzn;
    const int iy = (int)(gxy % nyn), ix = (int)(gxy / nyn);
    if (masked && iz == (int)nzn - 1) {
      c[g] = (T)0;
      continue;
    }
    int ex[2], lx[2], ey[2], ly[2], ez[2], lz[2], cx = 0, cy = 0, cz = 0;
    {
      const int q = ix / P, rr = ix - q * P;
      if (rr == 0 && q > 0) { ex[cx] = q - 1; lx[cx++] = P; }
      if (q < Nx) { ex[cx] = q; lx[cx++] = rr; }
    }
    {
      const int q = iy / P, rr = iy - q * P;
      if (rr == 0 && q > 0) { ey[cy] = q - 1; ly[cy++] = P; }
      if (q < Ny) { ey[cy] = q; ly[cy++] = rr; }
    }
    {
      const int q = iz / P, rr = iz - q * P;
      if (rr == 0 && q > 0) { ez[cz] = q - 1; lz[cz++] = P; }
      if (q < Nz) { ez[cz] = q; lz[cz++] = rr; }
    }
    float s = 0.f;
    for (int a = 0; a < cx; ++a)
      for (int b = 0; b < cy; ++b)
        for (int d = 0; d < cz; ++d) {
          const size_t e = ((size_t)ex[a] * Ny + ey[b]) * Nz + ez[d];
          s += CE[e * n + ((size_t)lx[a] * NP + ly[b]) * NP + lz[d]];
        }
    c[g] = (T)(s / (float)(cx * cy * cz));
  }
}

int stage_mlp_blocks(size_t E) { return (int)((E + 16 * MLP_TILES - 1) / (16 * MLP_TILES)); }

hipError_t stage_mlp(const Stage& s, bool dbl, const void* r, int masked, double* pcr,
                     hipStream_t st) {
  {  // r, the geometric half of layer 1, the element scales and the network read; CE written
    const double N = (double)(s.Nx * s.P + 1) * s.nyn * s.nzn, KR = pad16(s.nout);
    semk::acct_add((dbl ? 8.0 : 4.0) * N + 4.0 * s.E * (NH + 1) + 4.0 * s.E * s.nout +
                   2.0 * (NH * KR + NH * NH + KR * NH) + 4.0 * (NH + KR));
  }
  if (s.dim == 3) {
    if (s.P < 1 || s.P > 6 || s.nout != (s.P + 1) * (s.P + 1) * (s.P + 1)) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)stage_mlp_blocks(s.E);
#define SEM_STAGE_MLP3(PP, TT)                                                                   \
  hipLaunchKernelGGL((k_stage_mlp3d<PP, TT>), dim3(blocks), dim3(MLP_THREADS), 0, st,           \
                     (const TT*)r, s.W1r, s.Z1geo, s.W2, s.b2, s.W3, s.b3, s.abar, s.CE,         \
                     (int)s.E, s.Nx, s.Ny, s.Nz, (unsigned)s.nyn, (unsigned)s.nzn, masked, pcr)
#define SEM_STAGE_MLP3_P(PP)             \
  case PP:                               \
    if (dbl) SEM_STAGE_MLP3(PP, double); \
    else SEM_STAGE_MLP3(PP, float);      \
    break;
    switch (s.P) {
      SEM_STAGE_MLP3_P(1)
      SEM_STAGE_MLP3_P(2)
      SEM_STAGE_MLP3_P(3)
      SEM_STAGE_MLP3_P(4)
      SEM_STAGE_MLP3_P(5)
      SEM_STAGE_MLP3_P(6)
      default:
        return hipErrorInvalidValue;
    }
#undef SEM_STAGE_MLP3_P
#undef SEM_STAGE_MLP3
    return hipGetLastError();
  }
  if (s.P < 1 || s.P > 8 || s.nout != (s.P + 1) * (s.P + 1)) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)stage_mlp_blocks(s.E);
#define SEM_STAGE_MLP(PP, TT)                                                                    \
  hipLaunchKernelGGL((k_stage_mlp<PP, TT>), dim3(blocks), dim3(MLP_THREADS), 0, st,             \
                     (const TT*)r, s.W1r, s.Z1geo, s.W2, s.b2, s.W3, s.b3, s.abar, s.CE,         \
                     (int)s.E, s.Nx, s.Nz, (unsigned)s.nzn, masked, pcr)
#define SEM_STAGE_MLP_P(PP)             \
  case PP:                              \
    if (dbl) SEM_STAGE_MLP(PP, double); \
    else SEM_STAGE_MLP(PP, float);      \
    break;
  switch (s.P) {
    SEM_STAGE_MLP_P(1)
    SEM_STAGE_MLP_P(2)
    SEM_STAGE_MLP_P(3)
    SEM_STAGE_MLP_P(4)
    SEM_STAGE_MLP_P(5)
    SEM_STAGE_MLP_P(6)
    SEM_STAGE_MLP_P(7)
    SEM_STAGE_MLP_P(8)
    default:
      return hipErrorInvalidValue;
  }
#undef SEM_STAGE_MLP_P
#undef SEM_STAGE_MLP
  return hipGetLastError();
}

// c[g] = average of the element-local corrections of the elements holding node g (the weight
// W = (sum R R^T)^-1), zero on the Dirichlet surface when masked.  Contributions are added in a
// fixed order: (left, lower), (left, upper), (right, lower), (right, upper) element.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_stage_assemble(const float* __restrict__ CE,
                                                        T* __restrict__ c, int Nx, int Nz,
                                                        unsigned nzn, unsigned N, int masked) {
  constexpr int NP = P + 1, n = NP * NP;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    const int ix = g / nzn, iz = g - ix * nzn;
    if (masked && iz == (int)nzn - 1) {
      c[g] = (T)0;
      continue;
    }
    const int qx = ix / P, rx = ix - qx * P, qz = iz / P, rz = iz - qz * P;
    const bool xl = rx == 0 && qx > 0, xr = qx < Nx, zl = rz == 0 && qz > 0, zr = qz < Nz;
    float s = 0.f;
    int cnt = 0;
    if (xl && zl) { s += CE[semk::ce_index(qx - 1, P, qz - 1, P, Nz, NP)]; ++cnt; }
    if (xl && zr) { s += CE[semk::ce_index(qx - 1, P, qz, rz, Nz, NP)]; ++cnt; }
    if (xr && zl) { s += CE[semk::ce_index(qx, rx, qz - 1, P, Nz, NP)]; ++cnt; }
    if (xr && zr) { s += CE[semk::ce_index(qx, rx, qz, rz, Nz, NP)]; ++cnt; }
    c[g] = (T)(s / (float)cnt);
  }
}

hipError_t stage_assemble(const Stage& s, bool dbl, void* c, int masked, hipStream_t st) {
  semk::acct_add(4.0 * s.E * s.nout + (dbl ? 8.0 : 4.0) * (double)(s.Nx * s.P + 1) * s.nyn * s.nzn);
  if (s.dim == 3) {
    const size_t N = (size_t)(s.Nx * s.P + 1) * s.nyn * s.nzn;
    const unsigned blocks = (unsigned)std::min<size_t>(nblk(N, 256), 16384);
#define SEM_STAGE_ASM3(PP, TT)                                                                    \
  hipLaunchKernelGGL((k_stage_assemble3d<PP, TT>), dim3(blocks), dim3(256), 0, st, s.CE, (TT*)c, \
                     s.Nx, s.Ny, s.Nz, (unsigned)s.nyn, (unsigned)s.nzn, N, masked)
    switch (s.P) {
#define SEM_STAGE_ASM3_P(PP) \
  case PP:                   \
    if (dbl) SEM_STAGE_ASM3(PP, double); else SEM_STAGE_ASM3(PP, float); \
    break;
      SEM_STAGE_ASM3_P(1)
      SEM_STAGE_ASM3_P(2)
      SEM_STAGE_ASM3_P(3)
      SEM_STAGE_ASM3_P(4)
      SEM_STAGE_ASM3_P(5)
      SEM_STAGE_ASM3_P(6)
      default:
        return hipErrorInvalidValue;
    }
#undef SEM_STAGE_ASM3_P
#undef SEM_STAGE_ASM3
    return hipGetLastError();
  }
  const unsigned N = (unsigned)((size_t)(s.Nx * s.P + 1) * s.nzn);
  const unsigned blocks = std::min(nblk(N, 256), 8192u);
#define SEM_STAGE_ASM(PP, TT)                                                                   \
  hipLaunchKernelGGL((k_stage_assemble<PP, TT>), dim3(blocks), dim3(256), 0, st, s.CE, (TT*)c, \
                     s.Nx, s.Nz, (unsigned)s.nzn, N, masked)
#define SEM_STAGE_ASM_P(PP)              \
  case PP:                               \
    if (dbl) SEM_STAGE_ASM(PP, double);  \
    else SEM_STAGE_ASM(PP, float);       \
    break;
  switch (s.P) {
    SEM_STAGE_ASM_P(1)
    SEM_STAGE_ASM_P(2)
    SEM_STAGE_ASM_P(3)
    SEM_STAGE_ASM_P(4)
    SEM_STAGE_ASM_P(5)
    SEM_STAGE_ASM_P(6)
    SEM_STAGE_ASM_P(7)
    SEM_STAGE_ASM_P(8)
    default:
      return hipErrorInvalidValue;
  }
#undef SEM_STAGE_ASM_P
#undef SEM_STAGE_ASM
  return hipGetLastError();
}

// Step of the stage: alpha = c.r / c.q from the block partials of the network kernel (c.r) and of
// the apply of c (c.q), added in block order by every block (the same value everywhere,
// independent of scheduling).  Accepted if finite and positive (the A-norm of the error then
// drops by (c.r)^2 / c.q): x += alpha c and R = r - alpha q in place (R holds r on entry);
// otherwise R stays r and the rejection is counted.  Each thread first loads r, q and c of its
// first UPD_IT nodes, so that the loads are in flight during the reduction.
constexpr int UPD_IT = 4;
constexpr int UPD_THREADS = 256;  // small blocks: the step length's block reduction is short

template <typename T>
__global__ __launch_bounds__(1024) void k_stage_update(T* __restrict__ x, T* __restrict__ R,
                                                       const T* __restrict__ c,
                                                       const T* __restrict__ yq, const T* __restrict__ Sq,
                                                       const double* __restrict__ pcr, int ncr,
                                                       const double* __restrict__ pcq, int ncq,
                                                       int* skips, unsigned N, unsigned nzn, unsigned P,
                                                       const T* __restrict__ dinv, T* __restrict__ d,
                                                       T sr, int store_d) {
  __shared__ double sh[16];
  const unsigned stride = gridDim.x * blockDim.x;
  const unsigned g0 = blockIdx.x * blockDim.x + threadIdx.x;
  T rr[UPD_IT], qq[UPD_IT], cc[UPD_IT], xx[UPD_IT], di[UPD_IT];
#pragma unroll
  for (int k = 0; k < UPD_IT; ++k) {
    const unsigned g = g0 + k * stride;
    if (g < N) {
      rr[k] = R[g];
      qq[k] = ax_at(yq, Sq, g, nzn, P);
      cc[k] = c[g];
      xx[k] = x[g];
      di[k] = dinv ? dinv[g] : (T)0;
    }
  }
  double a0 = 0.0, a1 = 0.0;
  for (int k = threadIdx.x; k < ncr; k += blockDim.x) a0 += pcr[k];
  for (int k = threadIdx.x; k < ncq; k += blockDim.x) a1 += pcq[k];
  const double cr = bsum(a0, sh);
  const double cq = bsum(a1, sh);
  const double alpha = cr / cq;
  const bool ok = isfinite(alpha) && alpha > 0.0;
  const T al = ok ? (T)alpha : (T)0;
  // node g: x += alpha c, R = r - alpha q (accepted step); then, with dinv, the first smoothing
  // step from that residual: dn = sr dinv R, d = dn (store_d), x += dn
  auto node = [&](unsigned g, T r, T q, T cv, T xv, T dg) {
    if (ok) {
      xv += al * cv;
      r = r - al * q;
      R[g] = r;
    }
    if (dinv) {
      const T dn = sr * dg * r;
      if (store_d) d[g] = dn;
      xv += dn;
    }
    if (ok || dinv) x[g] = xv;
  };
#pragma unroll
  for (int k = 0; k < UPD_IT; ++k) {
    const unsigned g = g0 + k * stride;
    if (g < N) node(g, rr[k], qq[k], cc[k], xx[k], di[k]);
  }
  for (unsigned g = g0 + UPD_IT * stride; g < N; g += stride)
    node(g, R[g], ax_at(yq, Sq, g, nzn, P), c[g], x[g], dinv ? dinv[g] : (T)0);
  if (blockIdx.x == 0 && threadIdx.x == 0 && !ok) skips[0] += 1;
}

hipError_t stage_update(bool dbl, void* x, void* R, const void* c, const void* yq, const void* Sq,
                        const double* pcr, int ncr, const double* pcq, int ncq, int* skips,
                        unsigned N, unsigned nzn, unsigned P, const void* dinv, void* d,
                        double sr, int store_d, hipStream_t st) {
  semk::acct_add((dbl ? 8.0 : 4.0) * N * (6 + (dinv ? 1 : 0) + (store_d ? 1 : 0)));
  const unsigned blocks = nblk(N, UPD_THREADS * UPD_IT);
  if (dbl)
    hipLaunchKernelGGL(k_stage_update<double>, dim3(blocks), dim3(UPD_THREADS), 0, st, (double*)x,
                       (double*)R, (const double*)c, (const double*)yq, (const double*)Sq, pcr,
                       ncr, pcq, ncq, skips, N, nzn, P, (const double*)dinv, (double*)d, sr,
                       store_d);
  else
    hipLaunchKernelGGL(k_stage_update<float>, dim3(blocks), dim3(UPD_THREADS), 0, st, (float*)x,
                       (float*)R, (const float*)c, (const float*)yq, (const float*)Sq, pcr, ncr,
                       pcq, ncq, skips, N, nzn, P, (const float*)dinv, (float*)d, (float)sr,
                       store_d);
  return hipGetLastError();
}

// training features: one block per element.  Targets: (a_e/s_e) R_e e for a given error e, or
// (a_e/s_e) Ainv_e R_e r with the element-block inverse Ainv_e when e is null
__global__ __launch_bounds__(128) void k_features(const double* __restrict__ r,
                                                  const double* __restrict__ e,
                                                  const double* __restrict__ Ainv,
                                                  const float* __restrict__ geo,
                                                  const float* __restrict__ abar, float* __restrict__ X,
                                                  float* __restrict__ Tt, int P, int Nz, int nzn,
                                                  const int* __restrict__ elist) {
  __shared__ double sh[8];
  const int orow = blockIdx.x;                     // output row
  const int el = elist ? elist[orow] : orow;       // element it describes
  const int NP = P + 1, n = NP * NP;
  const int ex = el / Nz, ez = el - ex * Nz;
  double s2 = 0.0;
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const int i = l / NP, j = l - i * NP;
    const double v = r[(size_t)(ex * P + i) * nzn + ez * P + j];
    s2 += v * v;
  }
  const double s = sqrt(bsum(s2, sh));
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const int i = l / NP, j = l - i * NP;
    const size_t g = (size_t)(ex * P + i) * nzn + ez * P + j;
    X[(size_t)orow * 5 * n + l] = s > 0 ? (float)(r[g] / s) : 0.f;
    if (Tt && e) Tt[(size_t)orow * n + l] = s > 0 ? (float)((double)abar[el] / s * e[g]) : 0.f;
    if (Tt && !e) {
      double t = 0.0;
      const double* row = Ainv + ((size_t)el * n + l) * n;
      for (int q = 0; q < n; ++q) {
        const int qi = q / NP, qj = q - qi * NP;
        t += row[q] * r[(size_t)(ex * P + qi) * nzn + ez * P + qj];
      }
      Tt[(size_t)orow * n + l] = s > 0 ? (float)((double)abar[el] / s * t) : 0.f;
    }
  }
  for (int l = threadIdx.x; l < 4 * n; l += blockDim.x)
    X[(size_t)orow * 5 * n + n + l] = geo[(size_t)el * 4 * n + l];
}

// the same rows for hexahedra (element e = (ex Ny + ey) Nz + ez, local node (i NP + m) NP + j;
// X [rows x 7n]: r_e / s_e, then the 6n geometric features of geo)
__global__ __launch_bounds__(128) void k_features3d(const double* __restrict__ r,
                                                    const double* __restrict__ e,
                                                    const double* __restrict__ Ainv,
                                                    const float* __restrict__ geo,
                                                    const float* __restrict__ abar,
                                                    float* __restrict__ X, float* __restrict__ Tt,
                                                    int P, int Ny, int Nz, int nyn, int nzn,
                                                    const int* __restrict__ elist) {
  __shared__ double sh[8];
  const int orow = blockIdx.x;
  const int el = elist ? elist[orow] : orow;
  const int NP = P + 1, n = NP * NP * NP;
  const int ez = el % Nz, exy = el / Nz, ey = exy % Ny, ex = exy / Ny;
  auto gnode = [&](int l) {
    const int i = l / (NP * NP), m = (l / NP) % NP, j = l % NP;
    return ((size_t)(ex * P + i) * nyn + (size_t)(ey * P + m)) * nzn + ez * P + j;
  };
  double s2 = 0.0;
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const double v = r[gnode(l)];
    s2 += v * v;
  }
  const double s = sqrt(bsum(s2, sh));
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const size_t g = gnode(l);
    X[(size_t)orow * 7 * n + l] = s > 0 ? (float)(r[g] / s) : 0.f;
    if (Tt && e) Tt[(size_t)orow * n + l] = s > 0 ? (float)((double)abar[el] / s * e[g]) : 0.f;
    if (Tt && !e) {
      double t = 0.0;
      const double* arow = Ainv + ((size_t)el * n + l) * n;
      for (int q = 0; q < n; ++q) t += arow[q] * r[gnode(q)];
      Tt[(size_t)orow * n + l] = s > 0 ? (float)((double)abar[el] / s * t) : 0.f;
    }
  }
  for (int l = threadIdx.x; l < 6 * n; l += blockDim.x)
    X[(size_t)orow * 7 * n + n + l] = geo[(size_t)el * 6 * n + l];
}

hipError_t features3d(const double* r, const double* e, const double* Ainv, const float* geo,
                      const float* abar, float* X, float* T, size_t E, int P, int Ny, int Nz,
                      int nyn, int nzn, hipStream_t st, const int* elist, size_t nrows) {
  const size_t rows = elist ? nrows : E;
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features3d, dim3((unsigned)rows), dim3(128), 0, st, r, e, Ainv, geo, abar,
                     X, T, P, Ny, Nz, nyn, nzn, elist);
  return hipGetLastError();
}

hipError_t features(const double* r, const double* e, const double* Ainv, const float* geo,
                    const float* abar, float* X, float* T, size_t E, int P, int Nz, int nzn,
                    hipStream_t st, const int* elist, size_t nrows) {
  const size_t rows = elist ? nrows : E;
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)rows), dim3(128), 0, st, r, e, Ainv, geo, abar, X,
                     T, P, Nz, nzn, elist);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// batched forward without any device allocation: the network and one chunk of activations live
// in a file-scope device array (one copy per GPU, alive until the process ends)
// ------------------------------------------------------------------------------------------
namespace {

constexpr int NA_ROWS = 256;                  // rows per chunk
constexpr int NA_K1 = 416, NA_N3 = 96;        // padded input / output widths at the limits
constexpr size_t NA_BODY = (size_t)NA_K1 * NH + NH + (size_t)NH * NH + NH + (size_t)NH * NA_N3 + NA_N3;

constexpr size_t na_align(size_t b) { return (b + 255) / 256 * 256; }
// byte offsets of the regions of the array
constexpr size_t NA_OFF_BODY = 0;                                               // fp32 parameters
constexpr size_t NA_OFF_W1B = NA_OFF_BODY + na_align(NA_BODY * 4);              // bf16 [K1][NH]
constexpr size_t NA_OFF_W2B = NA_OFF_W1B + na_align((size_t)NA_K1 * NH * 2);    // bf16 [NH][NH]
constexpr size_t NA_OFF_W3B = NA_OFF_W2B + na_align((size_t)NH * NH * 2);       // bf16 [NH][N3]
constexpr size_t NA_OFF_IDX = NA_OFF_W3B + na_align((size_t)NH * NA_N3 * 2);    // int [K1 >= rows]
constexpr size_t NA_OFF_XB = NA_OFF_IDX + na_align((size_t)NA_K1 * 4);          // bf16 [rows][K1]
constexpr size_t NA_OFF_Z1 = NA_OFF_XB + na_align((size_t)NA_ROWS * NA_K1 * 2); // fp32 [rows][NH]
constexpr size_t NA_OFF_Z2 = NA_OFF_Z1 + na_align((size_t)NA_ROWS * NH * 4);
constexpr size_t NA_OFF_H1 = NA_OFF_Z2 + na_align((size_t)NA_ROWS * NH * 4);    // bf16 [rows][NH]
constexpr size_t NA_OFF_H2 = NA_OFF_H1 + na_align((size_t)NA_ROWS * NH * 2);
constexpr size_t NA_OFF_Y = NA_OFF_H2 + na_align((size_t)NA_ROWS * NH * 2);     // fp32 [rows][N3]
constexpr size_t NA_BYTES = NA_OFF_Y + na_align((size_t)NA_ROWS * NA_N3 * 4);
static_assert(NA_K1 >= NA_ROWS, "the row-index region also holds the K1 rows of W1");

// every byte a launch reads is written earlier in the same call, so nothing needs clearing
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int NA_MAX_DEV = 64;
std::mutex na_mu;
void* na_ptr[NA_MAX_DEV] = {nullptr};

// device address of this GPU's copy of the array (looked up once per device)
bool na_scratch(unsigned char** out, std::string& err) {
  int dev = 0;
  CK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NA_MAX_DEV) { err = "device index out of range"; return false; }
  std::lock_guard<std::mutex> g(na_mu);
  if (!na_ptr[dev]) {
    void* p = nullptr;
    CK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) { err = "no device address for the scratch array"; return false; }
    na_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(na_ptr[dev]);
  return true;
}

// idx[r] = r < nv ? first + r : -1 for r < M (r < nv rows of the chunk, the rest padding)
__global__ void k_chunk_rows(int* __restrict__ idx, int first, int nv, int M) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < M) idx[r] = r < nv ? first + r : -1;
}

}  // namespace

size_t forward_noalloc_bytes() { return NA_BYTES; }

bool forward_noalloc(const void* blob, size_t nbytes, const float* X, int n, float* Y,
                     std::string& err) {
  if (!blob || nbytes < sizeof(BlobHeader)) { err = "bad blob (too small)"; return false; }
  BlobHeader h;
  std::memcpy(&h, blob, sizeof h);
  if (h.magic != kMagic || h.version != 1 || h.nh != (uint32_t)NH) { err = "bad blob (not a network)"; return false; }
  if (h.nin < 1 || h.nout < 1 || pad16((int)h.nin) > NA_K1 || pad16((int)h.nout) > NA_N3) {
    err = "bad sizes: the allocation-free forward takes nin <= 416 and nout <= 96";
    return false;
  }
  if (nbytes != blob_size(h.nin, h.nout)) { err = "bad blob (size mismatch)"; return false; }
  if (!X || !Y || n < 1) { err = "bad arguments"; return false; }
  unsigned char* base = nullptr;
  if (!na_scratch(&base, err)) return false;
  const hipStream_t st = nullptr;
  Params p;
  p.nin = (int)h.nin;
  p.nout = (int)h.nout;
  p.K1 = pad16(p.nin);
  p.N3 = pad16(p.nout);
  float* body = reinterpret_cast<float*>(base + NA_OFF_BODY);
  // the blob's parameters as they are (unpadded): W1 [nin][NH], b1, W2, b2, W3 [NH][nout], b3
  p.W1 = body;
  p.b1 = p.W1 + (size_t)p.nin * NH;
  p.W2 = p.b1 + NH;
  p.b2 = p.W2 + (size_t)NH * NH;
  p.W3 = p.b2 + NH;
  p.b3 = p.W3 + (size_t)NH * p.nout;
  p.W1b = reinterpret_cast<uint16_t*>(base + NA_OFF_W1B);
  p.W2b = reinterpret_cast<uint16_t*>(base + NA_OFF_W2B);
  p.W3b = reinterpret_cast<uint16_t*>(base + NA_OFF_W3B);
  Acts a{};
  a.Bmax = NA_ROWS;
  a.K1 = p.K1;
  a.N3 = p.N3;
  a.idx = reinterpret_cast<int*>(base + NA_OFF_IDX);
  a.Xb = reinterpret_cast<uint16_t*>(base + NA_OFF_XB);
  a.Z1 = reinterpret_cast<float*>(base + NA_OFF_Z1);
  a.Z2 = reinterpret_cast<float*>(base + NA_OFF_Z2);
  a.H1b = reinterpret_cast<uint16_t*>(base + NA_OFF_H1);
  a.H2b = reinterpret_cast<uint16_t*>(base + NA_OFF_H2);
  a.Y = reinterpret_cast<float*>(base + NA_OFF_Y);
  const size_t np = (size_t)p.nin * NH + NH + (size_t)NH * NH + NH + (size_t)NH * p.nout + p.nout;
  CK(hipMemcpy(body, (const char*)blob + sizeof h, np * sizeof(float), hipMemcpyHostToDevice));
  // bf16 copies, zero-padded: W1 rows nin .. K1 - 1 through idx = -1, W3 columns nout .. N3 - 1
  hipLaunchKernelGGL(k_chunk_rows, dim3(nblk(p.K1, 256)), dim3(256), 0, st, a.idx, 0, p.nin,
                     p.K1);
  CK(hipGetLastError());
  CK(to_bf16_padded(p.W1, p.K1, NH, NH, p.W1b, NH, NH, a.idx, st));
  CK(to_bf16_padded(p.W2, NH, NH, NH, p.W2b, NH, NH, nullptr, st));
  CK(to_bf16_padded(p.W3, NH, p.nout, p.nout, p.W3b, p.N3, p.N3, nullptr, st));
  for (int s0 = 0; s0 < n; s0 += NA_ROWS) {
    const int nv = std::min(NA_ROWS, n - s0);
    const int M = (nv + 15) / 16 * 16;
    hipLaunchKernelGGL(k_chunk_rows, dim3(nblk(M, 256)), dim3(256), 0, st, a.idx, s0, nv, M);
    CK(hipGetLastError());
    if (!fwd(p, a, X, M, st, err)) return false;
    hipLaunchKernelGGL(k_out_bias, dim3(nblk((size_t)nv * p.nout, 256)), dim3(256), 0, st, a.Y,
                       p.N3, p.b3, nv, p.nout, Y + (size_t)s0 * p.nout);
    CK(hipGetLastError());
  }
  CK(hipStreamSynchronize(st));
  return true;
}

}  // namespace semm
