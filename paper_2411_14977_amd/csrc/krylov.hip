// GMRES outer-iteration vector kernels (see krylov.h).
#include "krylov.h"
#include "kernels.h"

namespace semk {

namespace {

constexpr int KT = 256;  // threads per workgroup; NRED workgroups (fixed: deterministic sums)

// fixed-order block sum (wave shuffle tree, then the waves in order); every thread gets it
__device__ double kry_block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < KT / 64; ++k) s += sh[k];
  return s;
}

// (A x)[g] from the column output y and the side buffer S of the next column's first line
__device__ double kry_ax(const double* y, const double* S, unsigned g, unsigned nzn, unsigned P) {
  if (!S) return y[g];
  const unsigned ix = g / nzn, iz = g - ix * nzn;
  double v = y[g];
  const unsigned q = ix / P;
  if (q * P == ix) v += S[q * nzn + iz];
  return v;
}

__global__ __launch_bounds__(KT) void k_kry_first(const double* __restrict__ y,
                                                  const double* __restrict__ S,
                                                  double* __restrict__ w,
                                                  const double* __restrict__ V, size_t ldv,
                                                  int nv, double* __restrict__ part, unsigned N,
                                                  unsigned nzn, unsigned P) {
  __shared__ double sh[KT / 64];
  const unsigned stride = gridDim.x * blockDim.x;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride)
    w[g] = kry_ax(y, S, g, nzn, P);
  for (int i = 0; i < nv; ++i) {
    const double* v = V + (size_t)i * ldv;
    double a = 0.0;
    for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride) a += w[g] * v[g];
    a = kry_block_sum(a, sh);
    if (threadIdx.x == 0) part[(size_t)i * NRED + blockIdx.x] = a;
  }
}

__global__ __launch_bounds__(KT) void k_kry_sub(double* __restrict__ w,
                                                const double* __restrict__ V, size_t ldv, int nv,
                                                KryCoef h, const double* __restrict__ hd,
                                                int dots, double* __restrict__ part,
                                                unsigned N) {
  __shared__ double sh[KT / 64];
  __shared__ double hs[KRY_MAX];
  if (hd) {  // coefficients from device memory
    for (int i = threadIdx.x; i < nv; i += blockDim.x) hs[i] = hd[i];
    __syncthreads();
  }
  const unsigned stride = gridDim.x * blockDim.x;
  double ww = 0.0;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride) {
    double s = w[g];
    for (int i = 0; i < nv; ++i) s -= (hd ? hs[i] : h.h[i]) * V[(size_t)i * ldv + g];
    w[g] = s;
    ww += s * s;
  }
  if (dots) {
    for (int i = 0; i < nv; ++i) {
      const double* v = V + (size_t)i * ldv;
      double a = 0.0;
      for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride)
        a += w[g] * v[g];
      a = kry_block_sum(a, sh);
      if (threadIdx.x == 0) part[(size_t)i * NRED + blockIdx.x] = a;
    }
  }
  ww = kry_block_sum(ww, sh);
  if (threadIdx.x == 0) part[(size_t)nv * NRED + blockIdx.x] = ww;
}

// one workgroup per set: the NRED partials summed in a fixed order (each thread a strided
// run, then the block tree)
__global__ __launch_bounds__(KT) void k_kry_sums(const double* __restrict__ part,
                                                 double* __restrict__ out) {
  __shared__ double sh[KT / 64];
  const double* p = part + (size_t)blockIdx.x * NRED;
  double a = 0.0;
  for (int q = threadIdx.x; q < NRED; q += KT) a += p[q];
  a = kry_block_sum(a, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = a;
}

__global__ __launch_bounds__(KT) void k_kry_finish(double* __restrict__ w,
                                                   const double* __restrict__ ww,
                                                   const double* __restrict__ h1,
                                                   const double* __restrict__ h2, int j,
                                                   double* __restrict__ col, unsigned N) {
  const double hn = sqrt(*ww);
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = h1[i] + h2[i];
    if (threadIdx.x == 0) col[j + 1] = hn;
  }
  if (!(hn > 0.0)) return;
  const double s = 1.0 / hn;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    w[g] *= s;
}

__global__ __launch_bounds__(KT) void k_kry_scale(double* __restrict__ w, double s, unsigned N) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x)
    w[g] *= s;
}

__global__ __launch_bounds__(KT) void k_kry_update(double* __restrict__ x,
                                                   const double* __restrict__ Z, size_t ldz,
                                                   int k, KryCoef y, unsigned N) {
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    double s = x[g];
    for (int i = 0; i < k; ++i) s += y.h[i] * Z[(size_t)i * ldz + g];
    x[g] = s;
  }
}

}  // namespace

hipError_t kry_first(const double* y, const double* S, double* w, const double* V, size_t ldv,
                     int nv, double* part, unsigned N, unsigned nzn, unsigned P, hipStream_t st) {
  acct_add(8.0 * N * (2 + nv));  // y read, w written, each basis vector read
  if (nv < 0 || nv > KRY_MAX + 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_kry_first, dim3(NRED), dim3(KT), 0, st, y, S, w, V, ldv, nv, part, N, nzn,
                     P);
  return hipGetLastError();
}

hipError_t kry_sub(double* w, const double* V, size_t ldv, int nv, const KryCoef& h, int dots,
                   double* part, unsigned N, hipStream_t st) {
  acct_add(8.0 * N * (2 + nv));  // w read and written, each basis vector read
  if (nv < 0 || nv > KRY_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_kry_sub, dim3(NRED), dim3(KT), 0, st, w, V, ldv, nv, h,
                     (const double*)nullptr, dots, part, N);
  return hipGetLastError();
}

hipError_t kry_sub_dev(double* w, const double* V, size_t ldv, int nv, const double* hd, int dots,
                       double* part, unsigned N, hipStream_t st) {
  acct_add(8.0 * N * (2 + nv));
  if (nv < 0 || nv > KRY_MAX || !hd) return hipErrorInvalidValue;
  KryCoef none{};
  hipLaunchKernelGGL(k_kry_sub, dim3(NRED), dim3(KT), 0, st, w, V, ldv, nv, none, hd, dots, part,
                     N);
  return hipGetLastError();
}

hipError_t kry_sums(const double* part, int nsets, double* out, hipStream_t st) {
  if (nsets < 1) return hipSuccess;
  hipLaunchKernelGGL(k_kry_sums, dim3(nsets), dim3(KT), 0, st, part, out);
  return hipGetLastError();
}

hipError_t kry_finish(double* w, const double* ww, const double* h1, const double* h2, int j,
                      double* col, unsigned N, hipStream_t st) {
  acct_add(16.0 * N);
  if (j < 0 || j >= KRY_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_kry_finish, dim3(NRED), dim3(KT), 0, st, w, ww, h1, h2, j, col, N);
  return hipGetLastError();
}

hipError_t kry_scale(double* w, double s, unsigned N, hipStream_t st) {
  acct_add(16.0 * N);
  hipLaunchKernelGGL(k_kry_scale, dim3(NRED), dim3(KT), 0, st, w, s, N);
  return hipGetLastError();
}

hipError_t kry_update(double* x, const double* Z, size_t ldz, int k, const KryCoef& y,
                      unsigned N, hipStream_t st) {
  acct_add(8.0 * N * (2 + k));
  if (k < 0 || k > KRY_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_kry_update, dim3(NRED), dim3(KT), 0, st, x, Z, ldz, k, y, N);
  return hipGetLastError();
}

}  // namespace semk
