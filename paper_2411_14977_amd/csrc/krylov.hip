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
                                                KryCoef h, int dots, double* __restrict__ part,
                                                unsigned N) {
  __shared__ double sh[KT / 64];
  const unsigned stride = gridDim.x * blockDim.x;
  double ww = 0.0;
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += stride) {
    double s = w[g];
    for (int i = 0; i < nv; ++i) s -= h.h[i] * V[(size_t)i * ldv + g];
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
  hipLaunchKernelGGL(k_kry_sub, dim3(NRED), dim3(KT), 0, st, w, V, ldv, nv, h, dots, part, N);
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
