// gfx950 operator of the 3D levels of order P = 1 (the last p-level and the h-levels below it,
// paper Sec. 5.1) as an assembled 27-point stencil.  At P = 1 every node lies on planes shared
// by element columns, so the matrix-free column operator finishes nothing by itself and needs
// its face fix-up pass over all nodes; the assembled stencil (built at set-up from the same
// element matrices, Dirichlet rows and columns masked) gives each node its row in one pass.
// Coefficients are stored offset-major, coef[k N + g] for offset k = (dx+1) 9 + (dy+1) 3 + (dz+1),
// so consecutive nodes read consecutive addresses.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace semk {

namespace {

template <typename T>
__global__ __launch_bounds__(64) void k_stencil3d(const T* __restrict__ x, T* __restrict__ y,
                                                  const T* __restrict__ coef, unsigned nxn,
                                                  unsigned nyn, unsigned nzn, unsigned N,
                                                  Step3 st3, T* __restrict__ xo) {
  // one wave per 64 nodes; neighbours outside the grid have zero coefficients, so their index
  // is clamped into the grid instead of branched around, and all 54 loads issue back to back
  for (unsigned g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    const unsigned iz = g % nzn, ixy = g / nzn;
    const unsigned iy = ixy % nyn, ix = ixy / nyn;
    const int xs[3] = {ix > 0 ? -(int)(nyn * nzn) : 0, 0, ix + 1 < nxn ? (int)(nyn * nzn) : 0};
    const int ys[3] = {iy > 0 ? -(int)nzn : 0, 0, iy + 1 < nyn ? (int)nzn : 0};
    const int zs[3] = {iz > 0 ? -1 : 0, 0, iz + 1 < nzn ? 1 : 0};
    // every load first (54 independent requests in flight), then the sum in offset order
    T cv[27], xv[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) cv[k] = coef[(size_t)k * N + g];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int q = 0; q < 3; ++q)
          xv[a * 9 + b * 3 + q] = x[(size_t)((int)g + xs[a] + ys[b] + zs[q])];
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 27; ++k) acc += cv[k] * xv[k];
    if (!st3.b) {
      y[g] = acc;
      continue;
    }
    T* d = static_cast<T*>(st3.d);
    const T r = static_cast<const T*>(st3.b)[g] - acc;
    T dn = (T)st3.cr * static_cast<const T*>(st3.dinv)[g] * r;
    if (st3.cd != 0.0) dn += (T)st3.cd * d[g];
    if (st3.store_d) d[g] = dn;
    xo[g] = x[g] + dn;
  }
}

}  // namespace

hipError_t stencil3d(bool dbl, const void* x, void* y, const void* coef, unsigned nxn,
                     unsigned nyn, unsigned nzn, hipStream_t st, Step3 st3, void* xo) {
  const size_t N = (size_t)nxn * nyn * nzn;
  if (N == 0 || N >= (1ull << 31)) return hipErrorInvalidValue;
  if (st3.b && (!xo || xo == x)) return hipErrorInvalidValue;
  {
    const double vs = dbl ? 8.0 : 4.0;
    const double nv = st3.b ? 4 + (st3.cd != 0.0) + (st3.store_d ? 1 : 0) : 2;
    acct_add(vs * N * (27 + nv));
  }
  const unsigned blocks = (unsigned)std::min<size_t>((N + 63) / 64, 32768);
  if (dbl)
    hipLaunchKernelGGL(k_stencil3d<double>, dim3(blocks), dim3(64), 0, st, (const double*)x,
                       (double*)y, (const double*)coef, nxn, nyn, nzn, (unsigned)N, st3,
                       (double*)xo);
  else
    hipLaunchKernelGGL(k_stencil3d<float>, dim3(blocks), dim3(64), 0, st, (const float*)x,
                       (float*)y, (const float*)coef, nxn, nyn, nzn, (unsigned)N, st3,
                       (float*)xo);
  return hipGetLastError();
}

}  // namespace semk
