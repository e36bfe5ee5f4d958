// gfx950 kernels of the additive Schwarz smoother (paper Sec. 5.3) over box subdomains: the
// subdomain of an element is its own node index box widened by `ov` node layers on every side
// and clipped to the grid, in 2D (ov >= 1; the element blocks of ov = 0 have their own kernels)
// and in 3D (any ov).  One sweep tail is
//   z_e = (R_e A R_e^T)^{-1} R_e r   for every subdomain e  (dense inverse, built at set-up),
//   x   = (set ? 0 : x) + W sum_e R_e^T z_e,  W = one over the number of boxes holding a node.
// The boxes are computed from (element, order, ov, grid size) in the kernels: no index lists.
// The inverse of subdomain e sits at Ainv + e nmax^2 as its own n_e x n_e matrix (symmetric),
// its result at z + e nmax; box-local node order is x outermost, sigma innermost, as the
// global one.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "kernels.h"

namespace semk {

namespace {

// node range of element k's box along one axis: first node and count
struct Span {
  int lo, len;
};
__device__ __forceinline__ Span span1(int k, int p, int ov, int nn) {
  const int lo = max(0, k * p - ov), hi = min(nn - 1, k * p + p + ov);
  return {lo, hi - lo + 1};
}

// subdomain e's box: spans along x, y (2D: one node), sigma
__device__ __forceinline__ void box_of(const AsmBox& bx, int e, Span* sx, Span* sy, Span* sz) {
  const int ez = e % bx.Nz, exy = e / bx.Nz;
  const int ey = exy % bx.Ny, ex = exy / bx.Ny;
  *sx = span1(ex, bx.P, bx.ov, (int)bx.nxn);
  *sy = span1(ey, bx.P, bx.ov, (int)bx.nyn);
  *sz = span1(ez, bx.P, bx.ov, (int)bx.nzn);
}

// z_e = Ainv_e R_e (r - y): spw subdomains per workgroup, tps threads each (one per row while
// n <= tps); the box's residual is gathered into LDS, the inverse read column by column so that
// consecutive rows read consecutive addresses.  y (optional) is A x, complete at every node.
template <typename T>
__global__ __launch_bounds__(256) void k_asmb_local(const T* __restrict__ r,
                                                    const T* __restrict__ y,
                                                    const T* __restrict__ Ainv,
                                                    T* __restrict__ z, AsmBox bx, int E, int spw,
                                                    int tps) {
  extern __shared__ unsigned char smem_raw[];
  T* sr = reinterpret_cast<T*>(smem_raw);
  const int sl = threadIdx.x / tps, lane = threadIdx.x - sl * tps;
  const int e = blockIdx.x * spw + sl;
  const bool act = sl < spw && e < E;
  Span sx{0, 0}, sy{0, 0}, sz{0, 0};
  if (act) box_of(bx, e, &sx, &sy, &sz);
  const int n = sx.len * sy.len * sz.len;
  T* s = sr + (size_t)(act ? sl : 0) * bx.nmax;
  if (act) {
    const int nyz = sy.len * sz.len;
    for (int q = lane; q < n; q += tps) {
      const int qx = q / nyz, rem = q - qx * nyz;
      const int qy = rem / sz.len, qz = rem - qy * sz.len;
      const size_t g = ((size_t)(sx.lo + qx) * bx.nyn + (sy.lo + qy)) * bx.nzn + (sz.lo + qz);
      s[q] = y ? r[g] - y[g] : r[g];
    }
  }
  __syncthreads();
  if (!act) return;
  const T* Ae = Ainv + (size_t)e * bx.nmax * bx.nmax;
  T* ze = z + (size_t)e * bx.nmax;
  for (int row = lane; row < n; row += tps) {
    T acc = 0;
    const T* a = Ae + row;
#pragma unroll 8
    for (int k = 0; k < n; ++k) acc += a[(size_t)k * n] * s[k];
    ze[row] = acc;
  }
}

// first and last element (along one axis) whose box holds node index g
__device__ __forceinline__ void owners1(int g, int p, int ov, int Ne, int* k0, int* k1) {
  *k0 = g - ov - 1 >= 0 ? (g - ov - 1) / p : 0;
  *k1 = min(Ne - 1, (g + ov) / p);
}

// x = (set ? 0 : x) + the average of the results of the boxes holding each node, in a fixed
// order (x, then y, then sigma element index ascending); the Dirichlet surface keeps x (zeroed
// when set) when masked.
template <typename T>
__global__ __launch_bounds__(256) void k_asmb_add(const T* __restrict__ z, T* __restrict__ x,
                                                  AsmBox bx, size_t N, int masked, int set) {
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < N;
       g += (size_t)gridDim.x * blockDim.x) {
    const int gz = (int)(g % bx.nzn);
    const size_t gxy = g / bx.nzn;
    const int gy = (int)(gxy % bx.nyn), gx = (int)(gxy / bx.nyn);
    if (masked && gz == (int)bx.nzn - 1) {
      if (set) x[g] = (T)0;
      continue;
    }
    int x0, x1, y0, y1, z0, z1;
    owners1(gx, bx.P, bx.ov, bx.Nx, &x0, &x1);
    owners1(gy, bx.P, bx.ov, bx.Ny, &y0, &y1);
    owners1(gz, bx.P, bx.ov, bx.Nz, &z0, &z1);
    T s = 0;
    int cnt = 0;
    for (int kx = x0; kx <= x1; ++kx) {
      const Span sx = span1(kx, bx.P, bx.ov, (int)bx.nxn);
      for (int ky = y0; ky <= y1; ++ky) {
        const Span sy = span1(ky, bx.P, bx.ov, (int)bx.nyn);
        for (int kz = z0; kz <= z1; ++kz) {
          const Span sz = span1(kz, bx.P, bx.ov, (int)bx.nzn);
          const int e = (kx * bx.Ny + ky) * bx.Nz + kz;
          const int loc = ((gx - sx.lo) * sy.len + (gy - sy.lo)) * sz.len + (gz - sz.lo);
          s += z[(size_t)e * bx.nmax + loc];
          ++cnt;
        }
      }
    }
    const T c = s / (T)cnt;
    x[g] = set ? c : x[g] + c;
  }
}

template <typename T>
hipError_t launch_box(const AsmBox& bx, const void* r, const void* y, const void* Ainv, void* z,
                      void* x, int masked, int set, hipStream_t st) {
  const int E = bx.Nx * bx.Ny * bx.Nz;
  const int spw = bx.nmax <= 128 ? 256 / bx.nmax : 1;
  const int tps = spw > 1 ? bx.nmax : 256;
  const size_t lds = (size_t)spw * bx.nmax * sizeof(T);
  const unsigned b1 = (unsigned)((E + spw - 1) / spw);
  hipLaunchKernelGGL(k_asmb_local<T>, dim3(b1), dim3(256), lds, st, (const T*)r, (const T*)y,
                     (const T*)Ainv, (T*)z, bx, E, spw, tps);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const size_t N = (size_t)bx.nxn * bx.nyn * bx.nzn;
  const unsigned b2 = (unsigned)std::min<size_t>((N + 255) / 256, 16384);
  hipLaunchKernelGGL(k_asmb_add<T>, dim3(b2), dim3(256), 0, st, (const T*)z, (T*)x, bx, N,
                     masked, set);
  return hipGetLastError();
}

}  // namespace

hipError_t asm_box_sweep(const AsmBox& bx, bool dbl, const void* r, const void* y,
                         const void* Ainv, void* z, void* x, int masked, int set,
                         hipStream_t st) {
  if (bx.nmax < 1 || bx.nmax > ASM_BOX_NMAX || bx.P < 1 || bx.ov < 0) return hipErrorInvalidValue;
  const double N = (double)bx.nxn * bx.nyn * bx.nzn, vs = dbl ? 8.0 : 4.0;
  acct_add(vs * (bx.ainv_vals + 2.0 * bx.z_vals + N * ((set ? 2 : 3) + (y ? 1 : 0))));
  return dbl ? launch_box<double>(bx, r, y, Ainv, z, x, masked, set, st)
             : launch_box<float>(bx, r, y, Ainv, z, x, masked, set, st);
}

}  // namespace semk
