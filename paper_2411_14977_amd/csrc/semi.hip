// gfx950 operator kernel for 2D elements whose GLL orders differ along x (PX) and sigma (PZ):
// the semi-coarsened levels of the p-multigrid hierarchy (paper Sec. 5.1) and meshes built
// with different orders in the two directions.
//
// The element stiffness is the same sum-factorised form as the equal-order kernel's,
// A_e u = D_r^T (G_rr D_r u + G_rs D_s u) + D_s^T (G_rs D_r u + G_ss D_s u), with D_r = D_x (x) I
// and D_s = I (x) D_z.  One workgroup owns one vertical column of Nz elements and one thread
// one element-local node (i, j); the column's nodal values, the two differentiation matrices
// and the intermediate fluxes sit in LDS.  The output format is the equal-order kernel's: the
// column's lines 0..PX-1 to y, its line PX to the side buffer S of the right neighbour (to y
// for the last column), so every consumer of (y, S) works unchanged with P = PX.  The orders
// are run-time values: these levels are small next to the equal-order ones (the semi-coarsened
// hierarchy returns to equal orders after one or two levels), so one kernel serves all pairs.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "kernels.h"

namespace semk {

namespace {

template <typename T, typename TG>
__device__ __forceinline__ T gval(const TG* p);
template <>
__device__ __forceinline__ double gval<double, double>(const double* p) { return *p; }
template <>
__device__ __forceinline__ float gval<float, float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float gval<float, uint16_t>(const uint16_t* p) {
  return __uint_as_float(((uint32_t)(*p)) << 16);
}

// LDS of one column, in T elements: D_x, D_z, the column input [NPX][nzn], the fluxes w_r and
// w_s of every node, and the top-face values of each element [Nz][NPX]
inline size_t rect_lds_elems(int PX, int PZ, int Nz) {
  const size_t NPX = PX + 1, NPZ = PZ + 1, nzn = (size_t)Nz * PZ + 1, nthr = NPX * NPZ * Nz;
  return NPX * NPX + NPZ * NPZ + NPX * nzn + 2 * nthr + (size_t)Nz * NPX;
}

// nf = 3: fields G_rr, G_rs, G_ss (symmetric); nf = 4: G_rr, G_rs, G_ss, G_sr with G_rs pairing
// the test function's r-derivative with the trial function's s-derivative and G_sr the reverse
// (the mixed-stage operator of two stage geometries)
template <typename T, typename TG>
__global__ __launch_bounds__(1024) void k_apply2r(const T* __restrict__ x, T* __restrict__ y,
                                                  T* __restrict__ S, const TG* __restrict__ G,
                                                  const double* __restrict__ Dx,
                                                  const double* __restrict__ Dz, int Nx, int Nz,
                                                  int PX, int PZ, int masked, int nf) {
  const int NPX = PX + 1, NPZ = PZ + 1, nloc = NPX * NPZ, nthr = nloc * Nz;
  const int nzn = Nz * PZ + 1;
  const int ex = blockIdx.x;
  const int t = threadIdx.x;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Dxs = reinterpret_cast<T*>(smem_raw);
  T* Dzs = Dxs + NPX * NPX;
  T* xs = Dzs + NPZ * NPZ;          // [NPX][nzn]
  T* wr = xs + NPX * nzn;           // [nthr]
  T* ws = wr + nthr;                // [nthr]
  T* vtop = ws + nthr;              // [Nz][NPX]
  const T* xc = x + (size_t)ex * PX * nzn;
  for (int k = t; k < NPX * NPX; k += blockDim.x) Dxs[k] = (T)Dx[k];
  for (int k = t; k < NPZ * NPZ; k += blockDim.x) Dzs[k] = (T)Dz[k];
  for (int k = t; k < NPX * nzn; k += blockDim.x) {
    const int li = k / nzn, iz = k - li * nzn;
    // the Dirichlet surface enters the element products as zero
    xs[k] = (masked && iz == nzn - 1) ? (T)0 : xc[(size_t)li * nzn + iz];
  }
  __syncthreads();
  const bool act = t < nthr;
  const int ez = t / nloc, l = t - ez * nloc, i = l / NPZ, j = l - i * NPZ;
  const int iz0 = ez * PZ;
  if (act) {
    T ur = 0, us = 0;
    for (int k = 0; k < NPX; ++k) ur += Dxs[i * NPX + k] * xs[k * nzn + iz0 + j];
    for (int k = 0; k < NPZ; ++k) us += Dzs[j * NPZ + k] * xs[i * nzn + iz0 + k];
    const TG* Gc = G + (size_t)ex * nf * nthr + t;
    const T g0 = gval<T, TG>(Gc), g1 = gval<T, TG>(Gc + nthr), g2 = gval<T, TG>(Gc + 2 * nthr);
    const T g3 = nf == 4 ? gval<T, TG>(Gc + 3 * nthr) : g1;
    wr[t] = g0 * ur + g1 * us;
    ws[t] = g3 * ur + g2 * us;
  }
  __syncthreads();
  T v = 0;
  if (act) {
    const int eb = ez * nloc;
    for (int k = 0; k < NPX; ++k) v += Dxs[k * NPX + i] * wr[eb + k * NPZ + j];
    for (int k = 0; k < NPZ; ++k) v += Dzs[k * NPZ + j] * ws[eb + i * NPZ + k];
    if (j == PZ) vtop[ez * NPX + i] = v;
  }
  __syncthreads();
  // node (line i, iz) of the column: the element below's top value joins the bottom node of
  // every element above the first; the top node of the top element is written by it
  if (act && (j < PZ || ez == Nz - 1)) {
    if (j == 0 && ez > 0) v += vtop[(ez - 1) * NPX + i];
    const int iz = iz0 + j;
    const bool top = iz == nzn - 1;
    if (masked && top) v = xc[(size_t)i * nzn + iz];  // identity row of the Dirichlet node
    if (i < PX || ex == Nx - 1) y[((size_t)ex * PX + i) * nzn + iz] = v;
    else S[(size_t)(ex + 1) * nzn + iz] = (masked && top) ? (T)0 : v;
  }
}

template <typename T, typename TG>
hipError_t launch(const void* x, void* y, void* S, const void* G, const double* Dx,
                  const double* Dz, int Nx, int Nz, int PX, int PZ, int masked, int nf,
                  hipStream_t st) {
  const int nthr = (PX + 1) * (PZ + 1) * Nz;
  const int block = (nthr + 63) / 64 * 64;
  const size_t smem = rect_lds_elems(PX, PZ, Nz) * sizeof(T);
  if (block > 1024 || smem > 65536) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_apply2r<T, TG>), dim3(Nx), dim3(block), smem, st, (const T*)x, (T*)y,
                     (T*)S, (const TG*)G, Dx, Dz, Nx, Nz, PX, PZ, masked, nf);
  return hipGetLastError();
}

}  // namespace

bool apply2r_fits(int PX, int PZ, int Nz, bool dbl) {
  return (PX + 1) * (PZ + 1) * Nz <= 1024 &&
         rect_lds_elems(PX, PZ, Nz) * (dbl ? 8 : 4) <= 65536;
}

hipError_t apply2r(int PX, int PZ, bool dbl, GType gt, const void* x, void* y, void* S,
                   const void* G, const double* Dx, const double* Dz, int Nx, int Nz, int masked,
                   hipStream_t st, int nf) {
  if (nf != 3 && nf != 4) return hipErrorInvalidValue;
  const double vs = dbl ? 8.0 : 4.0, gs = gt == G_F64 ? 8.0 : (gt == G_F32 ? 4.0 : 2.0);
  const double nodes = (double)(Nx * PX + 1) * (Nz * PZ + 1);
  // x read, y written (the shared lines once more into S), factors read once
  acct_add(vs * nodes * 2.0 + vs * (double)(Nx - 1) * (Nz * PZ + 1) +
           gs * nf * Nx * Nz * (PX + 1) * (PZ + 1));
  if (dbl) {
    if (gt != G_F64) return hipErrorInvalidValue;
    return launch<double, double>(x, y, S, G, Dx, Dz, Nx, Nz, PX, PZ, masked, nf, st);
  }
  if (gt == G_F32)
    return launch<float, float>(x, y, S, G, Dx, Dz, Nx, Nz, PX, PZ, masked, nf, st);
  if (gt == G_BF16)
    return launch<float, uint16_t>(x, y, S, G, Dx, Dz, Nx, Nz, PX, PZ, masked, nf, st);
  return hipErrorInvalidValue;
}

}  // namespace semk
