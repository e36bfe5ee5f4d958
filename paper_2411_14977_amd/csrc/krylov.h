// Vector kernels of the GMRES outer iteration (FP64, deterministic two-stage reductions over
// semk::NRED workgroups): the Arnoldi step's operator result, classical Gram-Schmidt against
// the basis (applied twice) and the solution update.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace semk {

constexpr int KRY_MAX = 64;  // longest restart cycle
struct KryCoef {
  double h[KRY_MAX];
};

// w = (A z) from the column output y and side buffer S (S null: y complete; nzn nodes per
// vertical line, order P), then part[i NRED + block] = block partial of w . V_i, i < nv, with
// V_i = V + i ldv.  N nodes.
hipError_t kry_first(const double* y, const double* S, double* w, const double* V, size_t ldv,
                     int nv, double* part, unsigned N, unsigned nzn, unsigned P, hipStream_t st);
// w -= sum_{i < nv} h_i V_i; then (dots) partials of w . V_i (i < nv) into part[i NRED + .],
// and always of w . w into part[nv NRED + .]
hipError_t kry_sub(double* w, const double* V, size_t ldv, int nv, const KryCoef& h, int dots,
                   double* part, unsigned N, hipStream_t st);
// the same with the coefficients h_i read from device memory (hd[0 .. nv)), so that the host
// need not see them between the steps of one Arnoldi step
hipError_t kry_sub_dev(double* w, const double* V, size_t ldv, int nv, const double* hd, int dots,
                       double* part, unsigned N, hipStream_t st);
// out[s] = the sum of the NRED partials of set s (s < nsets), in a fixed order
hipError_t kry_sums(const double* part, int nsets, double* out, hipStream_t st);
// Arnoldi step end: hn = sqrt(*ww); w *= 1 / hn (hn > 0); column j of the Hessenberg matrix,
// col[i] = h1[i] + h2[i] (i <= j), col[j + 1] = hn
hipError_t kry_finish(double* w, const double* ww, const double* h1, const double* h2, int j,
                      double* col, unsigned N, hipStream_t st);
// w *= s
hipError_t kry_scale(double* w, double s, unsigned N, hipStream_t st);
// x += sum_{i < k} y_i Z_i
hipError_t kry_update(double* x, const double* Z, size_t ldz, int k, const KryCoef& y,
                      unsigned N, hipStream_t st);

}  // namespace semk
