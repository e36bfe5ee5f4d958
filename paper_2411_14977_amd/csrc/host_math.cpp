// Host FP64 set-up math.  See host_math.h.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace semh {

// Classical Legendre P_n(x) and P_{n-1}(x) by the three-term recurrence
// n P_n = (2n-1) x P_{n-1} - (n-1) P_{n-2}.
static void legendre_pair(int n, double x, double& pn, double& pnm1) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { pn = 1.0; pnm1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pnm1 = p0;
}

void gll_rule(int P, std::vector<double>& r, std::vector<double>& w) {
  const int n = P + 1;
  r.assign(n, 0.0);
  w.assign(n, 0.0);
  // Newton on f(x) = x P_P(x) - P_{P-1}(x), which vanishes exactly at the GLL points
  // (it equals -(1-x^2) P_P'(x) / P); f'(x) = (P+1) P_P(x).  Start from Chebyshev-Lobatto
  // points, which interlace the GLL points.
  for (int k = 0; k < n; ++k) {
    double x = -std::cos(M_PI * k / P);
    if (k == 0 || k == P) { r[k] = x; continue; }
    for (int it = 0; it < 100; ++it) {
      double pn, pnm1;
      legendre_pair(P, x, pn, pnm1);
      double dx = (x * pn - pnm1) / ((P + 1) * pn);
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    r[k] = x;
  }
  r[0] = -1.0;
  r[P] = 1.0;
  for (int k = 0; k <= P / 2; ++k) {  // exact symmetry
    double a = 0.5 * (r[P - k] - r[k]);
    r[k] = -a;
    r[P - k] = a;
  }
  if (P % 2 == 0) r[P / 2] = 0.0;
  for (int k = 0; k < n; ++k) {
    double pn, pnm1;
    legendre_pair(P, r[k], pn, pnm1);
    w[k] = 2.0 / (P * (P + 1.0) * pn * pn);
  }
}

std::vector<double> diff_matrix(int P, const std::vector<double>& r) {
  // Closed form of the Lagrange derivative at GLL points:
  // D_ik = P_P(r_i) / (P_P(r_k) (r_i - r_k)) for i != k; D_00 = -P(P+1)/4, D_PP = +P(P+1)/4.
  const int n = P + 1;
  std::vector<double> D(n * n, 0.0), L(n);
  for (int i = 0; i < n; ++i) {
    double pn, pnm1;
    legendre_pair(P, r[i], pn, pnm1);
    L[i] = pn;
  }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k)
      if (i != k) D[i * n + k] = L[i] / (L[k] * (r[i] - r[k]));
  if (P >= 1) {
    D[0] = -P * (P + 1.0) / 4.0;
    D[n * n - 1] = P * (P + 1.0) / 4.0;
  }
  return D;
}

std::vector<double> interp_matrix(const std::vector<double>& rs, const std::vector<double>& rt) {
  const int ns = (int)rs.size(), nt = (int)rt.size();
  std::vector<double> bw(ns, 1.0);  // barycentric weights
  for (int k = 0; k < ns; ++k)
    for (int m = 0; m < ns; ++m)
      if (m != k) bw[k] /= (rs[k] - rs[m]);
  std::vector<double> M(nt * ns, 0.0);
  for (int a = 0; a < nt; ++a) {
    int hit = -1;
    for (int k = 0; k < ns; ++k)
      if (rt[a] == rs[k]) hit = k;
    if (hit >= 0) { M[a * ns + hit] = 1.0; continue; }
    double den = 0.0;
    for (int k = 0; k < ns; ++k) den += bw[k] / (rt[a] - rs[k]);
    for (int k = 0; k < ns; ++k) M[a * ns + k] = (bw[k] / (rt[a] - rs[k])) / den;
  }
  return M;
}

double bf16_round(double v) {
  float f = (float)v;
  uint16_t b = bf16_bits(f);
  uint32_t u = (uint32_t)b << 16;
  float g;
  std::memcpy(&g, &u, 4);
  return (double)g;
}

uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;  // round to nearest even
  return (uint16_t)(u >> 16);
}

double splitmix64_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

// --------------------------------------------------------------------------------------------
void build_level(LevelGeom& L, int dim, int Nx, int Ny, int Nz, int P, int Pf, double Lx,
                 double Ly, const double* hf, const double* ef, int Pz) {
  if (Pz < 1 || dim == 3) Pz = P;
  L.dim = dim;
  L.P = P;
  L.NP = P + 1;
  L.Pz = Pz;
  L.NPz = Pz + 1;
  L.Nx = Nx;
  L.Ny = dim == 3 ? Ny : 1;
  L.Nz = Nz;
  L.Lx = Lx;
  L.Ly = Ly;
  const int NP = P + 1;
  gll_rule(P, L.r, L.w);
  L.D = diff_matrix(P, L.r);
  if (Pz == P) {
    L.rz = L.r;
    L.wz = L.w;
    L.Dz = L.D;
  } else {
    gll_rule(Pz, L.rz, L.wz);
    L.Dz = diff_matrix(Pz, L.rz);
  }
  std::vector<double> rf, wf;
  gll_rule(Pf, rf, wf);
  std::vector<double> I = interp_matrix(rf, L.r);  // (NP) x (Pf+1)
  L.nxn = Nx * P + 1;
  L.nyn = dim == 3 ? Ny * P + 1 : 1;
  L.nzn = Nz * Pz + 1;
  L.N = (size_t)L.nxn * L.nyn * L.nzn;
  const double dx = Lx / Nx, dsig = 1.0 / Nz;
  const std::vector<double>& D = L.D;
  const std::vector<double>& w = L.w;
  if (dim == 2) {
    const int NPz = Pz + 1;
    const std::vector<double>& rz = L.rz;
    const std::vector<double>& wz = L.wz;
    L.E = (size_t)Nx * Nz;
    L.nfields = 3;
    const size_t NL = (size_t)NP * NPz;
    L.G.assign(3 * L.E * NL, 0.0);
    L.mass.assign(L.E * NL, 0.0);
    L.X.assign(L.N, 0.0);
    L.Z.assign(L.N, 0.0);
    L.col_h.assign((size_t)Nx * NP, 0.0);
    L.col_eta.assign((size_t)Nx * NP, 0.0);
    std::vector<double> h(NP), et(NP), d(NP), hx(NP), dxd(NP);
    for (int ex = 0; ex < Nx; ++ex) {
      for (int i = 0; i < NP; ++i) {
        double sh = 0, se = 0;
        for (int k = 0; k <= Pf; ++k) {
          sh += I[i * (Pf + 1) + k] * hf[ex * Pf + k];
          se += I[i * (Pf + 1) + k] * ef[ex * Pf + k];
        }
        h[i] = sh;
        et[i] = se;
        d[i] = sh + se;
        L.col_h[ex * NP + i] = sh;
        L.col_eta[ex * NP + i] = se;
      }
      for (int i = 0; i < NP; ++i) {
        double a = 0, b = 0;
        for (int k = 0; k < NP; ++k) {
          a += D[i * NP + k] * h[k];
          b += D[i * NP + k] * d[k];
        }
        hx[i] = 2.0 / dx * a;
        dxd[i] = 2.0 / dx * b;
      }
      for (int ez = 0; ez < Nz; ++ez) {
        const size_t e = (size_t)ex * Nz + ez;
        for (int i = 0; i < NP; ++i)
          for (int j = 0; j < NPz; ++j) {
            const double sig = (ez + (rz[j] + 1.0) / 2.0) / Nz;
            const double sx = (hx[i] - sig * dxd[i]) / d[i];
            const double ww = w[i] * wz[j];
            const size_t l = e * NL + i * NPz + j;
            L.G[0 * L.E * NL + l] = ww * d[i] * dsig / dx;
            L.G[1 * L.E * NL + l] = ww * d[i] * sx;
            L.G[2 * L.E * NL + l] = ww * (dx / dsig) * d[i] * (sx * sx + 1.0 / (d[i] * d[i]));
            L.mass[l] = ww * d[i] * dx * dsig / 4.0;
            const size_t g = (size_t)(ex * P + i) * L.nzn + ez * Pz + j;
            L.X[g] = Lx * (ex + (L.r[i] + 1.0) / 2.0) / Nx;
            L.Z[g] = -h[i] + sig * d[i];
          }
      }
    }
    // Neumann faces: x = 0, x = Lx, bottom
    L.face_idx.assign(3, {});
    L.face_w.assign(3, {});
    for (int f = 0; f < 2; ++f) {
      const int ex = f == 0 ? 0 : Nx - 1, i = f == 0 ? 0 : P;
      const double dd = L.col_h[ex * NP + i] + L.col_eta[ex * NP + i];
      L.face_idx[f].assign(L.nzn, 0);
      L.face_w[f].assign(L.nzn, 0.0);
      for (int ez = 0; ez < Nz; ++ez)
        for (int j = 0; j < NPz; ++j) {
          const int iz = ez * Pz + j;
          L.face_idx[f][iz] = (int64_t)(ex * P + i) * L.nzn + iz;
          L.face_w[f][iz] += wz[j] * dd * dsig / 2.0;
        }
    }
    L.face_idx[2].assign(L.nxn, 0);
    L.face_w[2].assign(L.nxn, 0.0);
    for (int ex = 0; ex < Nx; ++ex) {
      for (int i = 0; i < NP; ++i) {
        double a = 0;
        for (int k = 0; k < NP; ++k) a += D[i * NP + k] * L.col_h[ex * NP + k];
        const double hxi = 2.0 / dx * a;
        const int ix = ex * P + i;
        L.face_idx[2][ix] = (int64_t)ix * L.nzn;
        L.face_w[2][ix] += w[i] * (dx / 2.0) * std::sqrt(1.0 + hxi * hxi);
      }
    }
    return;
  }
  // ---------------- 3D ----------------
  const double dy = Ly / Ny;
  L.E = (size_t)Nx * Ny * Nz;
  L.nfields = 5;
  const size_t NL = (size_t)NP * NP * NP;
  L.G.assign(5 * L.E * NL, 0.0);
  L.mass.assign(L.E * NL, 0.0);
  L.X.assign(L.N, 0.0);
  L.Y.assign(L.N, 0.0);
  L.Z.assign(L.N, 0.0);
  const int nyf = Ny * Pf + 1;
  L.col_h.assign((size_t)Nx * Ny * NP * NP, 0.0);
  L.col_eta.assign((size_t)Nx * Ny * NP * NP, 0.0);
  std::vector<double> tmp(NP * (Pf + 1));
  std::vector<double> h(NP * NP), et(NP * NP), d(NP * NP), hx(NP * NP), hy(NP * NP),
      dxd(NP * NP), dyd(NP * NP);
  for (int ex = 0; ex < Nx; ++ex)
    for (int ey = 0; ey < Ny; ++ey) {
      for (int fld = 0; fld < 2; ++fld) {
        const double* src = fld == 0 ? hf : ef;
        double* dst = fld == 0 ? h.data() : et.data();
        // interpolate along x then y
        for (int i = 0; i < NP; ++i)
          for (int b = 0; b <= Pf; ++b) {
            double s = 0;
            for (int a = 0; a <= Pf; ++a)
              s += I[i * (Pf + 1) + a] * src[(size_t)(ex * Pf + a) * nyf + ey * Pf + b];
            tmp[i * (Pf + 1) + b] = s;
          }
        for (int i = 0; i < NP; ++i)
          for (int m = 0; m < NP; ++m) {
            double s = 0;
            for (int b = 0; b <= Pf; ++b) s += I[m * (Pf + 1) + b] * tmp[i * (Pf + 1) + b];
            dst[i * NP + m] = s;
          }
      }
      for (int q = 0; q < NP * NP; ++q) {
        d[q] = h[q] + et[q];
        L.col_h[((size_t)ex * Ny + ey) * NP * NP + q] = h[q];
        L.col_eta[((size_t)ex * Ny + ey) * NP * NP + q] = et[q];
      }
      for (int i = 0; i < NP; ++i)
        for (int m = 0; m < NP; ++m) {
          double a = 0, b = 0, c = 0, e2 = 0;
          for (int k = 0; k < NP; ++k) {
            a += D[i * NP + k] * h[k * NP + m];
            b += D[i * NP + k] * d[k * NP + m];
            c += D[m * NP + k] * h[i * NP + k];
            e2 += D[m * NP + k] * d[i * NP + k];
          }
          hx[i * NP + m] = 2.0 / dx * a;
          dxd[i * NP + m] = 2.0 / dx * b;
          hy[i * NP + m] = 2.0 / dy * c;
          dyd[i * NP + m] = 2.0 / dy * e2;
        }
      for (int ez = 0; ez < Nz; ++ez) {
        const size_t e = ((size_t)ex * Ny + ey) * Nz + ez;
        for (int i = 0; i < NP; ++i)
          for (int m = 0; m < NP; ++m)
            for (int j = 0; j < NP; ++j) {
              const int q = i * NP + m;
              const double sig = (ez + (L.r[j] + 1.0) / 2.0) / Nz;
              const double sx = (hx[q] - sig * dxd[q]) / d[q];
              const double sy = (hy[q] - sig * dyd[q]) / d[q];
              const double www = w[i] * w[m] * w[j];
              const double jac = (dx / 2.0) * (dy / 2.0) * (d[q] * dsig / 2.0);
              const double wj = www * jac;
              const double rx = 2.0 / dx, ty = 2.0 / dy, ss = 2.0 / dsig;
              const size_t l = e * NL + (size_t)(i * NP + m) * NP + j;
              L.G[0 * L.E * NL + l] = wj * rx * rx;
              L.G[1 * L.E * NL + l] = wj * ty * ty;
              L.G[2 * L.E * NL + l] = wj * rx * ss * sx;
              L.G[3 * L.E * NL + l] = wj * ty * ss * sy;
              L.G[4 * L.E * NL + l] = wj * ss * ss * (sx * sx + sy * sy + 1.0 / (d[q] * d[q]));
              L.mass[l] = www * (dx * dy * dsig / 8.0) * d[q];
              const size_t g = ((size_t)(ex * P + i) * L.nyn + ey * P + m) * L.nzn + ez * P + j;
              L.X[g] = Lx * (ex + (L.r[i] + 1.0) / 2.0) / Nx;
              L.Y[g] = Ly * (ey + (L.r[m] + 1.0) / 2.0) / Ny;
              L.Z[g] = -h[q] + sig * d[q];
            }
      }
    }
  // faces: x=0, x=Lx [(nyn)(nzn)], y=0, y=Ly [(nxn)(nzn)], bottom [(nxn)(nyn)]
  L.face_idx.assign(5, {});
  L.face_w.assign(5, {});
  for (int f = 0; f < 2; ++f) {
    const int ex = f == 0 ? 0 : Nx - 1, i = f == 0 ? 0 : P;
    L.face_idx[f].assign((size_t)L.nyn * L.nzn, 0);
    L.face_w[f].assign((size_t)L.nyn * L.nzn, 0.0);
    for (int ey = 0; ey < Ny; ++ey)
      for (int m = 0; m < NP; ++m) {
        const double dd = L.col_h[((size_t)ex * Ny + ey) * NP * NP + i * NP + m] +
                          L.col_eta[((size_t)ex * Ny + ey) * NP * NP + i * NP + m];
        for (int ez = 0; ez < Nz; ++ez)
          for (int j = 0; j < NP; ++j) {
            const int iy = ey * P + m, iz = ez * P + j;
            const size_t k = (size_t)iy * L.nzn + iz;
            L.face_idx[f][k] = ((int64_t)(ex * P + i) * L.nyn + iy) * L.nzn + iz;
            L.face_w[f][k] += w[m] * w[j] * (dy / 2.0) * dd * dsig / 2.0;
          }
      }
  }
  for (int f = 0; f < 2; ++f) {
    const int ey = f == 0 ? 0 : Ny - 1, m = f == 0 ? 0 : P;
    L.face_idx[2 + f].assign((size_t)L.nxn * L.nzn, 0);
    L.face_w[2 + f].assign((size_t)L.nxn * L.nzn, 0.0);
    for (int ex = 0; ex < Nx; ++ex)
      for (int i = 0; i < NP; ++i) {
        const double dd = L.col_h[((size_t)ex * Ny + ey) * NP * NP + i * NP + m] +
                          L.col_eta[((size_t)ex * Ny + ey) * NP * NP + i * NP + m];
        for (int ez = 0; ez < Nz; ++ez)
          for (int j = 0; j < NP; ++j) {
            const int ix = ex * P + i, iz = ez * P + j;
            const size_t k = (size_t)ix * L.nzn + iz;
            L.face_idx[2 + f][k] = ((int64_t)ix * L.nyn + ey * P + m) * L.nzn + iz;
            L.face_w[2 + f][k] += w[i] * w[j] * (dx / 2.0) * dd * dsig / 2.0;
          }
      }
  }
  L.face_idx[4].assign((size_t)L.nxn * L.nyn, 0);
  L.face_w[4].assign((size_t)L.nxn * L.nyn, 0.0);
  for (int ex = 0; ex < Nx; ++ex)
    for (int ey = 0; ey < Ny; ++ey) {
      const double* hc = &L.col_h[((size_t)ex * Ny + ey) * NP * NP];
      for (int i = 0; i < NP; ++i)
        for (int m = 0; m < NP; ++m) {
          double a = 0, b = 0;
          for (int k = 0; k < NP; ++k) {
            a += D[i * NP + k] * hc[k * NP + m];
            b += D[m * NP + k] * hc[i * NP + k];
          }
          const double hx1 = 2.0 / dx * a, hy1 = 2.0 / dy * b;
          const int ix = ex * P + i, iy = ey * P + m;
          const size_t k = (size_t)ix * L.nyn + iy;
          L.face_idx[4][k] = ((int64_t)ix * L.nyn + iy) * L.nzn;
          L.face_w[4][k] += w[i] * w[m] * (dx / 2.0) * (dy / 2.0) *
                            std::sqrt(1.0 + hx1 * hx1 + hy1 * hy1);
        }
    }
}

// --------------------------------------------------------------------------------------------
size_t local_to_global(const LevelGeom& L, size_t e, int l) {
  const int NP = L.NP, P = L.P;
  if (L.dim == 2) {
    const size_t ex = e / L.Nz, ez = e % L.Nz;
    const int i = l / L.NPz, j = l % L.NPz;
    return (ex * P + i) * (size_t)L.nzn + ez * L.Pz + j;
  }
  const size_t ez = e % L.Nz, ey = (e / L.Nz) % L.Ny, ex = e / ((size_t)L.Nz * L.Ny);
  const int j = l % NP, m = (l / NP) % NP, i = l / (NP * NP);
  return ((ex * P + i) * (size_t)L.nyn + ey * P + m) * L.nzn + ez * P + j;
}

static inline bool is_top(const LevelGeom& L, size_t g) { return (g % L.nzn) == (size_t)(L.nzn - 1); }

std::vector<double> assembled_diag(const LevelGeom& L, const std::vector<double>& Gr, bool masked) {
  std::vector<double> diag(L.N, 0.0);
  const int NP = L.NP, NPz = L.NPz;
  const size_t NL = L.dim == 2 ? (size_t)NP * NPz : (size_t)NP * NP * NP;
  const double* D = L.D.data();
  const double* Dz = L.Dz.data();
  for (size_t e = 0; e < L.E; ++e) {
    for (size_t l = 0; l < NL; ++l) {
      double s = 0;
      if (L.dim == 2) {
        const int i = l / NPz, j = l % NPz;
        const double* Grr = &Gr[0 * L.E * NL + e * NL];
        const double* Grs = &Gr[1 * L.E * NL + e * NL];
        const double* Gss = &Gr[2 * L.E * NL + e * NL];
        for (int k = 0; k < NP; ++k) s += D[k * NP + i] * D[k * NP + i] * Grr[k * NPz + j];
        s += 2.0 * D[i * NP + i] * Dz[j * NPz + j] * Grs[i * NPz + j];
        for (int k = 0; k < NPz; ++k) s += Dz[k * NPz + j] * Dz[k * NPz + j] * Gss[i * NPz + k];
      } else {
        const int j = l % NP, m = (l / NP) % NP, i = l / (NP * NP);
        auto G = [&](int f, int a, int b, int c) {
          return Gr[f * L.E * NL + e * NL + ((size_t)a * NP + b) * NP + c];
        };
        for (int k = 0; k < NP; ++k) s += D[k * NP + i] * D[k * NP + i] * G(0, k, m, j);
        for (int k = 0; k < NP; ++k) s += D[k * NP + m] * D[k * NP + m] * G(1, i, k, j);
        for (int k = 0; k < NP; ++k) s += D[k * NP + j] * D[k * NP + j] * G(4, i, m, k);
        s += 2.0 * D[i * NP + i] * D[j * NP + j] * G(2, i, m, j);
        s += 2.0 * D[m * NP + m] * D[j * NP + j] * G(3, i, m, j);
      }
      diag[local_to_global(L, e, (int)l)] += s;
    }
  }
  if (masked)
    for (size_t g = 0; g < L.N; ++g)
      if (is_top(L, g)) diag[g] = 1.0;
  return diag;
}

void element_matrix(const LevelGeom& L, const std::vector<double>& Gr, size_t e, double* Ae) {
  // A_e = sum_q sum_{a,b} G_ab(q) (D_a phi)(q) (D_b phi)(q), quadrature at the GLL nodes.
  const int NP = L.NP, NPz = L.NPz;
  const int dim = L.dim;
  const size_t NL = dim == 2 ? (size_t)NP * NPz : (size_t)NP * NP * NP;
  const double* D = L.D.data();
  const double* Ds = dim == 2 ? L.Dz.data() : D;  // sigma direction
  const int NS = dim == 2 ? NPz : NP;
  std::fill(Ae, Ae + NL * NL, 0.0);
  std::vector<double> gr(NL * 3);
  for (size_t q = 0; q < NL; ++q) {
    int qi, qm, qj;
    if (dim == 2) { qi = q / NPz; qm = 0; qj = q % NPz; }
    else { qj = q % NP; qm = (q / NP) % NP; qi = q / (NP * NP); }
    double Gq[3][3] = {{0}};
    if (dim == 2) {
      Gq[0][0] = Gr[0 * L.E * NL + e * NL + q];
      Gq[0][2] = Gq[2][0] = Gr[1 * L.E * NL + e * NL + q];
      Gq[2][2] = Gr[2 * L.E * NL + e * NL + q];
    } else {
      Gq[0][0] = Gr[0 * L.E * NL + e * NL + q];
      Gq[1][1] = Gr[1 * L.E * NL + e * NL + q];
      Gq[0][2] = Gq[2][0] = Gr[2 * L.E * NL + e * NL + q];
      Gq[1][2] = Gq[2][1] = Gr[3 * L.E * NL + e * NL + q];
      Gq[2][2] = Gr[4 * L.E * NL + e * NL + q];
    }
    // reference gradients of every basis function at q (axis 0 = r, 1 = t, 2 = s)
    for (size_t a = 0; a < NL; ++a) {
      int ai, am, aj;
      if (dim == 2) { ai = a / NPz; am = 0; aj = a % NPz; }
      else { aj = a % NP; am = (a / NP) % NP; ai = a / (NP * NP); }
      gr[a * 3 + 0] = (am == qm && aj == qj) ? D[qi * NP + ai] : 0.0;
      gr[a * 3 + 1] = (dim == 3 && ai == qi && aj == qj) ? D[qm * NP + am] : 0.0;
      gr[a * 3 + 2] = (ai == qi && am == qm) ? Ds[qj * NS + aj] : 0.0;
    }
    for (size_t a = 0; a < NL; ++a) {
      const double* ga = &gr[a * 3];
      if (ga[0] == 0.0 && ga[1] == 0.0 && ga[2] == 0.0) continue;
      for (size_t b = 0; b < NL; ++b) {
        const double* gb = &gr[b * 3];
        double s = 0;
        for (int u = 0; u < 3; ++u)
          for (int v = 0; v < 3; ++v) s += ga[u] * Gq[u][v] * gb[v];
        Ae[a * NL + b] += s;
      }
    }
  }
}

// ---- dense helpers ----------------------------------------------------------------------
static bool dense_inverse(int n, const double* A, double* Ainv) {
  std::vector<double> M(A, A + (size_t)n * n);
  for (int i = 0; i < n * n; ++i) Ainv[i] = 0.0;
  for (int i = 0; i < n; ++i) Ainv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
    if (M[piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(M[c * n + k], M[piv * n + k]);
        std::swap(Ainv[c * n + k], Ainv[piv * n + k]);
      }
    const double inv = 1.0 / M[c * n + c];
    for (int k = 0; k < n; ++k) {
      M[c * n + k] *= inv;
      Ainv[c * n + k] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = M[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        M[r * n + k] -= f * M[c * n + k];
        Ainv[r * n + k] -= f * Ainv[c * n + k];
      }
    }
  }
  return true;
}

bool dense_inverse_public(int n, const double* A, double* Ainv) { return dense_inverse(n, A, Ainv); }

static void matmul(int n, const double* A, const double* B, double* C) {  // C = A B
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
      C[i * n + j] = s;
    }
}

bool build_bcr(const LevelGeom& L, const std::vector<double>& Gr, BcrPlan& plan, char* err,
               size_t errlen, int dense_max) {
  // Blocks = x-lines (ix).  Free rows of a block: all (iy, iz) with iz < Nz P.
  const int nb = L.dim == 2 ? (L.nzn - 1) : L.nyn * (L.nzn - 1);
  const int nblocks = L.nxn;
  plan.nb = nb;
  plan.nblocks = nblocks;
  plan.bstride = L.nyn * L.nzn;
  plan.rowmap.resize(nb);
  for (int r = 0; r < nb; ++r) {
    const int iy = r / (L.nzn - 1), iz = r % (L.nzn - 1);
    plan.rowmap[r] = iy * L.nzn + iz;
  }
  // assemble block tridiagonal: Dg[b], Lg[b] (coupling b -> b-1), Ug[b] (b -> b+1)
  const size_t nn = (size_t)nb * nb;
  std::vector<double> Dg(nblocks * nn, 0.0), Lg(nblocks * nn, 0.0), Ug(nblocks * nn, 0.0);
  const size_t NL = L.dim == 2 ? L.NP * L.NP : (size_t)L.NP * L.NP * L.NP;
  std::vector<double> Ae(NL * NL);
  for (size_t e = 0; e < L.E; ++e) {
    element_matrix(L, Gr, e, Ae.data());
    for (size_t a = 0; a < NL; ++a) {
      const size_t ga = local_to_global(L, e, (int)a);
      if (is_top(L, ga)) continue;
      const int ba = (int)(ga / plan.bstride);
      const int ra_off = (int)(ga % plan.bstride);
      const int ra = (ra_off / L.nzn) * (L.nzn - 1) + ra_off % L.nzn;
      for (size_t b = 0; b < NL; ++b) {
        const size_t gb = local_to_global(L, e, (int)b);
        if (is_top(L, gb)) continue;
        const int bb = (int)(gb / plan.bstride);
        const int rb_off = (int)(gb % plan.bstride);
        const int rb = (rb_off / L.nzn) * (L.nzn - 1) + rb_off % L.nzn;
        const double v = Ae[a * NL + b];
        if (bb == ba) Dg[ba * nn + ra * nb + rb] += v;
        else if (bb == ba - 1) Lg[ba * nn + ra * nb + rb] += v;
        else if (bb == ba + 1) Ug[ba * nn + ra * nb + rb] += v;
        else {
          snprintf(err, errlen, "coarse operator is not block tridiagonal");
          return false;
        }
      }
    }
  }
  plan.levs.clear();
  plan.fwd.clear();
  plan.bwd.clear();
  int n = nblocks, stride = 1;
  std::vector<double> Dinv(nn), T1(nn), T2(nn);
  while (n > dense_max) {
    BcrPlan::Lev lv;
    lv.n = n;
    lv.stride = stride;
    lv.neven = (n + 1) / 2;
    lv.nodd = n / 2;
    lv.offM = plan.fwd.size();
    lv.offB = plan.bwd.size();
    std::vector<double> Dinvs(n * nn, 0.0);
    for (int k = 1; k < n; k += 2) {
      if (!dense_inverse(nb, &Dg[k * nn], &Dinvs[k * nn])) {
        snprintf(err, errlen, "singular block in coarse reduction");
        return false;
      }
    }
    plan.fwd.resize(plan.fwd.size() + (size_t)lv.neven * 2 * nn, 0.0);
    plan.bwd.resize(plan.bwd.size() + (size_t)lv.nodd * 3 * nn, 0.0);
    double* F = &plan.fwd[lv.offM];
    double* B = &plan.bwd[lv.offB];
    for (int k = 1; k < n; k += 2) {
      const int kk = k / 2;
      double* DO = B + (size_t)kk * 3 * nn;
      std::copy(&Dinvs[k * nn], &Dinvs[k * nn] + nn, DO);
      matmul(nb, &Dinvs[k * nn], &Lg[k * nn], DO + nn);
      if (k + 1 < n) matmul(nb, &Dinvs[k * nn], &Ug[k * nn], DO + 2 * nn);
    }
    const int nn2 = lv.neven;
    std::vector<double> Dn(nn2 * nn, 0.0), Ln(nn2 * nn, 0.0), Un(nn2 * nn, 0.0);
    for (int k = 0; k < n; k += 2) {
      const int kk = k / 2;
      double* Mm = F + (size_t)kk * 2 * nn;
      double* Mp = Mm + nn;
      std::copy(&Dg[k * nn], &Dg[k * nn] + nn, &Dn[kk * nn]);
      if (k > 0) {
        matmul(nb, &Lg[k * nn], &Dinvs[(k - 1) * nn], Mm);          // L_k D_{k-1}^-1
        matmul(nb, Mm, &Ug[(k - 1) * nn], T1.data());               // .. U_{k-1}
        for (size_t q = 0; q < nn; ++q) Dn[kk * nn + q] -= T1[q];
        if (k - 1 > 0) {
          matmul(nb, Mm, &Lg[(k - 1) * nn], T2.data());
          for (size_t q = 0; q < nn; ++q) Ln[kk * nn + q] = -T2[q];
        }
      }
      if (k + 1 < n) {
        matmul(nb, &Ug[k * nn], &Dinvs[(k + 1) * nn], Mp);          // U_k D_{k+1}^-1
        matmul(nb, Mp, &Lg[(k + 1) * nn], T1.data());               // .. L_{k+1}
        for (size_t q = 0; q < nn; ++q) Dn[kk * nn + q] -= T1[q];
        if (k + 2 < n) {
          matmul(nb, Mp, &Ug[(k + 1) * nn], T2.data());
          for (size_t q = 0; q < nn; ++q) Un[kk * nn + q] = -T2[q];
        }
      }
    }
    // the kernels read the factors column by column (entry (r, c) at c nb + r)
    auto transpose_all = [&](double* M, size_t count) {
      for (size_t m = 0; m < count; ++m) {
        double* A = M + m * nn;
        for (int r = 0; r < nb; ++r)
          for (int q = r + 1; q < nb; ++q) std::swap(A[r * nb + q], A[q * nb + r]);
      }
    };
    transpose_all(F, (size_t)lv.neven * 2);
    transpose_all(B, (size_t)lv.nodd * 3);
    plan.levs.push_back(lv);
    Dg.swap(Dn);
    Lg.swap(Ln);
    Ug.swap(Un);
    n = nn2;
    stride *= 2;
  }
  // explicit inverse of the remaining block tridiagonal system (n blocks)
  const int nd = n * nb;
  std::vector<double> Ad((size_t)nd * nd, 0.0);
  for (int k = 0; k < n; ++k)
    for (int r = 0; r < nb; ++r)
      for (int q = 0; q < nb; ++q) {
        Ad[(size_t)(k * nb + r) * nd + k * nb + q] = Dg[k * nn + r * nb + q];
        if (k > 0) Ad[(size_t)(k * nb + r) * nd + (k - 1) * nb + q] = Lg[k * nn + r * nb + q];
        if (k + 1 < n) Ad[(size_t)(k * nb + r) * nd + (k + 1) * nb + q] = Ug[k * nn + r * nb + q];
      }
  plan.dense.assign((size_t)nd * nd, 0.0);
  if (!dense_inverse(nd, Ad.data(), plan.dense.data())) {
    snprintf(err, errlen, "singular reduced coarse system");
    return false;
  }
  plan.dense_n = n;
  plan.dense_stride = stride;
  plan.last.assign(nn, 0.0);
  return true;
}

}  // namespace semh
