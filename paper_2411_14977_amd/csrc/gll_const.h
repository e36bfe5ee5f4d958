// Compile-time GLL nodes, weights and differentiation matrix for the device kernels, so that every
// entry of D enters an instruction as a literal operand (no loads, no registers).
//
// Nodes: the P+1 roots of (1 - x^2) L_P'(x) (Gauss-Lobatto-Legendre), found by Newton's method on
// x L_P(x) - L_{P-1}(x), which vanishes exactly at the GLL points, from the Chebyshev-Gauss-
// Lobatto points -cos(pi i / P); then made exactly symmetric, x_{P-i} = -x_i.
// D_ij = l_j'(x_i) in closed form: L_P(x_i) / (L_P(x_j) (x_i - x_j)) for i != j,
// D_00 = -P(P+1)/4, D_PP = P(P+1)/4, zero elsewhere on the diagonal.
// Because the nodes are symmetric, D is centro-antisymmetric, D_{P-i,P-j} = -D_ij, exactly in
// floating point, which the even-odd contraction below relies on.
#pragma once

#include <utility>

namespace semk {
namespace gllc {

constexpr double kPi = 3.14159265358979323846;

constexpr double cos_series(double x) {  // |x| <= pi; only seeds Newton's iteration
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

constexpr void legendre2(int n, double x, double& pn, double& pn1) {  // L_n(x), L_{n-1}(x)
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    pn = 1.0;
    pn1 = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

template <int P>
struct Tab {
  double x[P + 1] = {};
  double w[P + 1] = {};   // GLL weights 2 / (P (P+1) L_P(x_i)^2)
  double D[P + 1][P + 1] = {};
  constexpr Tab() {
    for (int i = 0; i <= P; ++i) {
      double xi = -cos_series(kPi * i / P);
      for (int it = 0; it < 100; ++it) {
        double ln = 0.0, ln1 = 0.0;
        legendre2(P, xi, ln, ln1);
        xi -= (xi * ln - ln1) / ((P + 1.0) * ln);
      }
      x[i] = xi;
    }
    for (int i = 0; i < (P + 1) / 2; ++i) {
      const double a = 0.5 * (x[P - i] - x[i]);
      x[i] = -a;
      x[P - i] = a;
    }
    if (P % 2 == 0) x[P / 2] = 0.0;
    double L[P + 1] = {};
    for (int i = 0; i <= P; ++i) {
      double ln1 = 0.0;
      legendre2(P, x[i], L[i], ln1);
    }
    for (int i = 0; i <= P; ++i) w[i] = 2.0 / (P * (P + 1.0) * L[i] * L[i]);
    for (int i = 0; i <= P; ++i)
      for (int j = 0; j <= P; ++j) D[i][j] = (i == j) ? 0.0 : L[i] / (L[j] * (x[i] - x[j]));
    D[0][0] = -P * (P + 1.0) / 4.0;
    D[P][P] = P * (P + 1.0) / 4.0;
  }
};

template <int P>
inline constexpr Tab<P> tab{};

// M[j][k] with M = D (TR false) or D^T (TR true)
template <int P, bool TR>
constexpr double mat(int j, int k) {
  return TR ? tab<P>.D[k][j] : tab<P>.D[j][k];
}

// compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1
template <typename F, int... I>
__device__ __forceinline__ void sfor_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

}  // namespace gllc

// y = M u along one line of P+1 GLL nodes, M = D or D^T, by the even-odd splitting (Solomonoff,
// "A fast algorithm for spectral differentiation", J. Comput. Phys. 98, 1992): with
// e_k = u_k + u_{P-k}, o_k = u_k - u_{P-k} (k < (P+1)/2) and the centro-antisymmetry of M,
//   y_j = a_j + b_j,  y_{P-j} = b_j - a_j,
//   a_j = sum_k (M_jk + M_j,P-k)/2 e_k (+ M_jm u_m for even P, m = P/2),
//   b_j = sum_k (M_jk - M_j,P-k)/2 o_k,   y_m = sum_k M_mk o_k,
// which halves the multiply count of the direct product.
template <int P, bool TR, typename T>
__device__ __forceinline__ void contract_eo(const T (&u)[P + 1], T (&y)[P + 1]) {
  constexpr int H = (P + 1) / 2;
  constexpr int m = P / 2;
  T e[H], o[H];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    e[k] = u[k] + u[P - k];
    o[k] = u[k] - u[P - k];
  }
  gllc::sfor<H>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    T a = 0, b = 0;
    if constexpr (P % 2 == 0) {
      constexpr T cm = (T)gllc::mat<P, TR>(j, m);
      a = cm * u[m];
    }
    gllc::sfor<H>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr T ep = (T)(0.5 * (gllc::mat<P, TR>(j, k) + gllc::mat<P, TR>(j, P - k)));
      constexpr T op = (T)(0.5 * (gllc::mat<P, TR>(j, k) - gllc::mat<P, TR>(j, P - k)));
      a += ep * e[k];
      b += op * o[k];
    });
    y[j] = a + b;
    y[P - j] = b - a;
  });
  if constexpr (P % 2 == 0) {
    T s = 0;
    gllc::sfor<H>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr T c = (T)gllc::mat<P, TR>(m, k);
      s += c * o[k];
    });
    y[m] = s;
  }
}

}  // namespace semk
