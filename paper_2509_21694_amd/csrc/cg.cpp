// Coupling tensors of the tensor-product messages, derived on the host from
// Wigner 3j symbols (Racah's closed form) and the unitary change of basis
// from complex to real spherical harmonics.
//
// For degrees (l1,l2,l3) with natural parity (l1+l2+l3 even, triangle rule)
// the complex Gaunt coefficient is
//   int Y_l1^m1 Y_l2^m2 Y_l3^m3 dOmega
//     = sqrt((2l1+1)(2l2+1)(2l3+1)/(4 pi)) (l1 l2 l3; 0 0 0)(l1 l2 l3; m1 m2 m3).
// Real harmonics (m ordered -l..l) are R_l,m = sum_mu U[m][mu] Y_l^mu with
//   m > 0: U[m][-m] = 1/sqrt2,  U[m][m] = (-1)^m/sqrt2
//   m < 0: U[m][m]  = i/sqrt2,  U[m][-m] = -i(-1)^m/sqrt2
//   m = 0: U[0][0]  = 1
// so the real Gaunt tensor is the three-fold contraction of U with the
// complex one (its imaginary part vanishes).  The tensor used by the kernels
// is that real tensor divided by its Frobenius norm; the overall positive
// normalisation of the harmonics drops out.
#include <cmath>
#include <complex>
#include <vector>

#include "cg.h"

namespace mpip {

static double fact(int n) {
  double r = 1.0;
  for (int k = 2; k <= n; ++k) r *= k;
  return r;
}

double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
  if (m1 + m2 + m3 != 0) return 0.0;
  if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0;
  double tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) / fact(j1 + j2 + j3 + 1);
  double pre = std::sqrt(tri * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) *
                         fact(j3 + m3) * fact(j3 - m3));
  double sum = 0.0;
  for (int k = 0; k <= j1 + j2 + j3; ++k) {
    int a = j3 - j2 + k + m1, b = j3 - j1 + k - m2, c = j1 + j2 - j3 - k, d = j1 - k - m1,
        e = j2 - k + m2;
    if (a < 0 || b < 0 || c < 0 || d < 0 || e < 0) continue;
    double den = fact(k) * fact(a) * fact(b) * fact(c) * fact(d) * fact(e);
    sum += ((k & 1) ? -1.0 : 1.0) / den;
  }
  int ph = j1 - j2 - m3;
  return ((ph % 2 != 0) ? -1.0 : 1.0) * pre * sum;
}

static std::complex<double> U(int l, int m, int mu) {
  const double s = 1.0 / std::sqrt(2.0);
  const std::complex<double> I(0.0, 1.0);
  (void)l;
  if (m == 0) return mu == 0 ? 1.0 : 0.0;
  if (m > 0) {
    if (mu == -m) return s;
    if (mu == m) return ((m & 1) ? -s : s);
    return 0.0;
  }
  int a = -m;  // m < 0
  if (mu == m) return I * s;
  if (mu == a) return -I * ((a & 1) ? -s : s);
  return 0.0;
}

bool natural_path(int l1, int l2, int l3) {
  return ((l1 + l2 + l3) % 2 == 0) && l3 >= std::abs(l1 - l2) && l3 <= l1 + l2;
}

bool coupling_tensor(int l1, int l2, int l3, double* out) {
  if (l1 < 0 || l2 < 0 || l3 < 0 || l1 > 2 || l2 > 2 || l3 > 2) return false;
  if (!natural_path(l1, l2, l3)) return false;
  const int n1 = 2 * l1 + 1, n2 = 2 * l2 + 1, n3 = 2 * l3 + 1;
  const double g0 = std::sqrt((double)n1 * n2 * n3 / (4.0 * M_PI)) * wigner3j(l1, l2, l3, 0, 0, 0);
  std::vector<std::complex<double>> G(n1 * n2 * n3);
  double norm2 = 0.0;
  for (int a = 0; a < n1; ++a)
    for (int b = 0; b < n2; ++b)
      for (int c = 0; c < n3; ++c) {
        std::complex<double> acc = 0.0;
        for (int u1 = -l1; u1 <= l1; ++u1) {
          std::complex<double> x1 = U(l1, a - l1, u1);
          if (x1 == 0.0) continue;
          for (int u2 = -l2; u2 <= l2; ++u2) {
            std::complex<double> x2 = U(l2, b - l2, u2);
            if (x2 == 0.0) continue;
            int u3 = -u1 - u2;
            if (u3 < -l3 || u3 > l3) continue;
            std::complex<double> x3 = U(l3, c - l3, u3);
            if (x3 == 0.0) continue;
            acc += x1 * x2 * x3 * g0 * wigner3j(l1, l2, l3, u1, u2, u3);
          }
        }
        G[(a * n2 + b) * n3 + c] = acc;
        norm2 += std::norm(acc);
      }
  const double inv = 1.0 / std::sqrt(norm2);
  for (int k = 0; k < n1 * n2 * n3; ++k) {
    if (std::abs(G[k].imag()) > 1e-12 * std::sqrt(norm2)) return false;
    out[k] = G[k].real() * inv;
  }
  return true;
}

std::vector<Path> layer_paths(int t, int l_max) {
  std::vector<Path> out;
  int l1_max = (t == 1) ? 0 : l_max;
  for (int l1 = 0; l1 <= l1_max; ++l1)
    for (int l2 = 0; l2 <= l_max; ++l2)
      for (int l3 = 0; l3 <= l_max; ++l3)
        if (natural_path(l1, l2, l3)) out.push_back({l1, l2, l3});
  return out;
}

}  // namespace mpip
