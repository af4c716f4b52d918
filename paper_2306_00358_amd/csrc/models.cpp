// Initial site tensors on the host, FP64 (arXiv 2306.00358, Sec. 3).
// Legs (left, up, right, down), row-major, left slowest.
#include <cmath>
#include <stdexcept>
#include <vector>

namespace hotrg {

// Ising (Sec. 3.2, bond dimension 2): the bond weight exp(beta J s s') is
// split as Q Q^T with Q[s][0] = sqrt(cosh(beta J)), Q[s][1] = s sqrt(sinh(beta J));
// the site tensor sums the spin over the four factors of its bonds.
std::vector<double> ising_tensor(double beta, double J) {
  const double bj = beta * J;
  if (!(bj >= 0.0)) throw std::invalid_argument("ising: beta*J must be >= 0");
  const double c = std::sqrt(std::cosh(bj)), s = std::sqrt(std::sinh(bj));
  const double Q[2][2] = {{c, s}, {c, -s}};
  std::vector<double> T(16, 0.0);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) {
          double v = 0.0;
          for (int sp = 0; sp < 2; ++sp) v += Q[sp][i] * Q[sp][j] * Q[sp][k] * Q[sp][l];
          T[((i * 2 + j) * 2 + k) * 2 + l] = v;
        }
  return T;
}

// Classical XY (Sec. 3.1 with Delta = 1, h = 0) by the character expansion
// exp(beta cos x) = sum_n I_n(beta) e^{inx}: charge conservation
// n_l + n_u = n_r + n_d at each site, each bond weight I_n split as
// sqrt(I_n) on its two ends, charges |n| <= n_max.
std::vector<double> xy_tensor(double beta, int n_max) {
  if (n_max < 0 || n_max > 64) throw std::invalid_argument("xy: 0 <= n_max <= 64");
  if (!(beta >= 0.0)) throw std::invalid_argument("xy: beta must be >= 0");
  const int D = 2 * n_max + 1;
  std::vector<double> w(D);
  for (int m = 0; m < D; ++m) w[m] = std::sqrt(std::cyl_bessel_i((double)std::abs(m - n_max), beta));
  std::vector<double> T((size_t)D * D * D * D, 0.0);
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b)
      for (int c = 0; c < D; ++c) {
        int d = a + b - c;
        if (d >= 0 && d < D) T[(((size_t)a * D + b) * D + c) * D + d] = w[a] * w[b] * w[c] * w[d];
      }
  return T;
}

// Generalized XY (Sec. 3.1, Eq. (gXY_ham) with h = 0): the bond weight
// exp(x cos t + y cos 2t), x = beta Delta, y = beta (1 - Delta), has character
// coefficients c_n = sum_m I_{n-2m}(x) I_m(y) (product of the two expansions);
// the tensor is the XY construction with I_n replaced by c_n.  The terms fall
// off like (x/2)^|k| / |k|! (y/2)^|m| / |m|!, so |m| <= n_max + 40 suffices.
std::vector<double> gxy_tensor(double beta, double delta, int n_max) {
  if (n_max < 0 || n_max > 64) throw std::invalid_argument("gxy: 0 <= n_max <= 64");
  if (!(beta >= 0.0)) throw std::invalid_argument("gxy: beta must be >= 0");
  if (!(delta >= 0.0 && delta <= 1.0)) throw std::invalid_argument("gxy: 0 <= delta <= 1");
  const double x = beta * delta, y = beta * (1.0 - delta);
  const int D = 2 * n_max + 1, mm = n_max + 40;
  std::vector<double> w(D);
  for (int i = 0; i < D; ++i) {
    const int n = i - n_max;
    double c = 0.0;
    for (int m = -mm; m <= mm; ++m)
      c += std::cyl_bessel_i((double)std::abs(n - 2 * m), x) *
           std::cyl_bessel_i((double)std::abs(m), y);
    w[i] = std::sqrt(c);
  }
  std::vector<double> T((size_t)D * D * D * D, 0.0);
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b)
      for (int c = 0; c < D; ++c) {
        int d = a + b - c;
        if (d >= 0 && d < D) T[(((size_t)a * D + b) * D + c) * D + d] = w[a] * w[b] * w[c] * w[d];
      }
  return T;
}

// q-state Potts (Sec. 3.3): W[a][b] = e^beta if a == b else 1, W = L L^T
// (Cholesky), T[i,j,k,l] = sum_s L[s][i] L[s][j] L[s][k] L[s][l].
std::vector<double> potts_tensor(double beta, int q) {
  if (q < 2 || q > 32) throw std::invalid_argument("potts: 2 <= q <= 32");
  if (!(beta >= 0.0)) throw std::invalid_argument("potts: beta must be >= 0");
  std::vector<double> W((size_t)q * q), L((size_t)q * q, 0.0);
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) W[a * q + b] = a == b ? std::exp(beta) : 1.0;
  for (int j = 0; j < q; ++j) {  // Cholesky-Banachiewicz, lower triangular
    for (int i = j; i < q; ++i) {
      double s = W[i * q + j];
      for (int k = 0; k < j; ++k) s -= L[i * q + k] * L[j * q + k];
      if (i == j) {
        if (!(s > 0.0)) throw std::invalid_argument("potts: weight matrix not positive definite");
        L[i * q + j] = std::sqrt(s);
      } else {
        L[i * q + j] = s / L[j * q + j];
      }
    }
  }
  std::vector<double> T((size_t)q * q * q * q, 0.0);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j)
      for (int k = 0; k < q; ++k)
        for (int l = 0; l < q; ++l) {
          double v = 0.0;
          for (int s = 0; s < q; ++s) v += L[s * q + i] * L[s * q + j] * L[s * q + k] * L[s * q + l];
          T[(((size_t)i * q + j) * q + k) * q + l] = v;
        }
  return T;
}

}  // namespace hotrg
