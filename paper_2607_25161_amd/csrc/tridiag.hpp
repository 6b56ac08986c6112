// The square root of a Lanczos tridiagonal applied to e1 (host code, no HIP).
//
// The Lanczos square root of the Brownian terms (Section 2.5, the method of Chow and Saad)
// needs T^{1/2} e1 for the k x k symmetric tridiagonal T of the Lanczos coefficients, at every
// convergence check.  The eigen-decomposition here is the implicit QL method with Wilkinson
// shifts for symmetric tridiagonal matrices (Bowdler, Martin, Reinsch and Wilkinson, Numer.
// Math. 11 (1968) 293-306), O(k^2) rotations with O(k) work each, instead of Jacobi sweeps on
// the dense k x k matrix.
#pragma once

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

namespace fsd {

// T^{1/2} e1 for the symmetric tridiagonal T with diagonal al (k entries) and off-diagonal be
// (k - 1 entries): sum over the eigenpairs (lambda_e, q_e) of q_e sqrt(lambda_e) q_e[0].  The
// matrices of the Lanczos roots are positive semi-definite; eigenvalues that rounding makes
// slightly negative are taken as zero.  The rotations are accumulated into the rows of
// Z = Q^T (row e holds eigenvector e), so each one updates two contiguous rows.
inline std::vector<double> tridiag_sqrt_e1(const std::vector<double>& al, const std::vector<double>& be) {
  const int n = int(al.size());
  std::vector<double> d(al), e(size_t(n), 0.0), z(size_t(n) * size_t(n), 0.0);
  for (int i = 0; i + 1 < n && i < int(be.size()); ++i) e[size_t(i)] = be[size_t(i)];
  for (int i = 0; i < n; ++i) z[size_t(i) * n + i] = 1.0;
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0; iter < 64; ++iter) {
      // the first negligible off-diagonal entry at or after l bounds the unreduced block
      int m = l;
      for (; m + 1 < n; ++m)
        if (std::fabs(e[m]) <= eps * (std::fabs(d[m]) + std::fabs(d[m + 1]))) break;
      if (m == l) break;  // d[l] is an eigenvalue
      // shift: the eigenvalue of the block's leading 2 x 2 part that is nearer d[l]
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      bool split = false;
      // chase the bulge from the bottom of the block to its top with plane rotations
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // the block splits here: restart on the shorter one
          d[i + 1] -= p;
          e[m] = 0.0;
          split = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        double* zi = &z[size_t(i) * n];
        double* zj = &z[size_t(i + 1) * n];
        for (int k = 0; k < n; ++k) {
          const double t = zj[k];
          zj[k] = s * zi[k] + c * t;
          zi[k] = c * zi[k] - s * t;
        }
      }
      if (split) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<double> out(size_t(n), 0.0);
  for (int ev = 0; ev < n; ++ev) {
    const double* q = &z[size_t(ev) * n];
    const double f = std::sqrt(std::max(d[ev], 0.0)) * q[0];
    for (int k = 0; k < n; ++k) out[k] += q[k] * f;
  }
  return out;
}

}  // namespace fsd
