// Symmetric eigen-decomposition for the bottom solver: Householder reduction
// to tridiagonal form followed by implicit symmetric QR steps with a
// Wilkinson shift (Golub & Van Loan, "Matrix Computations", sections 8.3.1
// and 8.3.3), eigenvectors accumulated from both stages.
#include <cmath>
#include <vector>

#include "host.hpp"

namespace ldgs {

void sym_eigen(int n, std::vector<double>& A, std::vector<double>& lam) {
  // Q^T A Q = T, Q stored as Zt (row i = column i of Q) for cache-friendly rotations
  std::vector<double> Zt(n * (size_t)n, 0.0);
  for (int i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    // Householder vector for A[k+1:, k]
    double sig = 0.0;
    for (int i = k + 1; i < n; ++i) sig += A[(size_t)i * n + k] * A[(size_t)i * n + k];
    double nrm = std::sqrt(sig);
    if (nrm == 0.0) continue;
    double x0 = A[(size_t)(k + 1) * n + k];
    double alpha = (x0 > 0) ? -nrm : nrm;
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    v[k + 1] = x0 - alpha;
    for (int i = k + 2; i < n; ++i) v[i] = A[(size_t)i * n + k];
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // A <- H A H on the trailing block, H = I - 2 v v^T
    double beta = 0.0;
    for (int i = k + 1; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += A[(size_t)i * n + j] * v[j];
      p[i] = s;
      beta += v[i] * s;
    }
    for (int i = k + 1; i < n; ++i) w[i] = 2.0 * (p[i] - beta * v[i]);
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= v[i] * w[j] + w[i] * v[j];
    A[(size_t)(k + 1) * n + k] = alpha;
    A[(size_t)k * n + k + 1] = alpha;
    for (int i = k + 2; i < n; ++i) {
      A[(size_t)i * n + k] = 0.0;
      A[(size_t)k * n + i] = 0.0;
    }
    // Q <- Q H: columns k+1.. of Q are rows of Zt
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += Zt[(size_t)i * n + r] * v[i];
      s *= 2.0;
      if (s != 0.0)
        for (int i = k + 1; i < n; ++i) Zt[(size_t)i * n + r] -= s * v[i];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];

  // implicit symmetric QR with Wilkinson shift on the unreduced trailing block
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int guard = 0;
  while (hi > 0 && guard < 60 * n) {
    ++guard;
    // deflate
    for (int i = 0; i < hi; ++i)
      if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    while (hi > 0 && e[hi - 1] == 0.0) --hi;
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    // Wilkinson shift from the trailing 2x2 block
    double a = d[hi - 1], b = e[hi - 1], c = d[hi];
    double del = 0.5 * (a - c);
    double sgn = (del >= 0.0) ? 1.0 : -1.0;
    double mu = c - b * b / (del + sgn * std::hypot(del, b));
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      // rotation R = [[cs, -sn], [sn, cs]] on rows/cols k, k+1, zeroing z against x
      double r = std::hypot(x, z);
      double cs = (r == 0.0) ? 1.0 : x / r;
      double sn = (r == 0.0) ? 0.0 : -z / r;
      if (k > lo) e[k - 1] = r;   // the bulge chased into e[k-1]
      double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = cs * cs * dk - 2.0 * cs * sn * ek + sn * sn * dk1;
      d[k + 1] = sn * sn * dk + 2.0 * cs * sn * ek + cs * cs * dk1;
      e[k] = cs * sn * (dk - dk1) + (cs * cs - sn * sn) * ek;
      if (k + 1 < hi) {
        double ek1 = e[k + 1];
        z = -sn * ek1;          // new bulge at (k, k+2)
        e[k + 1] = cs * ek1;
        x = e[k];
      }
      // accumulate Z <- Z R^T: columns k, k+1 of Z are rows k, k+1 of Zt
      double* zk = &Zt[(size_t)k * n];
      double* zk1 = &Zt[(size_t)(k + 1) * n];
      for (int q = 0; q < n; ++q) {
        double u0 = zk[q], u1 = zk1[q];
        zk[q] = cs * u0 - sn * u1;
        zk1[q] = sn * u0 + cs * u1;
      }
    }
  }
  lam = d;
  // return eigenvectors in columns of A
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = Zt[(size_t)j * n + i];
}

}  // namespace ldgs
