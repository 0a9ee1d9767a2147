// Symmetric eigen-decomposition of the 1-D operators that the fast-
// diagonalization Poisson solve needs, on the host, once per context.
//
// Cyclic Jacobi rotations (Rutishauser's stable update): A is reduced to
// diagonal form by plane rotations that zero one off-diagonal pair each;
// the product of the rotations gives an orthogonal Q with A = Q diag(lam) Q^T.
// Jacobi is slow (O(n^3) per sweep, a few sweeps) but simple and accurate,
// and n <= a few hundred here.
#include <cmath>
#include <vector>

#include "kv_internal.h"

namespace kv {

void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& lam) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  auto a = [&](int r, int c) -> double& { return A[(size_t)r * n + c]; };
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale += a(i, i) * a(i, i);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a(p, q) * a(p, q);
    if (off <= 1e-36 * scale) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        const double app = a(p, p), aqq = a(q, q);
        if (sweep > 3 && std::fabs(apq) < 1e-18 * (std::fabs(app) + std::fabs(aqq))) {
          a(p, q) = a(q, p) = 0.0;
          continue;
        }
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        const double tau = s / (1.0 + c);
        a(p, p) = app - t * apq;
        a(q, q) = aqq + t * apq;
        a(p, q) = a(q, p) = 0.0;
        for (int r = 0; r < n; ++r) {
          if (r == p || r == q) continue;
          const double arp = a(r, p), arq = a(r, q);
          a(r, p) = a(p, r) = arp - s * (arq + tau * arp);
          a(r, q) = a(q, r) = arq + s * (arp - tau * arq);
        }
        for (int r = 0; r < n; ++r) {
          const double qrp = Q[(size_t)r * n + p], qrq = Q[(size_t)r * n + q];
          Q[(size_t)r * n + p] = qrp - s * (qrq + tau * qrp);
          Q[(size_t)r * n + q] = qrq + s * (qrp - tau * qrq);
        }
      }
    }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = a(i, i);
}

}  // namespace kv
