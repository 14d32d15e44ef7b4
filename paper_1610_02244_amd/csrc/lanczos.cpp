// Lowest eigenpair of the two-site H_eff by Lanczos (Sec. 4.2: the network
// minimiser hands the contractor and the current tensor as initial guess to
// an iterative eigensolver).  Krylov vectors, re-orthogonalisation and the
// final Rayleigh quotient are FP64; the matvecs inside the iteration run in
// the requested precision.
#include "lanczos.h"

#include <algorithm>
#include <chrono>
#include <cmath>

namespace tnt {

// Eigen-decomposition of a small real symmetric matrix (row-major n x n) by
// cyclic Jacobi rotations; on return a holds the eigenvalues on its diagonal
// and v the eigenvectors as columns.  An off-diagonal entry too small to
// change either diagonal entry it couples (below their rounding, with a
// factor 100 of margin) is set to zero instead of rotated, and every rotated
// pair is zeroed exactly, so the off-diagonal sum reaches exactly zero and
// the sweeps stop (typically after 5 to 8).
void jacobi_eigh(std::vector<double>& a, std::vector<double>& v, int n) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) off += std::fabs(A(p, q));
    if (off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A(p, q);
        if (apq == 0.0) continue;
        const double app = A(p, p), aqq = A(q, q);
        const double g = 100.0 * std::fabs(apq);
        if (std::fabs(app) + g == std::fabs(app) && std::fabs(aqq) + g == std::fabs(aqq)) {
          A(p, q) = 0.0;
          A(q, p) = 0.0;
          continue;
        }
        // rotation angle that zeroes a[p][q]: tan(2 phi) = 2 apq / (aqq - app)
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A(k, p), akq = A(k, q);
          A(k, p) = cs * akp - sn * akq;
          A(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A(p, k), aqk = A(q, k);
          A(p, k) = cs * apk - sn * aqk;
          A(q, k) = sn * apk + cs * aqk;
        }
        A(p, q) = 0.0;
        A(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = cs * vkp - sn * vkq;
          v[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
}

void tridiag_lowest(const std::vector<double>& alpha, const std::vector<double>& beta,
                    double* eval, std::vector<double>& evec) {
  const int k = (int)alpha.size();
  std::vector<double> a((size_t)k * k, 0.0), v;
  for (int i = 0; i < k; ++i) a[(size_t)i * k + i] = alpha[i];
  for (int i = 0; i + 1 < k; ++i) {
    a[(size_t)i * k + i + 1] = beta[i];
    a[(size_t)(i + 1) * k + i] = beta[i];
  }
  jacobi_eigh(a, v, k);
  int best = 0;
  for (int i = 1; i < k; ++i)
    if (a[(size_t)i * k + i] < a[(size_t)best * k + best]) best = i;
  *eval = a[(size_t)best * k + best];
  evec.resize(k);
  for (int i = 0; i < k; ++i) evec[i] = v[(size_t)i * k + best];
}

// ---------------------------------------------------------------------------

void Krylov::reserve(Ctx& c, int kmax_, int64_t n_) {
  (void)kmax_;  // the recurrence sizes its basis from the parameters it runs with
  if (n_ != n || seg.nblk == 0) {
    seg.build(c, {0}, {n_});
    n = n_;
  }
}

LanczosOut lanczos_run(Ctx& c, HeffOp& op, Krylov& K, double* x, const tnt_lanczos_params& p,
                       Timers* tm) {
  if (K.n < 0 || K.seg.nblk == 0) fail(TNT_E_STATE, "Krylov space used before reserve");
  std::vector<LanczosOut> out;
  lanczos_core(c, op, K.seg, {K.n}, K.bk, x, p, out, tm);
  return out[0];
}

}  // namespace tnt
