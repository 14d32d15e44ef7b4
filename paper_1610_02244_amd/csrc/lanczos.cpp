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
// and v the eigenvectors as columns.
void jacobi_eigh(std::vector<double>& a, std::vector<double>& v, int n) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
        tot += x;
        if (i != j) off += x;
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        // rotation angle that zeroes a[p][q]: tan(2 phi) = 2 apq / (aqq - app)
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = cs * akp - sn * akq;
          a[(size_t)k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = cs * apk - sn * aqk;
          a[(size_t)q * n + k] = sn * apk + cs * aqk;
        }
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
  kmax = kmax_;
  n = n_;
  basis.ensure(&c.pool, (size_t)kmax * 2 * n * sizeof(double));
  w.ensure(&c.pool, (size_t)2 * n * sizeof(double));
  part.ensure(&c.pool, (size_t)RED_BLOCKS * 2 * (kmax + 1) * sizeof(double));
  scal.ensure(&c.pool, (size_t)(16 + 2 * (kmax + 1)) * sizeof(double));
  stage.ensure(8 + 2 * (kmax + 1));
}

// device scalar slots in Krylov::scal
enum { S_ALPHA = 0, S_BETA = 1, S_NRM2 = 2, S_E = 3, S_TMP = 4, S_COEF = 16 };

static double* slot(Krylov& K, int i) { return K.scal.as<double>() + i; }

// |x|^2 of a 2n-double vector into a device slot
static void norm2_to(Ctx& c, Krylov& K, const double* x, double* dst) {
  launch_norm2_partial(x, 2 * K.n, K.part.as<double>(), c.stream);
  launch_reduce_partials(K.part.as<double>(), 1, RED_BLOCKS, dst, c.stream);
}

static double read_scalar(Ctx& c, Krylov& K, const double* dev) {
  TNT_HIP(hipMemcpyAsync(K.stage.p, dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  return K.stage.p[0];
}

LanczosOut lanczos_run(Ctx& c, HeffOp& op, Krylov& K, double* x, const tnt_lanczos_params& p,
                       Timers* tm) {
  const int64_t n = K.n;
  const int64_t ld = 2 * n;
  double* V = K.basis.as<double>();
  double* w = K.w.as<double>();
  LanczosOut o;

  // v0 = x / |x|
  norm2_to(c, K, x, slot(K, S_NRM2));
  const double x2 = read_scalar(c, K, slot(K, S_NRM2));
  if (!std::isfinite(x2)) fail(TNT_E_NONFINITE, "start vector is not finite");
  if (x2 <= 0.0) fail(TNT_E_ARG, "start vector is zero");
  launch_normalize_copy(x, V, n, slot(K, S_NRM2), c.stream);

  std::vector<double> alpha, beta;
  const int kmax = p.kmax;
  for (int j = 0; j < kmax; ++j) {
    double* vj = V + (size_t)j * ld;
    // w = H v_j (iteration precision)
    if (tm) TNT_HIP(hipEventRecord(c.ev[0], c.stream));
    op.apply(vj, vj + n, w, w + n, p.precision, tm != nullptr);
    if (tm) TNT_HIP(hipEventRecord(c.ev[1], c.stream));
    o.matvecs++;
    // alpha_j = Re <v_j, w>
    launch_multidot(vj, ld, 1, w, n, K.part.as<double>(), c.stream);
    launch_reduce_partials(K.part.as<double>(), 2, RED_BLOCKS, slot(K, S_ALPHA), c.stream);
    // w -= alpha_j v_j + beta_{j-1} v_{j-1}
    launch_axpy2(vj, slot(K, S_ALPHA), j > 0 ? V + (size_t)(j - 1) * ld : nullptr,
                 slot(K, S_BETA), w, n, c.stream);
    // two passes of full re-orthogonalisation against v_0 .. v_j
    for (int pass = 0; pass < 2; ++pass) {
      launch_multidot(V, ld, j + 1, w, n, K.part.as<double>(), c.stream);
      launch_reduce_partials(K.part.as<double>(), 2 * (j + 1), RED_BLOCKS, slot(K, S_COEF),
                             c.stream);
      launch_multiaxpy_norm(V, ld, j + 1, slot(K, S_COEF), w, n, K.part.as<double>(),
                            c.stream);
    }
    launch_reduce_partials(K.part.as<double>(), 1, RED_BLOCKS, slot(K, S_NRM2), c.stream);
    // alpha and |w|^2 to the host (the one host round trip per step)
    TNT_HIP(hipMemcpyAsync(K.stage.p, slot(K, S_ALPHA), sizeof(double), hipMemcpyDeviceToHost,
                           c.stream));
    TNT_HIP(hipMemcpyAsync(K.stage.p + 1, slot(K, S_NRM2), sizeof(double),
                           hipMemcpyDeviceToHost, c.stream));
    TNT_HIP(hipStreamSynchronize(c.stream));
    if (tm) {
      float ms = 0, m1 = 0, m4 = 0;
      TNT_HIP(hipEventElapsedTime(&ms, c.ev[0], c.ev[1]));
      TNT_HIP(hipEventElapsedTime(&m1, c.ev[2], c.ev[3]));
      TNT_HIP(hipEventElapsedTime(&m4, c.ev[4], c.ev[5]));
      tm->matvec_s += ms * 1e-3;
      tm->gemm_s += (m1 + m4) * 1e-3;
      tm->gemm_launches += 2;
    }
    const double a = K.stage.p[0];
    const double b = std::sqrt(K.stage.p[1]);
    if (!std::isfinite(a) || !std::isfinite(b)) fail(TNT_E_NONFINITE, "Lanczos produced NaN/Inf");
    alpha.push_back(a);
    if (j == kmax - 1 || b <= p.beta_tol * std::max(1.0, std::fabs(alpha[0]))) break;
    beta.push_back(b);
    // beta_j to its device slot (read by the next step's three-term update)
    K.stage.p[2] = b;
    TNT_HIP(hipMemcpyAsync(slot(K, S_BETA), K.stage.p + 2, sizeof(double),
                           hipMemcpyHostToDevice, c.stream));
    launch_normalize_copy(w, V + (size_t)(j + 1) * ld, n, slot(K, S_NRM2), c.stream);
    // (the host rewrites stage slot 2 only after the next step's stream
    // synchronisation, so the asynchronous copy above has completed by then)
  }
  const int k = (int)alpha.size();
  std::vector<double> y;
  double ev = 0;
  tridiag_lowest(alpha, beta, &ev, y);
  o.E_ritz = ev;
  o.steps = k;
  // psi = V y, normalised, into x
  for (int i = 0; i < k; ++i) K.stage.p[8 + i] = y[i];
  TNT_HIP(hipMemcpyAsync(slot(K, S_COEF), K.stage.p + 8, k * sizeof(double),
                         hipMemcpyHostToDevice, c.stream));
  launch_combine_basis(V, ld, k, slot(K, S_COEF), x, n, c.stream);
  norm2_to(c, K, x, slot(K, S_NRM2));
  launch_normalize_copy(x, x, n, slot(K, S_NRM2), c.stream);
  // FP64 refinement: E = Re <psi, H psi>, r = |H psi - E psi|
  op.apply(x, x + n, w, w + n, TNT_FP64);
  launch_multidot(x, ld, 1, w, n, K.part.as<double>(), c.stream);
  launch_reduce_partials(K.part.as<double>(), 2, RED_BLOCKS, slot(K, S_E), c.stream);
  launch_axpy2(x, slot(K, S_E), nullptr, nullptr, w, n, c.stream);
  norm2_to(c, K, w, slot(K, S_NRM2));
  TNT_HIP(hipMemcpyAsync(K.stage.p, slot(K, S_E), sizeof(double), hipMemcpyDeviceToHost,
                         c.stream));
  TNT_HIP(hipMemcpyAsync(K.stage.p + 1, slot(K, S_NRM2), sizeof(double),
                         hipMemcpyDeviceToHost, c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  o.E = K.stage.p[0];
  o.residual = std::sqrt(std::max(0.0, K.stage.p[1]));
  if (!std::isfinite(o.E) || !std::isfinite(o.residual))
    fail(TNT_E_NONFINITE, "refined energy is not finite");
  return o;
}

}  // namespace tnt
