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
  scal.ensure(&c.pool, (size_t)(16 + 2 * (kmax + 1) + 4 * kmax) * sizeof(double));
  stage.ensure(16 + 4 * (kmax + 1));
}

// device scalar slots in Krylov::scal: fixed slots, the complex
// re-orthogonalisation coefficients at S_COEF, then the recurrence's
// <v_j, w> as (re, im) pairs [2 kmax] (alpha_j is the real part), beta[kmax]
// and the next-vector scales[kmax]
enum { S_ALPHA = 0, S_BETA = 1, S_NRM2 = 2, S_E = 3, S_TMP = 4, S_COEF = 16 };

static double* slot(Krylov& K, int i) { return K.scal.as<double>() + i; }
static double* alpha_slots(Krylov& K) { return slot(K, S_COEF + 2 * (K.kmax + 1)); }
static double* beta_slots(Krylov& K) { return alpha_slots(K) + 2 * K.kmax; }
static double* scale_slots(Krylov& K) { return beta_slots(K) + K.kmax; }

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

// Step j of the recurrence, entirely on the device (no host round trip):
//   w = H v_j;  alpha_j = Re <v_j, w>;  w -= alpha_j v_j + beta_{j-1} v_{j-1};
//   two passes w -= V (V^H w) over v_0 .. v_j;  beta_j = |w|;
//   v_{j+1} = w / beta_j (zero after a breakdown, see launch_lanczos_beta).
// With `ev` (6 events) the matvec and its two GEMM launches are bracketed.
static void lanczos_step(Ctx& c, HeffOp& op, Krylov& K, int j, int kmax, const tnt_lanczos_params& p,
                         const hipEvent_t* ev) {
  const int64_t n = K.n, ld = 2 * n;
  double* V = K.basis.as<double>();
  double* w = K.w.as<double>();
  double* A = alpha_slots(K);
  double* Bt = beta_slots(K);
  double* Sc = scale_slots(K);
  double* vj = V + (size_t)j * ld;
  if (ev) TNT_HIP(hipEventRecord(ev[0], c.stream));
  op.apply(vj, vj + n, w, w + n, p.precision, ev ? ev + 2 : nullptr);
  if (ev) TNT_HIP(hipEventRecord(ev[1], c.stream));
  launch_multidot(vj, ld, 1, w, n, K.part.as<double>(), c.stream);
  launch_reduce_partials(K.part.as<double>(), 2, RED_BLOCKS, A + 2 * j, c.stream);
  launch_axpy2(vj, A + 2 * j, j > 0 ? V + (size_t)(j - 1) * ld : nullptr,
               j > 0 ? Bt + j - 1 : nullptr, w, n, c.stream);
  for (int pass = 0; pass < 2; ++pass) {
    launch_multidot(V, ld, j + 1, w, n, K.part.as<double>(), c.stream);
    launch_reduce_partials(K.part.as<double>(), 2 * (j + 1), RED_BLOCKS, slot(K, S_COEF),
                           c.stream);
    launch_multiaxpy_norm(V, ld, j + 1, slot(K, S_COEF), w, n, K.part.as<double>(), c.stream);
  }
  launch_reduce_partials(K.part.as<double>(), 1, RED_BLOCKS, slot(K, S_NRM2), c.stream);
  launch_lanczos_beta(slot(K, S_NRM2), A, p.beta_tol, Bt + j, Sc + j, c.stream);
  if (j + 1 < kmax) launch_scale_copy(w, V + (size_t)(j + 1) * ld, n, Sc + j, c.stream);
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

  // the Krylov space of an n-dimensional operator has dimension <= n
  const int kmax = (int)std::min<int64_t>(p.kmax, n);
  if (tm) {
    while ((int)c.step_ev.size() < 6 * kmax) {
      hipEvent_t e;
      TNT_HIP(hipEventCreate(&e));
      c.step_ev.push_back(e);
    }
  }
  if (c.graphs && !tm) {
    // the whole recurrence as one HIP graph, re-captured only when a buffer
    // it references moved (or the step count / precision changed)
    op.prepare(V, V + n, w, w + n, p.precision);
    std::vector<const void*> key = {V, w, K.part.ptr, K.scal.ptr, (const void*)(intptr_t)kmax,
                                    (const void*)(intptr_t)p.precision,
                                    (const void*)(intptr_t)K.kmax, op.L_re, op.L_im, op.R_re,
                                    op.R_im};
    for (auto& b : c.ws) key.push_back(b.ptr);
    if (!op.graph.exec || op.graph.key != key) {
      if (op.graph.exec) {
        TNT_HIP(hipStreamSynchronize(c.stream));
        TNT_HIP(hipGraphExecDestroy(op.graph.exec));
        op.graph.exec = nullptr;
      }
      if (!c.gstream) TNT_HIP(hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      const hipStream_t main = c.stream;
      c.stream = c.gstream;  // every launch below is recorded, none runs
      hipError_t ce = hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed);
      if (ce == hipSuccess) {
        try {
          for (int j = 0; j < kmax; ++j) lanczos_step(c, op, K, j, kmax, p, nullptr);
        } catch (...) {
          (void)hipStreamEndCapture(c.stream, &g);
          if (g) (void)hipGraphDestroy(g);
          c.stream = main;
          throw;
        }
        ce = hipStreamEndCapture(c.stream, &g);
      }
      c.stream = main;
      if (ce != hipSuccess) fail(TNT_E_HIP, std::string("graph recording: ") + hipGetErrorString(ce));
      hipError_t ie = hipGraphInstantiate(&op.graph.exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        op.graph.exec = nullptr;
        fail(TNT_E_HIP, std::string("graph instantiation: ") + hipGetErrorString(ie));
      }
      op.graph.key = key;
    }
    TNT_HIP(hipGraphLaunch(op.graph.exec, c.stream));
  } else {
    for (int j = 0; j < kmax; ++j)
      lanczos_step(c, op, K, j, kmax, p, tm ? &c.step_ev[6 * j] : nullptr);
  }
  o.matvecs = kmax;
  // alpha and beta to the host: the one round trip of the recurrence
  TNT_HIP(hipMemcpyAsync(K.stage.p, alpha_slots(K), 3 * K.kmax * sizeof(double),
                         hipMemcpyDeviceToHost, c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  const double* ah = K.stage.p;                 // (re, im) pairs
  const double* bh = K.stage.p + 2 * K.kmax;
  std::vector<double> alpha, beta;
  const double thr = p.beta_tol * std::max(1.0, std::fabs(ah[0]));
  for (int j = 0; j < kmax; ++j) {
    if (!std::isfinite(ah[2 * j]) || !std::isfinite(bh[j]))
      fail(TNT_E_NONFINITE, "Lanczos produced NaN/Inf");
    alpha.push_back(ah[2 * j]);
    if (j == kmax - 1 || !(bh[j] > thr)) break;
    beta.push_back(bh[j]);
  }
  if (tm) {
    for (int j = 0; j < kmax; ++j) {
      const hipEvent_t* ev = &c.step_ev[6 * j];
      float ms = 0, m1 = 0, m4 = 0;
      TNT_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
      TNT_HIP(hipEventElapsedTime(&m1, ev[2], ev[3]));
      TNT_HIP(hipEventElapsedTime(&m4, ev[4], ev[5]));
      tm->matvec_s += ms * 1e-3;
      tm->gemm_s += (m1 + m4) * 1e-3;
      tm->gemm_launches += 2;
    }
  }
  const int k = (int)alpha.size();
  std::vector<double> y;
  double ev = 0;
  tridiag_lowest(alpha, beta, &ev, y);
  o.E_ritz = ev;
  o.steps = k;
  // psi = V y, normalised, into x
  double* yst = K.stage.p + 3 * K.kmax + 8;
  for (int i = 0; i < k; ++i) yst[i] = y[i];
  TNT_HIP(hipMemcpyAsync(slot(K, S_COEF), yst, k * sizeof(double), hipMemcpyHostToDevice,
                         c.stream));
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
