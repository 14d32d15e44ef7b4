// Batch operators and the batched Lanczos recurrence (see batch.h).
#include "batch.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace tnt {

// About this many workgroups per segmented launch, spread over the
// instances in proportion to their size (at least one each).
static constexpr int SEG_TARGET_BLOCKS = 1024;
static constexpr int64_t SEG_MIN_RANGE = 512;  // complex entries per workgroup at least

void SegLayout::build(Ctx& c, const std::vector<int64_t>& off, const std::vector<int64_t>& n) {
  blk.clear();
  inst_blk.clear();
  int64_t N = 0;
  for (int64_t v : n) N += v;
  for (size_t i = 0; i < n.size(); ++i) {
    int64_t nb = N > 0 ? (int64_t)std::llround((double)SEG_TARGET_BLOCKS * n[i] / N) : 1;
    nb = std::max<int64_t>(1, std::min(nb, (n[i] + SEG_MIN_RANGE - 1) / SEG_MIN_RANGE));
    const int64_t chunk = (n[i] + nb - 1) / std::max<int64_t>(nb, 1);
    const int first = (int)blk.size();
    for (int64_t lo = 0; lo < n[i]; lo += chunk)
      blk.push_back(SegBlock{(int)i, 0, off[i] + lo, off[i] + std::min(n[i], lo + chunk)});
    if ((int)blk.size() == first) blk.push_back(SegBlock{(int)i, 0, off[i], off[i]});
    inst_blk.push_back(int2{first, (int)blk.size()});
  }
  nblk = (int)blk.size();
  const size_t bytes = blk.size() * sizeof(SegBlock) + inst_blk.size() * sizeof(int2);
  std::vector<char> host(bytes);
  memcpy(host.data(), blk.data(), blk.size() * sizeof(SegBlock));
  memcpy(host.data() + blk.size() * sizeof(SegBlock), inst_blk.data(),
         inst_blk.size() * sizeof(int2));
  dev = DevBuf(&c.pool, bytes);
  TNT_HIP(hipMemcpyAsync(dev.ptr, host.data(), bytes, hipMemcpyHostToDevice, c.stream));
  // the host copy must outlive the transfer
  TNT_HIP(hipStreamSynchronize(c.stream));
}

RunTable::~RunTable() {
  if (done) (void)hipEventDestroy(done);
}

void RunTable::run(Ctx& c, const std::vector<CopyRun>& runs) {
  if (runs.empty()) return;
  const bool same = runs.size() == host.size() &&
                    memcmp(runs.data(), host.data(), runs.size() * sizeof(CopyRun)) == 0;
  if (!same) {
    if (done) TNT_HIP(hipEventSynchronize(done));  // the last upload has read `host`
    host = runs;
    max_count = 0;
    for (const CopyRun& r : host) max_count = std::max(max_count, r.count);
    dev.ensure(&c.pool, host.size() * sizeof(CopyRun));
    TNT_HIP(hipMemcpyAsync(dev.ptr, host.data(), host.size() * sizeof(CopyRun),
                           hipMemcpyHostToDevice, c.stream));
    if (!done) TNT_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    TNT_HIP(hipEventRecord(done, c.stream));
  }
  launch_copy_runs(dev.as<CopyRun>(), (int)host.size(), max_count, c.stream);
}

void build_batch(Ctx& c, BatchHeff& b, const std::vector<std::shared_ptr<HeffOp>>& ops,
                 const std::vector<int64_t>& n, int prec) {
  std::vector<const HeffPlan*> plans;
  std::vector<int64_t> Lx, Rx;
  for (const auto& op : ops) {
    if (op->precision != prec) fail(TNT_E_STATE, "batch operators disagree in precision");
    plans.push_back(&op->plan);
    Lx.push_back(op->L_ext);
    Rx.push_back(op->R_ext);
  }
  build_batch_plans(c, b, plans, Lx, Rx, n, prec, true);
}

void build_batch_plans(Ctx& c, BatchHeff& b, const std::vector<const HeffPlan*>& plans,
                       const std::vector<int64_t>& L_ext, const std::vector<int64_t>& R_ext,
                       const std::vector<int64_t>& n, int prec, bool tunable) {
  if (plans.empty() || plans.size() != n.size() || L_ext.size() != n.size() ||
      R_ext.size() != n.size())
    fail(TNT_E_ARG, "empty or inconsistent batch");
  b.n = n;
  b.precision = prec;
  b.parts.clear();
  b.L_ext.clear();
  b.R_ext.clear();
  b.N = b.L_tot = b.R_tot = 0;
  std::vector<int64_t> off;
  for (size_t i = 0; i < plans.size(); ++i) {
    if (plans[i]->packed != (prec != TNT_FP64)) fail(TNT_E_STATE, "plan built for another precision");
    b.parts.push_back(BatchPart{b.N, b.L_tot, b.R_tot});
    off.push_back(b.N);
    b.L_ext.push_back(L_ext[i]);
    b.R_ext.push_back(R_ext[i]);
    b.N += n[i];
    b.L_tot += L_ext[i];
    b.R_tot += R_ext[i];
  }
  b.op = std::make_shared<HeffOp>();
  b.op->build_plan(c, merge_heff_plans(plans, b.parts), prec, tunable);
  b.op->L_ext = b.L_tot;
  b.op->R_ext = b.R_tot;
  b.seg.build(c, off, n);
}

void bind_batch_envs(Ctx& c, BatchHeff& b, const std::vector<const double*>& Lre,
                     const std::vector<const double*>& Lim, const std::vector<const double*>& Rre,
                     const std::vector<const double*>& Rim) {
  const int m = b.ninst();
  b.envs.ensure(&c.pool, std::max<int64_t>(1, 2 * (b.L_tot + b.R_tot)) * sizeof(double));
  double* Lr = b.envs.as<double>();
  double* Li = Lr + b.L_tot;
  double* Rr = Li + b.L_tot;
  double* Ri = Rr + b.R_tot;
  std::vector<CopyRun> runs;
  for (int i = 0; i < m; ++i) {
    const BatchPart& w = b.parts[i];
    runs.push_back(CopyRun{Lre[i], Lr + w.L_off, b.L_ext[i]});
    runs.push_back(CopyRun{Lim[i], Li + w.L_off, b.L_ext[i]});
    runs.push_back(CopyRun{Rre[i], Rr + w.R_off, b.R_ext[i]});
    runs.push_back(CopyRun{Rim[i], Ri + w.R_off, b.R_ext[i]});
  }
  b.env_runs.run(c, runs);
  b.op->bind_envs(Lr, Li, Rr, Ri);
}

// ---------------------------------------------------------------------------
// batched Lanczos
// ---------------------------------------------------------------------------
// per-instance scalar block (stride S): the recurrence's <v_j, H v_j> pairs
// (alpha_j = real part), beta_j, next-vector scales, |w|^2, the
// refinement's <psi, H psi> pair and the Ritz coefficients
struct Slots {
  int apair, beta, scale, nrm2, e, y, S;
  explicit Slots(int kmax) {
    apair = 0;
    beta = apair + 2 * kmax;
    scale = beta + kmax;
    nrm2 = scale + kmax;
    e = nrm2 + 1;
    y = e + 2;
    S = y + kmax;
  }
};

void BatchKrylov::reserve(Ctx& c, int kmax_, int64_t N_, int ninst_, int nblk) {
  kmax = kmax_;
  N = N_;
  ninst = ninst_;
  S = Slots(kmax).S;
  basis.ensure(&c.pool, (size_t)kmax * 2 * N * sizeof(double));
  w.ensure(&c.pool, (size_t)2 * N * sizeof(double));
  part.ensure(&c.pool, (size_t)nblk * 2 * (kmax + 1) * sizeof(double));
  part2.ensure(&c.pool, (size_t)nblk * 2 * (kmax + 1) * sizeof(double));
  scal.ensure(&c.pool, (size_t)ninst * S * sizeof(double));
  kdev.ensure(&c.pool, (size_t)std::max(1, ninst) * sizeof(int));
  stage.ensure((size_t)ninst * S + 8);
}

// Step j of the recurrence for every instance, on the device:
//   w = H v_j;  c = V^H w over v_0 .. v_j (alpha_j = Re c_j);
//   w -= V c;  c' = V^H w;  w -= V c'  (classical Gram-Schmidt, twice);
//   beta_j = |w|;  v_{j+1} = w / beta_j (zero after a breakdown).
// Subtracting the full projection also removes alpha_j v_j and
// beta_{j-1} v_{j-1}, the three-term part of the recurrence.
static void lanczos_step_batched(Ctx& c, HeffOp& op, const SegLayout& seg, BatchKrylov& K,
                                 int j, const tnt_lanczos_params& p, const hipEvent_t* ev) {
  const Slots sl(K.kmax);
  const int64_t N = K.N, ld = 2 * N;
  const int S = K.S, nb = seg.nblk, k = j + 1;
  const SegBlock* blk = seg.d_blk();
  const int2* ib = seg.d_inst();
  double* V = K.basis.as<double>();
  double* w = K.w.as<double>();
  double* sc = K.scal.as<double>();
  double* pa = K.part.as<double>();
  double* pb = K.part2.as<double>();
  double* vj = V + (size_t)j * ld;
  if (ev) TNT_HIP(hipEventRecord(ev[0], c.stream));
  op.apply(vj, vj + N, w, w + N, p.precision, ev ? ev + 2 : nullptr);
  if (ev) TNT_HIP(hipEventRecord(ev[1], c.stream));
  launch_seg_cgs_dot(V, ld, k, w, N, blk, nb, pa, c.stream);
  launch_seg_cgs_update_dot(V, ld, k, pa, w, N, blk, ib, nb, pb, sc + sl.apair + 2 * j, S,
                            c.stream);
  launch_seg_cgs_update_norm(V, ld, k, pb, w, N, blk, ib, nb, pa, c.stream);
  launch_seg_cgs_next(pa, w, j + 1 < K.kmax ? V + (size_t)(j + 1) * ld : nullptr, N, blk, ib, nb,
                      sc, S, sl.nrm2, sl.apair, sl.beta + j, sl.scale + j, p.beta_tol, j,
                      K.kdev.as<int>(), c.stream);
}

void lanczos_core(Ctx& c, HeffOp& op, const SegLayout& seg, const std::vector<int64_t>& n,
                  BatchKrylov& K, double* x, const tnt_lanczos_params& p,
                  std::vector<LanczosOut>& out, Timers* tm) {
  const int m = (int)n.size();
  int64_t N = 0;
  for (int64_t v : n) N += v;
  const int64_t ld = 2 * N;
  const SegBlock* blk = seg.d_blk();
  const int2* ib = seg.d_inst();
  const int nb = seg.nblk;
  // the fused re-orthogonalisation kernels hold at most 32 coefficients
  if (p.kmax < 1 || p.kmax > 32) fail(TNT_E_ARG, "kmax must be in [1, 32]");
  // per-instance step counts: the Krylov space has dimension <= n_i
  std::vector<int> kmax_i(m);
  int kmax = 0;
  for (int i = 0; i < m; ++i) {
    kmax_i[i] = (int)std::min<int64_t>(p.kmax, n[i]);
    kmax = std::max(kmax, kmax_i[i]);
  }
  K.reserve(c, kmax, N, m, nb);
  const Slots sl(K.kmax);
  const int S = K.S;
  double* V = K.basis.as<double>();
  double* w = K.w.as<double>();
  double* sc = K.scal.as<double>();
  double* part = K.part.as<double>();
  // through the pinned stage, so the copy does not wait for the stream
  memcpy(K.stage.p, kmax_i.data(), m * sizeof(int));
  TNT_HIP(hipMemcpyAsync(K.kdev.ptr, K.stage.p, m * sizeof(int), hipMemcpyHostToDevice,
                         c.stream));
  // v0 = x / |x| per instance
  launch_seg_norm2(x, N, blk, nb, part, c.stream);
  launch_seg_reduce(part, 1, ib, m, sc + sl.nrm2, S, c.stream);
  TNT_HIP(hipMemcpyAsync(K.stage.p, sc, (size_t)m * S * sizeof(double), hipMemcpyDeviceToHost,
                         c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  for (int i = 0; i < m; ++i) {
    const double x2 = K.stage.p[(size_t)i * S + sl.nrm2];
    if (!std::isfinite(x2)) fail(TNT_E_NONFINITE, "start vector is not finite");
    if (x2 <= 0.0) fail(TNT_E_ARG, "start vector is zero");
  }
  launch_seg_scale_copy(x, V, N, blk, nb, sc + sl.nrm2, S, 1, c.stream);
  if (tm) {
    while ((int)c.step_ev.size() < 6 * kmax) {
      hipEvent_t e;
      TNT_HIP(hipEventCreate(&e));
      c.step_ev.push_back(e);
    }
  }
  if (c.graphs && !tm) {
    op.prepare(V, V + N, w, w + N, p.precision);
    std::vector<const void*> key = {V, w, K.part.ptr, K.part2.ptr, K.scal.ptr, K.kdev.ptr,
                                    seg.dev.ptr,
                                    (const void*)(intptr_t)kmax,
                                    (const void*)(intptr_t)p.precision, op.L_re, op.L_im,
                                    op.R_re, op.R_im};
    for (auto& bf : c.ws) key.push_back(bf.ptr);
    if (!op.graph.exec || op.graph.key != key) {
      if (op.graph.exec) {
        TNT_HIP(hipStreamSynchronize(c.stream));
        TNT_HIP(hipGraphExecDestroy(op.graph.exec));
        op.graph.exec = nullptr;
      }
      if (!c.gstream) TNT_HIP(hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      const hipStream_t main = c.stream;
      c.stream = c.gstream;  // recorded, not run
      hipError_t ce = hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed);
      if (ce == hipSuccess) {
        try {
          for (int j = 0; j < kmax; ++j) lanczos_step_batched(c, op, seg, K, j, p, nullptr);
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
      lanczos_step_batched(c, op, seg, K, j, p, tm ? &c.step_ev[6 * j] : nullptr);
  }
  // every instance's alpha / beta in one round trip
  TNT_HIP(hipMemcpyAsync(K.stage.p, sc, (size_t)m * S * sizeof(double), hipMemcpyDeviceToHost,
                         c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
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
  out.assign(m, LanczosOut{});
  std::vector<double> yall((size_t)m * S, 0.0);
  int kuse = 1;
  for (int i = 0; i < m; ++i) {
    const double* s = K.stage.p + (size_t)i * S;
    std::vector<double> alpha, beta;
    const double thr = p.beta_tol * std::max(1.0, std::fabs(s[sl.apair]));
    for (int j = 0; j < kmax_i[i]; ++j) {
      const double a = s[sl.apair + 2 * j], bb = s[sl.beta + j];
      if (!std::isfinite(a) || !std::isfinite(bb)) fail(TNT_E_NONFINITE, "Lanczos produced NaN/Inf");
      alpha.push_back(a);
      if (j == kmax_i[i] - 1 || !(bb > thr)) break;
      beta.push_back(bb);
    }
    std::vector<double> y;
    double ev = 0;
    tridiag_lowest(alpha, beta, &ev, y);
    out[i].E_ritz = ev;
    out[i].steps = (int)alpha.size();
    out[i].matvecs = kmax_i[i];
    kuse = std::max(kuse, (int)alpha.size());
    for (size_t q = 0; q < y.size(); ++q) yall[(size_t)i * S + sl.y + q] = y[q];
  }
  // psi_i = V y_i (y_i zero beyond the instance's steps), normalised
  memcpy(K.stage.p, yall.data(), yall.size() * sizeof(double));
  TNT_HIP(hipMemcpyAsync(sc, K.stage.p, yall.size() * sizeof(double), hipMemcpyHostToDevice,
                         c.stream));
  launch_seg_combine_basis(V, ld, kuse, sc + sl.y, S, x, N, blk, nb, c.stream);
  launch_seg_norm2(x, N, blk, nb, part, c.stream);
  launch_seg_reduce(part, 1, ib, m, sc + sl.nrm2, S, c.stream);
  launch_seg_scale_copy(x, x, N, blk, nb, sc + sl.nrm2, S, 1, c.stream);
  // FP64 refinement for all instances: E_i = Re <psi_i, H psi_i>, r_i
  op.apply(x, x + N, w, w + N, TNT_FP64);
  launch_seg_cgs_dot(x, ld, 1, w, N, blk, nb, part, c.stream);
  launch_seg_reduce(part, 2, ib, m, sc + sl.e, S, c.stream);
  launch_seg_axpy2(x, sc + sl.e, S, nullptr, nullptr, S, w, N, blk, nb, c.stream);
  launch_seg_norm2(w, N, blk, nb, part, c.stream);
  launch_seg_reduce(part, 1, ib, m, sc + sl.nrm2, S, c.stream);
  TNT_HIP(hipMemcpyAsync(K.stage.p, sc, (size_t)m * S * sizeof(double), hipMemcpyDeviceToHost,
                         c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  for (int i = 0; i < m; ++i) {
    const double* s = K.stage.p + (size_t)i * S;
    out[i].E = s[sl.e];
    out[i].residual = std::sqrt(std::max(0.0, s[sl.nrm2]));
    if (!std::isfinite(out[i].E) || !std::isfinite(out[i].residual))
      fail(TNT_E_NONFINITE, "refined energy is not finite");
  }
}

void lanczos_run_batched(Ctx& c, BatchHeff& b, BatchKrylov& K, double* x,
                         const tnt_lanczos_params& p, std::vector<LanczosOut>& out, Timers* tm) {
  lanczos_core(c, *b.op, b.seg, b.n, K, x, p, out, tm);
}

}  // namespace tnt
