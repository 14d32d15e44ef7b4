// Truncated SVD of a two-site vector (appendix B.1.2) with U(1) sectors.
//
// For every middle charge m = q_a + s1, theta restricted to m is a matrix
// X_m with rows (s1, a) and columns (s2, b).  Its singular vectors are
// obtained from the FP64 Hermitian eigendecomposition of a Gram matrix
// (rocSOLVER zheevd, divide and conquer), built blockwise on the grouped
// MFMA GEMM:
//   absorb RIGHT (A = U, B = S V^+): G = X X^+ ; A = eigenvectors (an exact
//     isometry), B = A^+ X (an exact projection, GEMM);
//   absorb LEFT  (A = U S, B = V^+): G = X^+ X ; B = eigenvectors^+, A = X V.
// The isometric factor is therefore orthonormal to working precision and the
// other factor is the exact projection of theta onto the kept space; the
// singular values are sqrt of the Gram eigenvalues.  Eigenvalues below the
// Gram matrix's rounding floor (n * 4 eps * largest) carry no information and
// are set to zero.  All sectors' values are pooled on the host, sorted and
// cut by the four truncation rules; the centre factor is renormalised to unit
// Frobenius norm on the device.
#include "svd.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <set>

#include "kernels.h"
#include "plan.h"

namespace tnt {

void destroy_blas(void* h) { rocblas_destroy_handle(static_cast<rocblas_handle>(h)); }

static rocblas_handle blas(Ctx& c) {
  if (!c.blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success)
      fail(TNT_E_HIP, "rocblas_create_handle failed");
    c.blas = h;
  }
  rocblas_handle h = static_cast<rocblas_handle>(c.blas);
  if (rocblas_set_stream(h, c.stream) != rocblas_status_success)
    fail(TNT_E_HIP, "rocblas_set_stream failed");
  return h;
}

void* blas_handle(Ctx& c) { return blas(c); }

// Lazily create the side streams (non-blocking, default priority) and their
// rocBLAS handles.
static void ensure_side(Ctx& c) {
  if (c.side[0]) return;
  for (int i = 0; i < Ctx::kSide; ++i) {
    TNT_HIP(hipStreamCreateWithFlags(&c.side[i], hipStreamNonBlocking));
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success)
      fail(TNT_E_HIP, "rocblas_create_handle failed");
    if (rocblas_set_stream(h, c.side[i]) != rocblas_status_success)
      fail(TNT_E_HIP, "rocblas_set_stream failed");
    c.side_blas[i] = h;
  }
  for (auto& e : c.side_ev) TNT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

double trunc_error(const double* lam, int n, int kind) {
  double s = 0;
  if (kind == TNT_ERR_1NORM) {
    for (int i = 0; i < n; ++i) s += std::fabs(lam[i]);
    return s;
  }
  for (int i = 0; i < n; ++i) s += lam[i] * lam[i];
  return kind == TNT_ERR_SUMSQ ? s : std::sqrt(s);
}

int trunc_select(const double* lam, int n, const tnt_trunc_params& p, double* eps) {
  if (n <= 0) {
    if (eps) *eps = 0;
    return 0;
  }
  int chi = std::min(p.chi_max, n);
  if (p.abs_tol > 0) {
    int k = 0;
    while (k < n && lam[k] >= p.abs_tol) ++k;
    chi = std::min(chi, k);
  }
  if (p.rel_tol > 0) {
    int k = 0;
    while (k < n && lam[k] / lam[0] >= p.rel_tol) ++k;
    chi = std::min(chi, k);
  }
  if (p.err_tol > 0) {
    // smallest k whose discarded tail lam[k..n) has error strictly below err_tol
    int best = n;
    for (int k = n; k >= 0; --k) {
      if (trunc_error(lam + k, n - k, p.err_type) < p.err_tol) best = k;
      else break;
    }
    chi = std::min(chi, best);
  }
  chi = std::max(chi, 1);
  if (eps) *eps = trunc_error(lam + chi, n - chi, p.err_type);
  return chi;
}

SiteH make_site(const Bond& left, const Bond& right, int d) {
  SiteH h;
  int64_t off = 0;
  for (auto& l : left)
    for (int s = 0; s < d; ++s) {
      auto it = right.find(l.first + s);
      if (it == right.end()) continue;
      h.blocks[{l.first, s}] = BlockRef{off, l.second, it->second};
      off += (int64_t)l.second * it->second;
    }
  h.elems = off;
  return h;
}

namespace {
struct Sector {
  int m = 0;
  std::vector<std::pair<int, int>> rows, cols;  // (s1, q_a), (s2, q_b) ascending
  std::vector<int> roff, coff;
  int R = 0, C = 0;
  int n = 0;             // Gram dimension (R for absorb right, C for absorb left)
  int64_t gbase = 0;     // offset of the n x n Gram matrix (elements / complex elements)
  int ebase = 0;         // offset of its eigenvalues
  int kept = 0;
  int64_t tbase = 0;     // offset of V_kept (C x kept) in the left-absorb temp
};

// Sectors from the blocks present: rows (s1, q_a), columns (s2, q_b).
std::vector<Sector> sectors_of(const ThetaH& th) {
  std::map<int, std::set<std::pair<int, int>>> rows, cols;
  for (auto& kv : th.blocks) {
    const int qa = kv.first[0], s1 = kv.first[1], s2 = kv.first[2];
    const int m = qa + s1;
    rows[m].insert({s1, qa});
    cols[m].insert({s2, m + s2});
  }
  std::vector<Sector> out;
  for (auto& kv : rows) {
    Sector s;
    s.m = kv.first;
    s.rows.assign(kv.second.begin(), kv.second.end());
    s.cols.assign(cols[kv.first].begin(), cols[kv.first].end());
    for (auto& r : s.rows) { s.roff.push_back(s.R); s.R += th.left.at(r.second); }
    for (auto& cc : s.cols) { s.coff.push_back(s.C); s.C += th.right.at(cc.second); }
    out.push_back(std::move(s));
  }
  return out;
}

// Batch size class of an n x n sector eigenproblem.
int padded_size(int n) {
  static const int sizes[] = {8,   16,  24,  32,  48,   64,   96,   128,  160,  192,  256,
                              320, 384, 512, 640, 768, 1024, 1280, 1536, 2048, 2560, 3072,
                              4096};
  for (int v : sizes)
    if (n <= v) return v;
  return (n + 511) / 512 * 512;
}

int index_of(const std::vector<std::pair<int, int>>& v, int first) {
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i].first == first) return (int)i;
  return -1;
}
}  // namespace

// State of one theta between the SVD phases.
struct SvdJob {
  ThetaH th;
  const double* re = nullptr;
  const double* im = nullptr;
  bool right = true;
  std::vector<Sector> secs;
  int64_t gsize = 0;  // complex elements of the Gram matrices
  int esize = 0;      // eigenvalues
  DevTables tg;
  DevBuf gram, z, ev, info;
  std::vector<rocblas_int> hinfo;  // per sector, from the batched eigensolve
};


std::shared_ptr<SvdJob> svd_begin(Ctx& c, const ThetaH& th, const double* re, const double* im,
                                  int absorb) {
  if (absorb != TNT_ABSORB_RIGHT && absorb != TNT_ABSORB_LEFT) fail(TNT_E_ARG, "bad absorb");
  auto job = std::make_shared<SvdJob>();
  SvdJob& J = *job;
  J.th = th;
  J.re = re;
  J.im = im;
  J.right = absorb == TNT_ABSORB_RIGHT;
  const bool right = J.right;
  std::vector<Sector>& secs = J.secs;
  secs = sectors_of(th);
  if (secs.empty()) fail(TNT_E_SHAPE, "theta has no sector to decompose");
  int64_t& gsize = J.gsize;
  int& esize = J.esize;
  for (auto& s : secs) {
    s.n = right ? s.R : s.C;
    s.gbase = gsize;
    gsize += (int64_t)s.n * s.n;
    s.ebase = esize;
    esize += s.n;
  }
  // --- Gram matrices (split planes, row-major n x n per sector) -------------
  HostGemm gg;
  for (auto& s : secs) {
    if (right) {
      // conj(X_i X_j^+) = conj(X_i) X_j^T summed over column groups s2
      for (size_t i = 0; i < s.rows.size(); ++i)
        for (size_t j = 0; j < s.rows.size(); ++j) {
          const int s1i = s.rows[i].first, qai = s.rows[i].second;
          const int s1j = s.rows[j].first, qaj = s.rows[j].second;
          gg.add_task(s.gbase + (int64_t)s.roff[i] * s.n + s.roff[j], th.left.at(qai),
                      th.left.at(qaj), s.n);
          for (auto& cc : s.cols) {
            auto a = th.blocks.find({qai, s1i, cc.first});
            auto b = th.blocks.find({qaj, s1j, cc.first});
            if (a == th.blocks.end() || b == th.blocks.end()) continue;
            gg.add_seg(a->second.off, a->second.cols, b->second.off, b->second.cols,
                       a->second.cols);
          }
        }
    } else {
      // X_i^+ X_j summed over row groups s1
      for (size_t i = 0; i < s.cols.size(); ++i)
        for (size_t j = 0; j < s.cols.size(); ++j) {
          const int s2i = s.cols[i].first, s2j = s.cols[j].first;
          gg.add_task(s.gbase + (int64_t)s.coff[i] * s.n + s.coff[j],
                      th.right.at(s.cols[i].second), th.right.at(s.cols[j].second), s.n);
          for (auto& rr : s.rows) {
            auto a = th.blocks.find({rr.second, rr.first, s2i});
            auto b = th.blocks.find({rr.second, rr.first, s2j});
            if (a == th.blocks.end() || b == th.blocks.end()) continue;
            gg.add_seg(a->second.off, a->second.cols, b->second.off, b->second.cols,
                       a->second.rows);
          }
        }
    }
  }
  gg.finalize(default_tile_cfg(gg, PATH_F64));
  J.tg.upload(c, {&gg}, {});
  J.gram = DevBuf(&c.pool, std::max<int64_t>(1, 2 * gsize) * sizeof(double));
  J.z = DevBuf(&c.pool, std::max<int64_t>(1, 2 * gsize) * sizeof(double));
  J.ev = DevBuf(&c.pool, (size_t)std::max(1, 2 * esize) * sizeof(double));
  J.info = DevBuf(&c.pool, std::max<size_t>(secs.size(), 1) * sizeof(rocblas_int));
  J.hinfo.assign(secs.size(), 0);
  double* g = J.gram.as<double>();
  run_gemm(c, J.tg.g[0], right ? FORM_cNT : FORM_CN, PATH_F64, re, im, ET_F64, re, im, ET_F64, g,
           g + gsize, ET_F64);
  // the row-major buffer read column-major is G (absorb right) or conj(G) (left)
  launch_interleave(g, g + gsize, J.z.as<double>(), gsize, right ? 0 : 1, c.stream);
  return job;
}

void svd_eig(Ctx& c, const std::vector<SvdJob*>& jobs) {
  // Small sectors are solved by cyclic Jacobi in LDS (see below).  For the
  // larger ones each decomposition is a long
  // chain of small, latency-bound launches, so the sectors of all jobs go
  // through a few strided-batched calls
  // (buckets): every sector is padded to its bucket's size (G plus negative
  // eigenvalues below its spectrum, mixed by a fixed reflector so that no
  // exact split remains; see the padding kernels).  The buckets run
  // concurrently on side streams, forked from and joined back into the main
  // stream; G's eigenpairs are extracted back into each job's z and W.
  ensure_side(c);
  struct Ref { SvdJob* job; int sec; };
  struct Bucket {
    int npad = 0;
    std::vector<Ref> secs;
    std::vector<PadTask> tasks;
    DevBuf slots, w, e, tab, info;
  };
  // at most one bucket per side stream (the last stream runs the Jacobi launches)
  constexpr int kMaxBuckets = Ctx::kSide - 1;
  std::vector<Ref> all, small[2];
  auto n_of = [](const Ref& r) { return r.job->secs[r.sec].n; };
  // Small sectors (order <= EIG_SMALL_MAX) go to the Jacobi kernel beside
  // the library calls, in two launches (orders <= 16 and <= 32, so that the
  // smallest take less LDS).
  for (SvdJob* j : jobs)
    for (size_t i = 0; i < j->secs.size(); ++i) {
      const Ref r{j, (int)i};
      const int n = n_of(r);
      if (n <= EIG_SMALL_MAX) small[n <= 16 ? 0 : 1].push_back(r);
      else all.push_back(r);
    }
  std::stable_sort(all.begin(), all.end(),
                   [&](const Ref& a, const Ref& b) { return n_of(a) > n_of(b); });
  // The large sectors form buckets, each one batched library call padded to
  // the size class of its largest sector.  The calls' launch chains are
  // enqueued one after another, so their times add up; a bucket of `cnt`
  // matrices of padded order np is modelled as
  //   latency 0.028 np ms  +  cnt x (0.020 (np / 128)^2.2 ms  for np > 64,
  //                                  0.1 (np / 32)^2 ms      for np <= 64),
  // fitted to timings of the library's batched Hermitian eigensolver on one
  // MI355X (np = 32 .. 256, batches 1 .. 512; at np <= 64 its time grows
  // linearly with the batch).  Few sectors (one chain) give one or two
  // buckets; many sectors (many chains in a step) give more, so that small
  // ones are not padded to the largest.  The bucketing that minimises the
  // modelled time over contiguous runs of size classes (at most
  // kMaxBuckets buckets) is found by dynamic programming.
  auto cost = [](int np, int cnt) {
    const double x = np;
    const double per = np > 64 ? 0.020 * std::pow(x / 128.0, 2.2) : 0.1 * (x / 32.0) * (x / 32.0);
    return 0.028 * x + cnt * per;
  };
  std::vector<std::pair<int, int>> cls;  // (padded order, first index into all), descending
  for (size_t i = 0; i < all.size(); ++i) {
    const int np = padded_size(n_of(all[i]));
    if (cls.empty() || cls.back().first != np) cls.push_back({np, (int)i});
  }
  const int nc = (int)cls.size();
  auto first = [&](int k) { return k < nc ? cls[k].second : (int)all.size(); };
  // best[b][k]: least modelled time of classes [0, k) in b buckets
  const double inf = 1e300;
  std::vector<std::vector<double>> best(kMaxBuckets + 1, std::vector<double>(nc + 1, inf));
  std::vector<std::vector<int>> from(kMaxBuckets + 1, std::vector<int>(nc + 1, -1));
  best[0][0] = 0;
  for (int b = 1; b <= kMaxBuckets; ++b)
    for (int k = 1; k <= nc; ++k)
      for (int a = 0; a < k; ++a) {
        if (best[b - 1][a] >= inf) continue;
        const double v = best[b - 1][a] + cost(cls[a].first, first(k) - first(a));
        if (v < best[b][k]) {
          best[b][k] = v;
          from[b][k] = a;
        }
      }
  int nb = 0;
  for (int b = 1; b <= kMaxBuckets; ++b)
    if (nc > 0 && (nb == 0 || best[b][nc] < best[nb][nc])) nb = b;
  std::vector<Bucket> buckets(nb);
  for (int b = nb, k = nc; b > 0; --b) {
    const int a = from[b][k];
    Bucket& bk = buckets[b - 1];
    bk.npad = cls[a].first;
    for (int i = first(a); i < first(k); ++i) bk.secs.push_back(all[i]);
    k = a;
  }
  TNT_HIP(hipEventRecord(c.side_ev[Ctx::kSide], c.stream));
  bool used[Ctx::kSide] = {};
  // the Jacobi launches go first, on the last side stream, so that they run
  // while the library's launch chains are being enqueued
  struct SmallSet {
    std::vector<PadTask> tasks;
    DevBuf tab, info;
    int maxn = 1;
  } sm[2];
  const int js = Ctx::kSide - 1;
  for (int g = 0; g < 2; ++g) {
    if (small[g].empty()) continue;
    SmallSet& S = sm[g];
    for (const Ref& r : small[g]) {
      SvdJob& J = *r.job;
      const Sector& sc = J.secs[r.sec];
      S.tasks.push_back(PadTask{J.z.as<double>(), J.ev.as<double>(), sc.gbase, 0, 0, sc.ebase,
                                sc.n, sc.n});
      S.maxn = std::max(S.maxn, sc.n);
    }
    S.tab = DevBuf(&c.pool, S.tasks.size() * sizeof(PadTask));
    S.info = DevBuf(&c.pool, S.tasks.size() * sizeof(int));
    if (!used[js]) {
      TNT_HIP(hipStreamWaitEvent(c.side[js], c.side_ev[Ctx::kSide], 0));
      used[js] = true;
    }
    TNT_HIP(hipMemcpyAsync(S.tab.ptr, S.tasks.data(), S.tasks.size() * sizeof(PadTask),
                           hipMemcpyHostToDevice, c.side[js]));
    launch_eig_small(S.tab.as<PadTask>(), (int)S.tasks.size(), S.maxn, S.info.as<int>(),
                     c.side[js]);
  }
  int k = 0;
  for (Bucket& bk : buckets) {
    const int np = bk.npad, cnt = (int)bk.secs.size();
    const int64_t slot = (int64_t)np * np;
    int maxn = 1;
    for (int q = 0; q < cnt; ++q) {
      SvdJob& J = *bk.secs[q].job;
      const Sector& sc = J.secs[bk.secs[q].sec];
      bk.tasks.push_back(PadTask{J.z.as<double>(), J.ev.as<double>(), sc.gbase, q * slot,
                                 (int64_t)q * np, sc.ebase, sc.n, np});
      maxn = std::max(maxn, sc.n);
    }
    bk.slots = DevBuf(&c.pool, (size_t)2 * slot * cnt * sizeof(double));
    bk.w = DevBuf(&c.pool, (size_t)np * cnt * sizeof(double));
    // e: the embedding's work vectors (2 np per slot), then heevd's off-diagonals
    bk.e = DevBuf(&c.pool, (size_t)2 * np * cnt * sizeof(double));
    bk.tab = DevBuf(&c.pool, bk.tasks.size() * sizeof(PadTask));
    bk.info = DevBuf(&c.pool, (size_t)cnt * sizeof(rocblas_int));
    hipStream_t ss = c.side[k];
    if (!used[k]) {
      TNT_HIP(hipStreamWaitEvent(ss, c.side_ev[Ctx::kSide], 0));
      used[k] = true;
    }
    TNT_HIP(hipMemcpyAsync(bk.tab.ptr, bk.tasks.data(), bk.tasks.size() * sizeof(PadTask),
                           hipMemcpyHostToDevice, ss));
    launch_pad_embed(bk.tab.as<PadTask>(), cnt, maxn, np, bk.e.as<double>(),
                     bk.slots.as<double>(), ss);
    if (rocsolver_zheevd_strided_batched(
            static_cast<rocblas_handle>(c.side_blas[k]), rocblas_evect_original,
            rocblas_fill_upper, np, reinterpret_cast<rocblas_double_complex*>(bk.slots.ptr), np,
            slot, bk.w.as<double>(), np, bk.e.as<double>(), np, bk.info.as<rocblas_int>(),
            cnt) != rocblas_status_success)
      fail(TNT_E_HIP, "rocsolver_zheevd_strided_batched failed");
    launch_pad_extract(bk.tab.as<PadTask>(), cnt, maxn, bk.slots.as<double>(), bk.w.as<double>(),
                       ss);
    k = (k + 1) % (Ctx::kSide - 1);
  }
  for (int q = 0; q < Ctx::kSide; ++q) {
    if (!used[q]) continue;
    TNT_HIP(hipEventRecord(c.side_ev[q], c.side[q]));
    TNT_HIP(hipStreamWaitEvent(c.stream, c.side_ev[q], 0));
  }
  // the buckets (device slots and host task lists) live until here
  TNT_HIP(hipStreamSynchronize(c.stream));
  for (Bucket& bk : buckets) {
    std::vector<rocblas_int> raw(bk.secs.size());
    TNT_HIP(hipMemcpy(raw.data(), bk.info.ptr, raw.size() * sizeof(rocblas_int),
                      hipMemcpyDeviceToHost));
    for (size_t q = 0; q < raw.size(); ++q) bk.secs[q].job->hinfo[bk.secs[q].sec] = raw[q];
  }
  for (int g = 0; g < 2; ++g) {
    if (small[g].empty()) continue;
    std::vector<int> raw(small[g].size());
    TNT_HIP(hipMemcpy(raw.data(), sm[g].info.ptr, raw.size() * sizeof(int),
                      hipMemcpyDeviceToHost));
    for (size_t q = 0; q < raw.size(); ++q) small[g][q].job->hinfo[small[g][q].sec] = raw[q];
  }
}

SvdOut svd_finish(Ctx& c, SvdJob& J, const tnt_trunc_params& p, const FactorAlloc& alloc) {
  if (p.chi_max < 1) fail(TNT_E_ARG, "chi_max must be >= 1");
  const ThetaH& th = J.th;
  const double* re = J.re;
  const double* im = J.im;
  const bool right = J.right;
  std::vector<Sector>& secs = J.secs;
  const int64_t gsize = J.gsize;
  const int esize = J.esize;
  DevBuf& z = J.z;
  DevBuf& info = J.info;
  double* g = J.gram.as<double>();
  double* W = J.ev.as<double>();
  rocblas_handle h = blas(c);
  std::vector<double> mu(esize);
  std::vector<rocblas_int>& hinfo = J.hinfo;
  TNT_HIP(hipMemcpyAsync(mu.data(), W, esize * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  // divide and conquer can fail on large clusters of (near-)zero eigenvalues;
  // redo such a sector with the Jacobi eigensolver from the kept Gram planes
  for (size_t i = 0; i < secs.size(); ++i) {
    if (hinfo[i] == 0) continue;
    const Sector& s = secs[i];
    DevBuf rj(&c.pool, 64);
    auto* A = reinterpret_cast<rocblas_double_complex*>(z.as<double>()) + s.gbase;
    launch_interleave(g + s.gbase, g + gsize + s.gbase, z.as<double>() + 2 * s.gbase,
                      (int64_t)s.n * s.n, right ? 0 : 1, c.stream);
    if (rocsolver_zheevj(h, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_upper,
                         s.n, A, s.n, 0.0, rj.as<double>(), 100, rj.as<rocblas_int>() + 4,
                         W + s.ebase, info.as<rocblas_int>() + i) != rocblas_status_success)
      fail(TNT_E_HIP, "rocsolver_zheevj failed");
    TNT_HIP(hipMemcpyAsync(mu.data() + s.ebase, W + s.ebase, s.n * sizeof(double),
                           hipMemcpyDeviceToHost, c.stream));
    TNT_HIP(hipMemcpyAsync(&hinfo[i], info.as<rocblas_int>() + i, sizeof(rocblas_int),
                           hipMemcpyDeviceToHost, c.stream));
    TNT_HIP(hipStreamSynchronize(c.stream));
    if (hinfo[i] != 0) fail(TNT_E_HIP, "eigensolver did not converge in a sector");
  }
  double mumax = 0;
  int nmax = 1;
  for (double v : mu) {
    if (!std::isfinite(v)) fail(TNT_E_NONFINITE, "non-finite Gram eigenvalue (theta not finite?)");
    mumax = std::max(mumax, v);
  }
  for (auto& s : secs) nmax = std::max(nmax, s.n);
  if (!(mumax > 0)) fail(TNT_E_NONFINITE, "theta has zero norm");
  const double floor = 4.0 * 2.220446049250313e-16 * nmax * mumax;
  // pool (lambda desc, then sector asc, then index asc), select
  struct Ent { double lam; int sec, idx; };
  std::vector<Ent> pool;
  pool.reserve(esize);
  for (size_t i = 0; i < secs.size(); ++i) {
    const Sector& s = secs[i];
    const int K = std::min(s.R, s.C);  // rank bound: at most K nonzero singular values
    for (int k = 0; k < K; ++k) {
      const double m = mu[s.ebase + s.n - 1 - k];  // descending
      pool.push_back({m > floor ? std::sqrt(m) : 0.0, (int)i, k});
    }
  }
  std::stable_sort(pool.begin(), pool.end(), [](const Ent& a, const Ent& b) {
    if (a.lam != b.lam) return a.lam > b.lam;
    if (a.sec != b.sec) return a.sec < b.sec;
    return a.idx < b.idx;
  });
  std::vector<double> sorted(pool.size());
  for (size_t i = 0; i < pool.size(); ++i) sorted[i] = pool[i].lam;
  SvdOut out;
  double eps = 0;
  const int chi = trunc_select(sorted.data(), (int)sorted.size(), p, &eps);
  double nk = 0;
  for (int i = 0; i < chi; ++i) {
    nk += sorted[i] * sorted[i];
    secs[pool[i].sec].kept++;
  }
  nk = std::sqrt(nk);
  out.chi = chi;
  out.eps = eps;
  out.lambda0 = sorted.empty() ? 0 : sorted[0];
  out.norm_kept = nk;
  const double scale = p.renormalise && nk > 0 ? 1.0 / nk : 1.0;
  for (auto& s : secs) {
    if (s.kept == 0) continue;
    out.bond[s.m] = s.kept;
    for (int k = 0; k < s.kept; ++k) {
      const double m = mu[s.ebase + s.n - 1 - k];
      out.lam.push_back((m > floor ? std::sqrt(m) : 0.0) * scale);
    }
  }
  // factor layouts: A blocks (q_a, s1) ascending, B blocks (m, s2) ascending
  {
    std::map<std::pair<int, int>, std::pair<int, int>> ablk, bblk;
    for (auto& s : secs) {
      if (s.kept == 0) continue;
      for (auto& r : s.rows) ablk[{r.second, r.first}] = {th.left.at(r.second), s.kept};
      for (auto& cc : s.cols) bblk[{s.m, cc.first}] = {s.kept, th.right.at(cc.second)};
    }
    int64_t off = 0;
    for (auto& kv : ablk) {
      out.A.blocks[kv.first] = BlockRef{off, kv.second.first, kv.second.second};
      off += (int64_t)kv.second.first * kv.second.second;
    }
    out.A.elems = off;
    off = 0;
    for (auto& kv : bblk) {
      out.B.blocks[kv.first] = BlockRef{off, kv.second.first, kv.second.second};
      off += (int64_t)kv.second.first * kv.second.second;
    }
    out.B.elems = off;
  }
  const FactorPlanes fp = alloc(out);
  // --- factors -----------------------------------------------------------
  const double* zz = z.as<double>();
  std::vector<ScatterTask> st;
  int mr = 1, mc = 1;
  auto add_st = [&](int64_t src, int64_t rs, int64_t cs, int64_t dst, int rows, int cols,
                    int conj) {
    st.push_back(ScatterTask{src, rs, cs, dst, rows, cols, conj, 0});
    mr = std::max(mr, rows);
    mc = std::max(mc, cols);
  };
  HostGemm gp;  // projection: the non-isometric factor
  DevBuf tmp;
  int64_t tsize = 0;
  if (right) {
    // A(q_a, s1)[r, c] = eigvec(roff + r, n - 1 - c)
    for (auto& s : secs) {
      if (s.kept == 0) continue;
      for (size_t i = 0; i < s.rows.size(); ++i) {
        const BlockRef& b = out.A.blocks.at({s.rows[i].second, s.rows[i].first});
        add_st(s.gbase + s.roff[i] + (int64_t)(s.n - 1) * s.n, 1, -(int64_t)s.n, b.off, b.rows,
               b.cols, 0);
      }
      // B(m, s2) = sum_{s1} A(q_a, s1)^+ theta(q_a, s1, s2)
      for (size_t j = 0; j < s.cols.size(); ++j) {
        const int s2 = s.cols[j].first;
        const BlockRef& ob = out.B.blocks.at({s.m, s2});
        gp.add_task(ob.off, ob.rows, ob.cols, ob.cols);
        for (auto& rr : s.rows) {
          auto tb = th.blocks.find({rr.second, rr.first, s2});
          if (tb == th.blocks.end()) continue;
          const BlockRef& ab = out.A.blocks.at({rr.second, rr.first});
          gp.add_seg(ab.off, ab.cols, tb->second.off, tb->second.cols, ab.rows);
        }
      }
    }
  } else {
    // the interleave conjugated the row-major X^+ X back into G = X^+ X, so the
    // eigenvectors are the columns of V:  B(m, s2)[r, c] = conj(V(coff + c, n - 1 - r))
    for (auto& s : secs) {
      if (s.kept == 0) continue;
      s.tbase = tsize;
      tsize += (int64_t)s.C * s.kept;
      for (size_t j = 0; j < s.cols.size(); ++j) {
        const BlockRef& b = out.B.blocks.at({s.m, s.cols[j].first});
        add_st(s.gbase + s.coff[j] + (int64_t)(s.n - 1) * s.n, -(int64_t)s.n, 1, b.off, b.rows,
               b.cols, 1);
      }
    }
  }
  const size_t nfac = st.size();
  if (!right) {
    // V_kept row-major (C x kept): V_kept(r, c) = V(r, n - 1 - c)
    for (auto& s : secs) {
      if (s.kept == 0) continue;
      add_st(s.gbase + (int64_t)(s.n - 1) * s.n, 1, -(int64_t)s.n, s.tbase, s.C, s.kept, 0);
      // A(q_a, s1) = sum_{s2} theta(q_a, s1, s2) V_kept[(s2, b) rows]
      for (auto& rr : s.rows) {
        const BlockRef& ab = out.A.blocks.at({rr.second, rr.first});
        gp.add_task(ab.off, ab.rows, ab.cols, ab.cols);
        for (size_t j = 0; j < s.cols.size(); ++j) {
          auto tb = th.blocks.find({rr.second, rr.first, s.cols[j].first});
          if (tb == th.blocks.end()) continue;
          gp.add_seg(tb->second.off, tb->second.cols, s.tbase + (int64_t)s.coff[j] * s.kept,
                     s.kept, tb->second.cols);
        }
      }
    }
    tmp = DevBuf(&c.pool, std::max<int64_t>(1, 2 * tsize) * sizeof(double));
  }
  gp.finalize(default_tile_cfg(gp, PATH_F64));
  DevBuf stab(&c.pool, std::max<size_t>(st.size(), 1) * sizeof(ScatterTask));
  if (!st.empty())
    TNT_HIP(hipMemcpyAsync(stab.ptr, st.data(), st.size() * sizeof(ScatterTask),
                           hipMemcpyHostToDevice, c.stream));
  const ScatterTask* sdev = stab.as<ScatterTask>();
  DevTables tp;
  tp.upload(c, {&gp}, {});
  DevBuf part(&c.pool, (RED_BLOCKS + 8) * sizeof(double));
  double* centre;
  int64_t centre_n;
  if (right) {
    launch_scatter_z(sdev, (int)nfac, mr, mc, zz, fp.a_re, fp.a_im, c.stream);
    run_gemm(c, tp.g[0], FORM_CN, PATH_F64, fp.a_re, fp.a_im, ET_F64, re, im, ET_F64, fp.b_re,
             fp.b_im, ET_F64);
    centre = fp.b_re;
    centre_n = out.B.elems;
  } else {
    double* t = tmp.as<double>();
    launch_scatter_z(sdev, (int)nfac, mr, mc, zz, fp.b_re, fp.b_im, c.stream);
    launch_scatter_z(sdev + nfac, (int)(st.size() - nfac), mr, mc, zz, t, t + tsize, c.stream);
    run_gemm(c, tp.g[0], FORM_NN, PATH_F64, re, im, ET_F64, t, t + tsize, ET_F64, fp.a_re,
             fp.a_im, ET_F64);
    centre = fp.a_re;
    centre_n = out.A.elems;
  }
  if (p.renormalise) {
    // unit Frobenius norm of the centre factor (re and im planes are separate)
    double* pp = part.as<double>();
    const double* cim = right ? fp.b_im : fp.a_im;
    launch_norm2_partial(centre, centre_n, pp, c.stream);
    launch_reduce_partials(pp, 1, RED_BLOCKS, pp + RED_BLOCKS, c.stream);
    launch_norm2_partial(cim, centre_n, pp, c.stream);
    launch_reduce_partials(pp, 1, RED_BLOCKS, pp + RED_BLOCKS + 1, c.stream);
    double nn[2] = {0, 0};
    TNT_HIP(hipMemcpyAsync(nn, pp + RED_BLOCKS, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           c.stream));
    TNT_HIP(hipStreamSynchronize(c.stream));
    const double f = 1.0 / std::sqrt(nn[0] + nn[1]);
    if (!std::isfinite(f)) fail(TNT_E_NONFINITE, "kept part of theta has zero norm");
    launch_scale_host(centre, centre_n, f, c.stream);
    launch_scale_host(const_cast<double*>(cim), centre_n, f, c.stream);
  }
  // the host task vectors above must outlive the asynchronous copies
  TNT_HIP(hipStreamSynchronize(c.stream));
  return out;
}

SvdOut svd_truncate_dev(Ctx& c, const ThetaH& th, const double* re, const double* im,
                        const tnt_trunc_params& p, int absorb, const FactorAlloc& alloc) {
  if (p.chi_max < 1) fail(TNT_E_ARG, "chi_max must be >= 1");
  auto job = svd_begin(c, th, re, im, absorb);
  svd_eig(c, {job.get()});
  return svd_finish(c, *job, p, alloc);
}

}  // namespace tnt
