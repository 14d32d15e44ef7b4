// Truncated SVD of a two-site vector (appendix B.1.2) with U(1) sectors.
//
// For every middle charge m = q_a + s1, theta restricted to m is a matrix
// X_m with rows (s1, a) and columns (s2, b).  Its singular vectors are
// obtained from FP64 Hermitian eigendecompositions, built blockwise on the
// grouped MFMA GEMM:
//   absorb RIGHT (A = U, B = S V^+): G = X X^+ ; A = eigenvectors (an exact
//     isometry), B = A^+ X (an exact projection, GEMM);
//   absorb LEFT  (A = U S, B = V^+): G = X^+ X ; B = eigenvectors^+, A = X V.
// The isometric factor is orthonormal to working precision and the other
// factor is the exact projection of theta onto the kept space.
//
// Singular values by deflation.  An eigenvalue of G carries an absolute
// error of about eps |G| = eps sigma_0^2, so sqrt of a Gram eigenvalue says
// nothing about a singular value below ~1e-7 sigma_0.  Instead, with U the
// eigenvectors, the rows of B = U^+ Y (Y = X, or X^+ for LEFT) are taken:
// the norm of row i is sigma_i to about eps sigma_0 absolute whenever its
// eigenvalue lies well above the rounding band (its vector then mixes with
// the others only by ~eps |G| / gap).  The rows whose eigenvalue lies below
// tau mu_max (the "cluster") span the small-value subspace to the same
// accuracy but are mixed among themselves, so they form the next level's
// problem: B_c (cluster rows) has the cluster's singular values, and the
// Gram matrix B_c B_c^+ is decomposed again with a rounding band scaled by
// its own, much smaller, norm.  Before that, B_c is orthogonalised (twice)
// against the normalised resolved rows of every level so far: a cluster
// vector mixes with a resolved direction j by ~eps mu_max / mu_j, which puts
// a component of size eps sigma_0^2 / sigma_j along that row's direction
// into B_c (~1e-11 sigma_0 for sigma_j just above the threshold); it lies in
// the span of the resolved rows, so the projection removes it and the small
// values keep an absolute accuracy of ~eps sigma_0.  Levels repeat until the truncation rules can
// be decided (the cut lies above every unresolved cluster, whose exact sum
// of squares |B_c|_F^2 then enters the truncation error) or the cluster is at
// the noise level of the projection.  The kept vectors of level L are
// Q_L U_L[:, i], with Q_L the product of the earlier levels' cluster bases.
// All sectors' values are pooled on the host, sorted and cut by the four
// truncation rules; the centre factor is renormalised to unit Frobenius norm
// on the device.
#include "svd.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <limits>
#include <numeric>
#include <set>

#include "kernels.h"
#include "plan.h"

namespace tnt {

void destroy_blas(void* h) { rocblas_destroy_handle(static_cast<rocblas_handle>(h)); }

int64_t blas_workspace_bytes(const Ctx& c) {
  int64_t total = 0;
  auto add = [&](void* h) {
    size_t b = 0;
    if (h && rocblas_get_device_memory_size(static_cast<rocblas_handle>(h), &b) ==
                 rocblas_status_success)
      total += (int64_t)b;
  };
  add(c.blas);
  for (void* h : c.side_blas) add(h);
  return total;
}

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
constexpr double kEps = 2.220446049250313e-16;
// Eigenvalues below kTau * (largest of the level) form the next level.  The
// eigensolver's backward error b is ~6e-16 |G| at unit scale and order 100,
// ~2e-15 |G| at order 1000 (measured), and a resolved value's row norm has a
// relative error of about (b / kTau)^2 from mixing with the cluster: with
// kTau = 1e-10, 4e-10 at the threshold (~4e-15 sigma_0 absolute), falling
// 100-fold per decade above it.
constexpr double kTau = 1e-10;
constexpr int kMaxLevels = 4;

// One level of a sector's deflated eigendecomposition.  Level 0 is the Gram
// matrix of theta's sector; level L >= 1 is the Gram matrix of the previous
// level's cluster rows.  Matrices are interleaved complex, column-major.
struct Level {
  int n = 0;                  // order of the eigenproblem
  DevBuf buf;                 // level >= 1: U (n x n), Z (nother x n), Q (ngram x n, L >= 2), w
  double* U = nullptr;        // eigenvectors (ld n), ascending eigenvalues
  double* w = nullptr;        // eigenvalues (device)
  double* Z = nullptr;        // B^+ = (U^+ Y)^+ (ld nother): column i has norm sigma_i
  const double* Q = nullptr;  // basis of this level's index space (ld ngram); null at level 0
  std::vector<double> mu;     // host: eigenvalues, ascending
  std::vector<double> s2;     // host: squared column norms of Z
  int clus = 0;               // indices [0, clus) unresolved (the next level's problem)
  double bound = 0;           // upper bound of the cluster's singular values
  double fro2 = 0;            // sum of squares of the cluster's singular values
  int info = 0;
};

struct Sector {
  int m = 0;
  std::vector<std::pair<int, int>> rows, cols;  // (s1, q_a), (s2, q_b) ascending
  std::vector<int> roff, coff;
  int R = 0, C = 0;
  int n = 0;             // Gram dimension (R for absorb right, C for absorb left)
  int nother = 0;        // the other dimension
  int64_t gbase = 0;     // offset of the n x n Gram matrix (complex elements)
  int ebase = 0;         // offset of its eigenvalues
  int64_t zbase = 0;     // offset of level 0's Z (nother x n) in the job's zb buffer
  double sigma0 = 0;     // largest singular value of the sector
  std::vector<Level> lv;
  DevBuf vres;           // normalised resolved directions of all levels (nother x nres)
  int nres = 0;
  bool open = false;     // the last level has an unresolved cluster
  bool noise = false;    // refinement stopped at the noise level
  // resolved spectrum, descending: (value, level, index in that level)
  struct Val { double lam; int level, idx; };
  std::vector<Val> vals;
  int kept = 0;
  int64_t ukbase = 0;    // offset of the kept isometric vectors (n x kept) in the job's uk
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

// One Hermitian eigenproblem of a batch: the n x n matrix at z + 2 zoff
// (interleaved, column-major, upper triangle read) is replaced by its
// eigenvectors and its ascending eigenvalues go to w + woff.  `rebuild`
// writes the input matrix again (for the fallback solver).
struct EigProb {
  double* z = nullptr;
  double* w = nullptr;
  int64_t zoff = 0;
  int64_t woff = 0;
  int n = 0;
  int* info = nullptr;
  std::function<void()> rebuild;
};

rocblas_double_complex* zc(double* p) { return reinterpret_cast<rocblas_double_complex*>(p); }
const rocblas_double_complex* zc(const double* p) {
  return reinterpret_cast<const rocblas_double_complex*>(p);
}

// C = alpha op(A) op(B) + beta C (interleaved complex, column-major)
void zgemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
           const double* A, int lda, const double* B, int ldb, double* C, int ldc,
           double alpha = 1.0, double beta = 0.0) {
  if (m <= 0 || n <= 0) return;
  const rocblas_double_complex a{alpha, 0.0}, b{beta, 0.0};
  if (k <= 0) fail(TNT_E_ARG, "empty inner dimension in an SVD product");
  if (rocblas_zgemm(h, ta, tb, m, n, k, &a, zc(A), lda, zc(B), ldb, &b, zc(C), ldc) !=
      rocblas_status_success)
    fail(TNT_E_HIP, "rocblas_zgemm failed");
}
// Tiles of several independent products C = op(A) B or C -= op(A) B
// (interleaved complex, column-major), run as one grouped launch on the
// context's stream.  The object (its host table) must live until that stream
// has been synchronised.
struct ZGroup {
  std::vector<ZTask> t;
  DevBuf tab;
  void add(int opa, bool sub, int m, int n, int k, const double* A, int lda, const double* B,
           int ldb, double* C, int ldc) {
    if (m <= 0 || n <= 0) return;
    if (k <= 0) fail(TNT_E_ARG, "empty inner dimension in an SVD product");
    for (int j0 = 0; j0 < n; j0 += 64)
      for (int i0 = 0; i0 < m; i0 += 64)
        t.push_back(ZTask{A, B, C, m, n, k, lda, ldb, ldc, i0, j0, opa, sub ? 1 : 0});
  }
  void run(Ctx& c) {
    if (t.empty()) return;
    tab = DevBuf(&c.pool, t.size() * sizeof(ZTask));
    TNT_HIP(hipMemcpyAsync(tab.ptr, t.data(), t.size() * sizeof(ZTask), hipMemcpyHostToDevice,
                           c.stream));
    launch_zgemm_grouped(tab.as<ZTask>(), (int)t.size(), c.stream);
  }
};
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
  int64_t zsize = 0;  // complex elements of the level-0 projections
  DevTables tg;
  DevBuf gram, z, ev, zb;
  int levels = 1;
  bool open = false;              // refinement still needed
  double extra_tail = 0;          // sum of squares of the unresolved (discarded) clusters
};

int svd_levels(const SvdJob& job) { return job.levels; }

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
    s.nother = right ? s.C : s.R;
    s.gbase = gsize;
    gsize += (int64_t)s.n * s.n;
    s.ebase = esize;
    esize += s.n;
    s.zbase = J.zsize;
    J.zsize += (int64_t)s.n * s.nother;
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
  double* g = J.gram.as<double>();
  run_gemm(c, J.tg.g[0], right ? FORM_cNT : FORM_CN, PATH_F64, re, im, ET_F64, re, im, ET_F64, g,
           g + gsize, ET_F64);
  // the row-major buffer read column-major is G (absorb right) or conj(G) (left)
  launch_interleave(g, g + gsize, J.z.as<double>(), gsize, right ? 0 : 1, c.stream);
  return job;
}

// Eigenpairs of cnt Hermitian matrices of order np (b.A, full storage):
// tridiagonal form by the panel kernels (trd.hip) with one complex GEMM per
// panel for the trailing update, then per matrix the library's tridiagonal
// divide and conquer (eigenvalues ascending into b.d, eigenvectors of T into
// z) and its back-transformation z <- Q z with the reflectors left in b.A.
static void trd_eig_bucket(rocblas_handle h, hipStream_t s, const TrdBatch& b, int cnt,
                           double* z, rocblas_int* info) {
  const int np = b.np;
  const rocblas_double_complex m1{-1.0, 0.0}, p1{1.0, 0.0};
  for (int j0 = 0; j0 < np; j0 += TRD_NB) {
    const int nbp = std::min(TRD_NB, np - j0);
    for (int i = 0; i < nbp; ++i) {
      launch_trd_column(b, cnt, j0, nbp, i, 1, s);
      if (j0 + i < np - 1) launch_trd_gemv(b, cnt, j0 + i, i, nbp, s);
    }
    const int t0 = j0 + nbp;
    if (t0 >= np) continue;
    launch_trd_column(b, cnt, j0, nbp, nbp, 0, s);
    // A(t0:, t0:) -= [V W] [W V]^H
    const int mt = np - t0;
    auto* X = reinterpret_cast<rocblas_double_complex*>(b.X);
    auto* A = reinterpret_cast<rocblas_double_complex*>(b.A);
    if (rocblas_zgemm_strided_batched(h, rocblas_operation_none,
                                      rocblas_operation_conjugate_transpose, mt, mt, 2 * nbp, &m1,
                                      X + t0, np, b.sX, X + t0 + (int64_t)nbp * np, np, b.sX,
                                      &p1, A + t0 + (int64_t)t0 * np, np, b.sA,
                                      cnt) != rocblas_status_success)
      fail(TNT_E_HIP, "rocblas_zgemm_strided_batched failed");
  }
  for (int q = 0; q < cnt; ++q) {
    auto* zq = reinterpret_cast<rocblas_double_complex*>(z) + (int64_t)q * b.sA;
    if (rocsolver_zstedc(h, rocblas_evect_tridiagonal, np, b.d + q * b.sd, b.e + q * b.se, zq,
                         np, info + q) != rocblas_status_success)
      fail(TNT_E_HIP, "rocsolver_zstedc failed");
    if (rocsolver_zunmtr(h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, np,
                         np, reinterpret_cast<rocblas_double_complex*>(b.A + q * b.sA), np,
                         reinterpret_cast<rocblas_double_complex*>(b.tau + q * b.stau), zq,
                         np) != rocblas_status_success)
      fail(TNT_E_HIP, "rocsolver_zunmtr failed");
  }
}

// Eigendecompositions of a batch of Hermitian matrices of any orders.
static void eig_batch(Ctx& c, std::vector<EigProb>& probs) {
  // Small problems are solved by cyclic Jacobi in LDS (see below).  For the
  // larger ones each decomposition is a long chain of small, latency-bound
  // launches, so the problems go through a few strided-batched calls
  // (buckets): every matrix is padded to its bucket's size (the matrix plus
  // negative eigenvalues below its spectrum, mixed by a fixed reflector so
  // that no exact split remains; see the padding kernels).  The buckets run
  // concurrently on side streams, forked from and joined back into the main
  // stream; the eigenpairs are extracted back into each problem's buffers.
  ensure_side(c);
  struct Bucket {
    int npad = 0;
    std::vector<int> ids;
    std::vector<PadTask> tasks;
    DevBuf slots, w, e, tab, info, sc;
    DevBuf X, yp, tp, tau, zv;  // own tridiagonal reduction (trd_eig_bucket)
  };
  constexpr int kMaxBuckets = Ctx::kSide - 1;
  std::vector<int> all, small[2];
  for (size_t i = 0; i < probs.size(); ++i) {
    const int n = probs[i].n;
    if (n <= 0) continue;
    if (n <= EIG_SMALL_MAX) small[n <= 16 ? 0 : 1].push_back((int)i);
    else all.push_back((int)i);
  }
  std::stable_sort(all.begin(), all.end(),
                   [&](int a, int b) { return probs[a].n > probs[b].n; });
  // A bucket of `cnt` matrices of padded order np is modelled as
  //   latency 0.028 np ms  +  cnt x (0.020 (np / 128)^2.2 ms  for np > 64,
  //                                  0.1 (np / 32)^2 ms      for np <= 64),
  // fitted to timings of the library's batched Hermitian eigensolver on one
  // MI355X (np = 32 .. 256, batches 1 .. 512; at np <= 64 its time grows
  // linearly with the batch).  The bucketing that minimises the modelled
  // time over contiguous runs of size classes (at most kMaxBuckets buckets)
  // is found by dynamic programming.
  auto cost = [](int np, int cnt) {
    const double x = np;
    const double per = np > 64 ? 0.020 * std::pow(x / 128.0, 2.2) : 0.1 * (x / 32.0) * (x / 32.0);
    return 0.028 * x + cnt * per;
  };
  std::vector<std::pair<int, int>> cls;  // (padded order, first index into all), descending
  for (size_t i = 0; i < all.size(); ++i) {
    const int np = padded_size(probs[all[i]].n);
    if (cls.empty() || cls.back().first != np) cls.push_back({np, (int)i});
  }
  const int nc = (int)cls.size();
  auto first = [&](int k) { return k < nc ? cls[k].second : (int)all.size(); };
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
    for (int i = first(a); i < first(k); ++i) bk.ids.push_back(all[i]);
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
    for (int id : small[g]) {
      const EigProb& P = probs[id];
      S.tasks.push_back(PadTask{P.z, P.w, P.zoff, 0, 0, P.woff, P.n, P.n, nullptr});
      S.maxn = std::max(S.maxn, P.n);
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
    const int np = bk.npad, cnt = (int)bk.ids.size();
    const int64_t slot = (int64_t)np * np;
    int maxn = 1;
    bk.sc = DevBuf(&c.pool, (size_t)cnt * sizeof(double));
    for (int q = 0; q < cnt; ++q) {
      const EigProb& P = probs[bk.ids[q]];
      bk.tasks.push_back(PadTask{P.z, P.w, P.zoff, q * slot, (int64_t)q * np, P.woff, P.n, np,
                                 bk.sc.as<double>() + q});
      maxn = std::max(maxn, P.n);
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
    const rocblas_handle hs = static_cast<rocblas_handle>(c.side_blas[k]);
    if (c.eig_trd_min > 0 && np >= c.eig_trd_min && np <= TRD_MAX_N) {
      // the slots keep the reflectors; the eigenvectors go to bk.zv
      bk.X = DevBuf(&c.pool, (size_t)cnt * np * 3 * TRD_NB * sizeof(double2));
      const int64_t nt = (np + 63) / 64;
      bk.yp = DevBuf(&c.pool, (size_t)cnt * nt * np * sizeof(double2));
      bk.tp = DevBuf(&c.pool, (size_t)cnt * nt * 2 * TRD_NB * sizeof(double2));
      bk.tau = DevBuf(&c.pool, (size_t)cnt * np * sizeof(double2));
      bk.zv = DevBuf(&c.pool, (size_t)2 * slot * cnt * sizeof(double));
      TrdBatch b;
      b.A = bk.slots.as<double2>();
      b.sA = slot;
      b.X = bk.X.as<double2>();
      b.sX = (int64_t)np * 3 * TRD_NB;
      b.yp = bk.yp.as<double2>();
      b.sY = nt * np;
      b.tp = bk.tp.as<double2>();
      b.sT = nt * 2 * TRD_NB;
      b.d = bk.w.as<double>();
      b.sd = np;
      b.e = bk.e.as<double>();
      b.se = np;
      b.tau = bk.tau.as<double2>();
      b.stau = np;
      b.np = np;
      trd_eig_bucket(hs, ss, b, cnt, bk.zv.as<double>(), bk.info.as<rocblas_int>());
      launch_pad_extract(bk.tab.as<PadTask>(), cnt, maxn, bk.zv.as<double>(), bk.w.as<double>(),
                         ss);
    } else {
      if (rocsolver_zheevd_strided_batched(
              hs, rocblas_evect_original, rocblas_fill_upper, np,
              reinterpret_cast<rocblas_double_complex*>(bk.slots.ptr), np, slot,
              bk.w.as<double>(), np, bk.e.as<double>(), np, bk.info.as<rocblas_int>(),
              cnt) != rocblas_status_success)
        fail(TNT_E_HIP, "rocsolver_zheevd_strided_batched failed");
      launch_pad_extract(bk.tab.as<PadTask>(), cnt, maxn, bk.slots.as<double>(),
                         bk.w.as<double>(), ss);
    }
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
    std::vector<rocblas_int> raw(bk.ids.size());
    TNT_HIP(hipMemcpy(raw.data(), bk.info.ptr, raw.size() * sizeof(rocblas_int),
                      hipMemcpyDeviceToHost));
    for (size_t q = 0; q < raw.size(); ++q) *probs[bk.ids[q]].info = raw[q];
  }
  for (int g = 0; g < 2; ++g) {
    if (small[g].empty()) continue;
    std::vector<int> raw(small[g].size());
    TNT_HIP(hipMemcpy(raw.data(), sm[g].info.ptr, raw.size() * sizeof(int),
                      hipMemcpyDeviceToHost));
    for (size_t q = 0; q < raw.size(); ++q) *probs[small[g][q]].info = raw[q];
  }
  // divide and conquer can fail on large clusters of (near-)zero eigenvalues,
  // with an error code or with non-finite eigenvectors and a zero code;
  // redo such a problem with the library's Jacobi eigensolver
  std::vector<FiniteTask> ft;
  int64_t ftmax = 0;
  for (size_t i = 0; i < probs.size(); ++i) {
    const EigProb& P = probs[i];
    if (P.n <= 0) continue;
    ft.push_back(FiniteTask{P.z + 2 * P.zoff, 2 * (int64_t)P.n * P.n, (int)i});
    ft.push_back(FiniteTask{P.w + P.woff, P.n, (int)i});
    ftmax = std::max<int64_t>(ftmax, 2 * (int64_t)P.n * P.n);
  }
  std::vector<int> bad(probs.size(), 0);
  if (!ft.empty()) {
    DevBuf ftab(&c.pool, ft.size() * sizeof(FiniteTask));
    DevBuf flags(&c.pool, probs.size() * sizeof(int));
    TNT_HIP(hipMemcpyAsync(ftab.ptr, ft.data(), ft.size() * sizeof(FiniteTask),
                           hipMemcpyHostToDevice, c.stream));
    TNT_HIP(hipMemcpyAsync(flags.ptr, bad.data(), bad.size() * sizeof(int),
                           hipMemcpyHostToDevice, c.stream));
    launch_check_finite_batch(ftab.as<FiniteTask>(), (int)ft.size(), ftmax, flags.as<int>(),
                              c.stream);
    TNT_HIP(hipMemcpyAsync(bad.data(), flags.ptr, bad.size() * sizeof(int),
                           hipMemcpyDeviceToHost, c.stream));
    TNT_HIP(hipStreamSynchronize(c.stream));
  }
  rocblas_handle h = blas(c);
  for (size_t i = 0; i < probs.size(); ++i) {
    EigProb& P = probs[i];
    if (P.n <= 0 || (*P.info == 0 && !bad[i])) continue;
    ++c.eig_retries;
    P.rebuild();
    DevBuf rj(&c.pool, 64), inf(&c.pool, sizeof(rocblas_int));
    if (rocsolver_zheevj(h, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_upper,
                         P.n, zc(P.z) + P.zoff, P.n, 0.0, rj.as<double>(), 100,
                         rj.as<rocblas_int>() + 4, P.w + P.woff,
                         inf.as<rocblas_int>()) != rocblas_status_success)
      fail(TNT_E_HIP, "rocsolver_zheevj failed");
    TNT_HIP(hipMemcpyAsync(P.info, inf.ptr, sizeof(rocblas_int), hipMemcpyDeviceToHost,
                           c.stream));
    TNT_HIP(hipStreamSynchronize(c.stream));
    if (*P.info != 0) fail(TNT_E_HIP, "eigensolver did not converge in a sector");
  }
}

void svd_eig(Ctx& c, const std::vector<SvdJob*>& jobs) {
  std::vector<EigProb> probs;
  for (SvdJob* jp : jobs) {
    SvdJob& J = *jp;
    for (Sector& s : J.secs) {
      s.lv.clear();
      s.nres = 0;
      s.lv.reserve(kMaxLevels);  // levels are referenced by address while refining
      s.lv.emplace_back();
      Level& L0 = s.lv[0];
      L0.n = s.n;
      L0.U = J.z.as<double>() + 2 * s.gbase;
      L0.w = J.ev.as<double>() + s.ebase;
      EigProb P;
      P.z = J.z.as<double>();
      P.w = J.ev.as<double>();
      P.zoff = s.gbase;
      P.woff = s.ebase;
      P.n = s.n;
      P.info = &L0.info;
      const double* g = J.gram.as<double>();
      const int64_t gsize = J.gsize, gb = s.gbase, nn = (int64_t)s.n * s.n;
      double* zz = J.z.as<double>();
      const int conj = J.right ? 0 : 1;
      hipStream_t st = c.stream;
      P.rebuild = [=]() { launch_interleave(g + gb, g + gsize + gb, zz + 2 * gb, nn, conj, st); };
      probs.push_back(std::move(P));
    }
  }
  eig_batch(c, probs);
}

namespace {
// Squared column norms of a level's Z, read back with its eigenvalues.
struct NormReads {
  std::vector<ZNormTask> tasks;
  std::vector<std::pair<Level*, int>> dst;  // (level, first column) per run of columns
  std::vector<std::pair<Level*, int64_t>> mu;  // eigenvalues to read
  void add(Level& L, int nother) {
    dst.push_back({&L, (int)tasks.size()});
    for (int i = 0; i < L.n; ++i) tasks.push_back(ZNormTask{L.Z + 2 * (int64_t)i * nother, nullptr, nother});
    mu.push_back({&L, 0});
  }
  void run(Ctx& c) {
    if (tasks.empty()) return;
    DevBuf out(&c.pool, tasks.size() * sizeof(double));
    for (size_t i = 0; i < tasks.size(); ++i) tasks[i].out = out.as<double>() + i;
    DevBuf tab(&c.pool, tasks.size() * sizeof(ZNormTask));
    TNT_HIP(hipMemcpyAsync(tab.ptr, tasks.data(), tasks.size() * sizeof(ZNormTask),
                           hipMemcpyHostToDevice, c.stream));
    launch_znorm2(tab.as<ZNormTask>(), (int)tasks.size(), c.stream);
    std::vector<double> h(tasks.size());
    TNT_HIP(hipMemcpyAsync(h.data(), out.ptr, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c.stream));
    for (auto& m : mu) {
      m.first->mu.resize(m.first->n);
      TNT_HIP(hipMemcpyAsync(m.first->mu.data(), m.first->w, m.first->n * sizeof(double),
                             hipMemcpyDeviceToHost, c.stream));
    }
    TNT_HIP(hipStreamSynchronize(c.stream));
    for (auto& d : dst) {
      Level& L = *d.first;
      L.s2.assign(h.begin() + d.second, h.begin() + d.second + L.n);
    }
  }
};

// After a level's eigenvalues and column norms are known: split off its
// cluster, or close the sector.
void classify(Sector& s, int level) {
  Level& L = s.lv[level];
  const int n = L.n;
  for (double v : L.mu)
    if (!std::isfinite(v)) fail(TNT_E_NONFINITE, "non-finite Gram eigenvalue (theta not finite?)");
  for (double v : L.s2)
    if (!std::isfinite(v)) fail(TNT_E_NONFINITE, "non-finite singular value (theta not finite?)");
  const double mumax = n > 0 ? std::max(0.0, L.mu[n - 1]) : 0.0;
  if (level == 0) s.sigma0 = std::sqrt(mumax);
  int clus = 0;
  if (mumax > 0)
    while (clus < n && L.mu[clus] < kTau * mumax) ++clus;
  L.clus = clus;
  L.fro2 = 0;
  for (int i = 0; i < clus; ++i) L.fro2 += L.s2[i];
  // the cluster's eigenvalues lie below tau mu_max up to the rounding band
  L.bound = clus ? std::sqrt((kTau + 8.0 * kEps) * mumax) : 0.0;
  // the projection itself carries ~eps sigma_0 per singular value; a cluster
  // at that level is noise and is taken as it stands
  const double noise = 8.0 * kEps * std::sqrt((double)std::max(s.n, s.nother)) * s.sigma0;
  if (clus && (L.bound <= noise || level + 1 >= kMaxLevels || mumax <= 0)) {
    L.clus = 0;
    L.fro2 = 0;
    L.bound = 0;
    s.noise = true;
  }
  s.open = L.clus > 0;
}

// The sector's resolved values (all levels so far), descending; a level's
// values never exceed the smallest resolved value of the level above it.
void collect(Sector& s) {
  s.vals.clear();
  double cap = std::numeric_limits<double>::infinity();
  for (int l = 0; l < (int)s.lv.size(); ++l) {
    const Level& L = s.lv[l];
    std::vector<Sector::Val> v;
    for (int i = L.clus; i < L.n; ++i)
      v.push_back({std::min(cap, std::sqrt(std::max(0.0, L.s2[i]))), l, i});
    std::stable_sort(v.begin(), v.end(), [](const Sector::Val& a, const Sector::Val& b) {
      if (a.lam != b.lam) return a.lam > b.lam;
      return a.idx > b.idx;
    });
    for (auto& x : v) s.vals.push_back(x);
    if (!v.empty()) cap = v.back().lam;
  }
  // at most min(R, C) singular values per sector
  const int K = std::min(s.R, s.C);
  if ((int)s.vals.size() > K) s.vals.resize(K);
}

// Whether a value no larger than U is surely discarded, whatever the
// unresolved values are: chi_max resolved values lie above it, or the
// absolute or relative rule cuts above it.  r: resolved values, descending.
bool surely_cut(const std::vector<double>& r, double U, const tnt_trunc_params& p) {
  int cnt = 0;
  while (cnt < (int)r.size() && r[cnt] > U) ++cnt;
  if (cnt >= p.chi_max) return true;
  if (p.abs_tol > 0 && p.abs_tol > U) return true;
  if (p.rel_tol > 0 && !r.empty() && p.rel_tol * r[0] > U) return true;
  return false;
}

// Whether the truncation rules are decided with the sectors' unresolved
// clusters all discarded (every active rule would need a value above the
// clusters' bound to keep one of them).
bool decided(const std::vector<Sector>& secs, const tnt_trunc_params& p, double* extra) {
  double U = 0, f = 0;
  bool any = false;
  std::vector<double> r;
  for (const Sector& s : secs) {
    for (auto& v : s.vals) r.push_back(v.lam);
    if (s.open) {
      any = true;
      U = std::max(U, s.lv.back().bound);
      f += s.lv.back().fro2;
    }
  }
  *extra = f;
  if (!any) return true;
  std::sort(r.begin(), r.end(), std::greater<double>());
  if (surely_cut(r, U, p)) return true;
  if (p.err_tol > 0) {
    // the error rule cuts above every cluster when the tail after the
    // resolved values above U (with the clusters' exact sums) is below e
    if (p.err_type == TNT_ERR_1NORM) return false;
    int cnt = 0;
    while (cnt < (int)r.size() && r[cnt] > U) ++cnt;
    double t = f;
    for (size_t i = cnt; i < r.size(); ++i) t += r[i] * r[i];
    const double err = p.err_type == TNT_ERR_SUMSQ ? t : std::sqrt(t);
    return err < p.err_tol;
  }
  // without the error rule each cluster may be judged by its own bound
  for (const Sector& s : secs)
    if (s.open && !surely_cut(r, s.lv.back().bound, p)) return false;
  return true;
}
}  // namespace

void svd_refine(Ctx& c, const std::vector<SvdJob*>& jobs,
                const std::vector<tnt_trunc_params>& params) {
  if (params.size() != jobs.size()) fail(TNT_E_ARG, "one truncation rule set per theta");
  // --- level 0: Z = B^+ with B = U^+ Y, from theta's blocks ------------------
  NormReads nr;
  for (SvdJob* jp : jobs) {
    SvdJob& J = *jp;
    const ThetaH& th = J.th;
    const bool right = J.right;
    J.levels = 1;
    J.zb = DevBuf(&c.pool, std::max<int64_t>(1, 2 * J.zsize) * sizeof(double));
    // eigenvectors into split planes, row-major: RIGHT U[r][i], LEFT Vt[i][c]
    DevBuf up(&c.pool, std::max<int64_t>(1, 2 * J.gsize) * sizeof(double));
    DevBuf bp(&c.pool, std::max<int64_t>(1, 2 * J.zsize) * sizeof(double));
    std::vector<ScatterTask> st;
    int mr = 1, mc = 1;
    HostGemm gb;
    for (Sector& s : J.secs) {
      if (right) st.push_back(ScatterTask{s.gbase, 1, s.n, s.gbase, s.n, s.n, 0, 0});
      else st.push_back(ScatterTask{s.gbase, s.n, 1, s.gbase, s.n, s.n, 0, 0});
      mr = std::max(mr, s.n);
      mc = std::max(mc, s.n);
      if (right) {
        // B[i, (s2, b)] = sum_r conj(U[r, i]) X[r, (s2, b)]   (n x C, ld C)
        for (size_t j = 0; j < s.cols.size(); ++j) {
          const int s2 = s.cols[j].first;
          gb.add_task(s.zbase + s.coff[j], s.n, th.right.at(s.cols[j].second), s.C);
          for (size_t i = 0; i < s.rows.size(); ++i) {
            auto tb = th.blocks.find({s.rows[i].second, s.rows[i].first, s2});
            if (tb == th.blocks.end()) continue;
            gb.add_seg(s.gbase + (int64_t)s.roff[i] * s.n, s.n, tb->second.off, tb->second.cols,
                       tb->second.rows);
          }
        }
      } else {
        // P[i, (s1, a)] = sum_c V[c, i] X[(s1, a), c] = conj(B[i, (s1, a)])   (n x R, ld R)
        for (size_t i = 0; i < s.rows.size(); ++i) {
          gb.add_task(s.zbase + s.roff[i], s.n, th.left.at(s.rows[i].second), s.R);
          for (size_t j = 0; j < s.cols.size(); ++j) {
            auto tb = th.blocks.find({s.rows[i].second, s.rows[i].first, s.cols[j].first});
            if (tb == th.blocks.end()) continue;
            gb.add_seg(s.gbase + s.coff[j], s.n, tb->second.off, tb->second.cols,
                       tb->second.cols);
          }
        }
      }
    }
    DevBuf stab(&c.pool, st.size() * sizeof(ScatterTask));
    TNT_HIP(hipMemcpyAsync(stab.ptr, st.data(), st.size() * sizeof(ScatterTask),
                           hipMemcpyHostToDevice, c.stream));
    launch_scatter_z(stab.as<ScatterTask>(), (int)st.size(), mr, mc, J.z.as<double>(),
                     up.as<double>(), up.as<double>() + J.gsize, c.stream);
    gb.finalize(default_tile_cfg(gb, PATH_F64));
    DevTables tb;
    tb.upload(c, {&gb}, {});
    double* u = up.as<double>();
    double* b = bp.as<double>();
    run_gemm(c, tb.g[0], right ? FORM_CN : FORM_NT, PATH_F64, u, u + J.gsize, ET_F64, J.re,
             J.im, ET_F64, b, b + J.zsize, ET_F64);
    // RIGHT: B row-major (n x C) read column-major with conj = B^+ (C x n);
    // LEFT: P row-major (n x R) read column-major = P^T = B^+ (R x n)
    launch_interleave(b, b + J.zsize, J.zb.as<double>(), J.zsize, right ? 1 : 0, c.stream);
    for (Sector& s : J.secs) {
      Level& L0 = s.lv[0];
      L0.Z = J.zb.as<double>() + 2 * s.zbase;
      nr.add(L0, s.nother);
    }
    // the host tables and temporaries must outlive the launches
    TNT_HIP(hipStreamSynchronize(c.stream));
  }
  nr.run(c);
  for (size_t q = 0; q < jobs.size(); ++q) {
    SvdJob& J = *jobs[q];
    J.open = false;
    for (Sector& s : J.secs) {
      s.noise = false;
      classify(s, 0);
      collect(s);
    }
    J.open = !decided(J.secs, params[q], &J.extra_tail);
  }
  // --- levels 1, 2, ...: the clusters' Gram matrices --------------------------
  rocblas_handle h = blas(c);
  for (int level = 1; level < kMaxLevels; ++level) {
    // refine the open sectors whose cluster may still hold a kept value; a
    // cluster every rule discards stays unresolved (its exact sum of squares
    // enters the truncation error)
    std::vector<std::pair<SvdJob*, Sector*>> act;
    for (size_t q = 0; q < jobs.size(); ++q) {
      SvdJob* J = jobs[q];
      if (!J->open) continue;
      std::vector<double> r;
      for (const Sector& s : J->secs)
        for (auto& v : s.vals) r.push_back(v.lam);
      std::sort(r.begin(), r.end(), std::greater<double>());
      const bool err_rule = params[q].err_tol > 0;
      for (Sector& s : J->secs)
        if (s.open && (err_rule || !surely_cut(r, s.lv.back().bound, params[q])))
          act.push_back({J, &s});
    }
    if (act.empty()) break;
    // the previous level's resolved rows join the sector's resolved set, and
    // its cluster rows are orthogonalised against the whole set (twice)
    {
      std::vector<ZCopyTask> cp;
      int64_t cpmax = 1;
      for (auto& a : act) {
        Sector& s = *a.second;
        const Level& P = s.lv[level - 1];
        if (!s.vres.ptr)
          s.vres = DevBuf(&c.pool, std::max<size_t>(1, (size_t)2 * s.nother * s.n) * sizeof(double));
        for (int i = P.clus; i < P.n; ++i) {
          if (s.nres >= s.n) fail(TNT_E_STATE, "SVD resolved set exceeds the sector order");
          const double nrm = std::sqrt(P.s2[i]);
          cp.push_back(ZCopyTask{P.Z + 2 * (int64_t)i * s.nother,
                                 s.vres.as<double>() + 2 * (int64_t)s.nres * s.nother, s.nother,
                                 nrm > 0 ? 1.0 / nrm : 0.0});
          cpmax = std::max<int64_t>(cpmax, s.nother);
          ++s.nres;
        }
      }
      DevBuf tab(&c.pool, std::max<size_t>(1, cp.size()) * sizeof(ZCopyTask));
      if (!cp.empty()) {
        TNT_HIP(hipMemcpyAsync(tab.ptr, cp.data(), cp.size() * sizeof(ZCopyTask),
                               hipMemcpyHostToDevice, c.stream));
        launch_zcopy(tab.as<ZCopyTask>(), (int)cp.size(), cpmax, c.stream);
      }
      // T_s = V_s^+ Z_c,s ; Z_c,s -= V_s T_s, every sector in one launch per
      // product (twice)
      std::vector<int64_t> toff(act.size());
      int64_t tsum = 0;
      for (size_t i = 0; i < act.size(); ++i) {
        const Sector& s = *act[i].second;
        toff[i] = tsum;
        tsum += (int64_t)s.nres * s.lv[level - 1].clus;
      }
      DevBuf t(&c.pool, (size_t)2 * std::max<int64_t>(1, tsum) * sizeof(double));
      ZGroup proj[2], upd[2];
      for (int pass = 0; pass < 2; ++pass) {
        for (size_t i = 0; i < act.size(); ++i) {
          Sector& s = *act[i].second;
          Level& P = s.lv[level - 1];
          proj[pass].add(1, false, s.nres, P.clus, s.nother, s.vres.as<double>(), s.nother, P.Z,
                         s.nother, t.as<double>() + 2 * toff[i], s.nres);
          upd[pass].add(0, true, s.nother, P.clus, s.nres, s.vres.as<double>(), s.nother,
                        t.as<double>() + 2 * toff[i], s.nres, P.Z, s.nother);
        }
        proj[pass].run(c);
        upd[pass].run(c);
      }
      // the copies' and products' host tables must outlive the launches
      TNT_HIP(hipStreamSynchronize(c.stream));
    }
    std::vector<EigProb> probs;
    probs.reserve(act.size());
    ZGroup builds;  // Q_L (level >= 2) and the clusters' Gram matrices, one launch
    for (auto& a : act) {
      Sector& s = *a.second;
      if ((int)s.lv.size() != level) fail(TNT_E_STATE, "SVD level bookkeeping");
      s.lv.emplace_back();  // capacity reserved: no reallocation
      const Level& P = s.lv[level - 1];
      const int n = P.clus, no = s.nother, ng = s.n;
      Level& L = s.lv.back();
      L.n = n;
      const int64_t uz = (int64_t)n * n, zz = (int64_t)no * n, qz = level >= 2 ? (int64_t)ng * n : 0;
      L.buf = DevBuf(&c.pool, (size_t)(2 * (uz + zz + qz) + n) * sizeof(double));
      L.U = L.buf.as<double>();
      L.Z = L.U + 2 * uz;
      L.w = L.Z + 2 * zz + 2 * qz;
      if (level == 1) {
        L.Q = s.lv[0].U;  // the first n columns of level 0's eigenvectors
      } else {
        double* Q = L.Z + 2 * zz;  // Q_L = Q_P U_P
        builds.add(0, false, ng, n, P.n, P.Q, ng, P.U, P.n, Q, ng);
        L.Q = Q;
      }
      // G = Z_c^+ Z_c  (the cluster rows' Gram matrix; the fallback solver
      // rebuilds it with the library's product)
      const double* Zc = P.Z;
      double* U = L.U;
      builds.add(1, false, n, n, no, Zc, no, Zc, no, U, n);
      auto build = [=]() {
        zgemm(h, rocblas_operation_conjugate_transpose, rocblas_operation_none, n, n, no, Zc, no,
              Zc, no, U, n);
      };
      EigProb E;
      E.z = L.U;
      E.w = L.w;
      E.n = n;
      E.info = &L.info;
      E.rebuild = build;
      probs.push_back(std::move(E));
    }
    builds.run(c);
    eig_batch(c, probs);  // synchronises the context's stream
    NormReads lr;
    ZGroup zl;
    for (auto& a : act) {
      Sector& s = *a.second;
      Level& P = s.lv[level - 1];
      Level& L = s.lv[level];
      // Z_L = Z_c U_L
      zl.add(0, false, s.nother, L.n, L.n, P.Z, s.nother, L.U, L.n, L.Z, s.nother);
      lr.add(L, s.nother);
    }
    zl.run(c);
    lr.run(c);  // synchronises the context's stream
    for (auto& a : act) {
      classify(*a.second, level);
      collect(*a.second);
    }
    for (size_t q = 0; q < jobs.size(); ++q) {
      SvdJob& J = *jobs[q];
      if (!J.open) continue;
      J.levels = level + 1;
      J.open = !decided(J.secs, params[q], &J.extra_tail);
    }
  }
  for (SvdJob* J : jobs) {
    // whatever is still open after the last level is taken as resolved noise
    if (!J->open) continue;
    for (Sector& s : J->secs) {
      if (!s.open) continue;
      s.lv.back().clus = 0;
      s.lv.back().fro2 = 0;
      s.open = false;
      collect(s);
    }
    J->open = false;
    J->extra_tail = 0;
  }
}

SvdOut svd_finish(Ctx& c, SvdJob& J, const tnt_trunc_params& p, const FactorAlloc& alloc) {
  if (p.chi_max < 1) fail(TNT_E_ARG, "chi_max must be >= 1");
  const ThetaH& th = J.th;
  const double* re = J.re;
  const double* im = J.im;
  const bool right = J.right;
  std::vector<Sector>& secs = J.secs;
  // pool (lambda desc, then sector asc, then in-sector position asc), select
  struct Ent { double lam; int sec, pos; };
  std::vector<Ent> pool;
  for (size_t i = 0; i < secs.size(); ++i) {
    secs[i].kept = 0;
    for (size_t k = 0; k < secs[i].vals.size(); ++k)
      pool.push_back({secs[i].vals[k].lam, (int)i, (int)k});
  }
  if (pool.empty()) fail(TNT_E_NONFINITE, "theta has zero norm");
  std::stable_sort(pool.begin(), pool.end(), [](const Ent& a, const Ent& b) {
    if (a.lam != b.lam) return a.lam > b.lam;
    if (a.sec != b.sec) return a.sec < b.sec;
    return a.pos < b.pos;
  });
  if (!(pool[0].lam > 0)) fail(TNT_E_NONFINITE, "theta has zero norm");
  std::vector<double> sorted(pool.size());
  for (size_t i = 0; i < pool.size(); ++i) sorted[i] = pool[i].lam;
  SvdOut out;
  out.levels = J.levels;
  // the unresolved clusters are discarded: their exact sum of squares joins
  // every tail of the error rule and the reported error
  const double extra = J.extra_tail;
  int chi;
  double eps = 0;
  if (extra > 0) {
    tnt_trunc_params q = p;
    if (q.err_tol > 0) {
      // error rule with the clusters in every tail
      const int n = (int)sorted.size();
      int best = n;
      for (int k = n; k >= 0; --k) {
        double t = extra;
        for (int i = k; i < n; ++i) t += sorted[i] * sorted[i];
        const double e = q.err_type == TNT_ERR_SUMSQ ? t : std::sqrt(t);
        if (e < q.err_tol) best = k;
        else break;
      }
      q.err_tol = -1;
      chi = std::min(trunc_select(sorted.data(), n, q, nullptr), std::max(best, 1));
    } else {
      chi = trunc_select(sorted.data(), (int)sorted.size(), q, nullptr);
    }
    double t = extra;
    for (size_t i = chi; i < sorted.size(); ++i) t += sorted[i] * sorted[i];
    if (p.err_type == TNT_ERR_1NORM) {
      double s1 = std::sqrt(extra);  // a lower bound: the clusters' values are not resolved
      for (size_t i = chi; i < sorted.size(); ++i) s1 += sorted[i];
      eps = s1;
    } else {
      eps = p.err_type == TNT_ERR_SUMSQ ? t : std::sqrt(t);
    }
  } else {
    chi = trunc_select(sorted.data(), (int)sorted.size(), p, &eps);
  }
  double nk = 0;
  for (int i = 0; i < chi; ++i) {
    nk += sorted[i] * sorted[i];
    secs[pool[i].sec].kept++;
  }
  nk = std::sqrt(nk);
  out.chi = chi;
  out.eps = eps;
  out.lambda0 = sorted[0];
  out.norm_kept = nk;
  const double scale = p.renormalise && nk > 0 ? 1.0 / nk : 1.0;
  for (auto& s : secs) {
    if (s.kept == 0) continue;
    out.bond[s.m] = s.kept;
    for (int k = 0; k < s.kept; ++k) out.lam.push_back(s.vals[k].lam * scale);
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
  // --- kept isometric vectors: uk (n x kept per sector, column-major) -----------
  int64_t uksize = 0;
  for (auto& s : secs) {
    s.ukbase = uksize;
    uksize += (int64_t)s.n * s.kept;
  }
  DevBuf uk(&c.pool, std::max<int64_t>(1, 2 * uksize) * sizeof(double));
  double* ukp = uk.as<double>();
  // level-0 vectors are copied; deeper levels' are Q_L T with T the kept
  // columns of U_L (gathered into tmp first)
  std::vector<ZCopyTask> cp;
  int64_t cpmax = 1;
  struct Prod { const Sector* s; int level, pos, cnt; int64_t toff; };
  std::vector<Prod> prods;
  int64_t tsz = 0;
  for (auto& s : secs) {
    int k = 0;
    while (k < s.kept) {
      const int l = s.vals[k].level;
      int e = k;
      while (e < s.kept && s.vals[e].level == l) ++e;
      if (l == 0) {
        for (int q = k; q < e; ++q) {
          cp.push_back(ZCopyTask{s.lv[0].U + 2 * (int64_t)s.vals[q].idx * s.n,
                                 ukp + 2 * (s.ukbase + (int64_t)q * s.n), s.n, 1.0});
          cpmax = std::max<int64_t>(cpmax, s.n);
        }
      } else {
        prods.push_back({&s, l, k, e - k, tsz});
        tsz += (int64_t)s.lv[l].n * (e - k);
      }
      k = e;
    }
  }
  DevBuf tprod(&c.pool, std::max<int64_t>(1, 2 * tsz) * sizeof(double));
  for (auto& pr : prods) {
    const Level& L = pr.s->lv[pr.level];
    for (int q = 0; q < pr.cnt; ++q) {
      cp.push_back(ZCopyTask{L.U + 2 * (int64_t)pr.s->vals[pr.pos + q].idx * L.n,
                             tprod.as<double>() + 2 * (pr.toff + (int64_t)q * L.n), L.n, 1.0});
      cpmax = std::max<int64_t>(cpmax, L.n);
    }
  }
  DevBuf cptab(&c.pool, std::max<size_t>(1, cp.size()) * sizeof(ZCopyTask));
  if (!cp.empty()) {
    TNT_HIP(hipMemcpyAsync(cptab.ptr, cp.data(), cp.size() * sizeof(ZCopyTask),
                           hipMemcpyHostToDevice, c.stream));
    launch_zcopy(cptab.as<ZCopyTask>(), (int)cp.size(), cpmax, c.stream);
  }
  ZGroup kp;  // kept vectors of the refined levels: Q_L times their eigenvectors
  for (auto& pr : prods) {
    const Sector& s = *pr.s;
    const Level& L = s.lv[pr.level];
    kp.add(0, false, s.n, pr.cnt, L.n, L.Q, s.n, tprod.as<double>() + 2 * pr.toff, L.n,
           ukp + 2 * (s.ukbase + (int64_t)pr.pos * s.n), s.n);
  }
  kp.run(c);
  // --- factors -----------------------------------------------------------
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
    // A(q_a, s1)[r, c] = uk(roff + r, c)
    for (auto& s : secs) {
      if (s.kept == 0) continue;
      for (size_t i = 0; i < s.rows.size(); ++i) {
        const BlockRef& b = out.A.blocks.at({s.rows[i].second, s.rows[i].first});
        add_st(s.ukbase + s.roff[i], 1, s.n, b.off, b.rows, b.cols, 0);
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
    // the vectors are the columns of V:  B(m, s2)[r, c] = conj(V(coff + c, r))
    for (auto& s : secs) {
      if (s.kept == 0) continue;
      s.tbase = tsize;
      tsize += (int64_t)s.C * s.kept;
      for (size_t j = 0; j < s.cols.size(); ++j) {
        const BlockRef& b = out.B.blocks.at({s.m, s.cols[j].first});
        add_st(s.ukbase + s.coff[j], s.n, 1, b.off, b.rows, b.cols, 1);
      }
    }
  }
  const size_t nfac = st.size();
  if (!right) {
    // V_kept row-major (C x kept): V_kept(r, c) = uk(r, c)
    for (auto& s : secs) {
      if (s.kept == 0) continue;
      add_st(s.ukbase, 1, s.n, s.tbase, s.C, s.kept, 0);
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
    launch_scatter_z(sdev, (int)nfac, mr, mc, ukp, fp.a_re, fp.a_im, c.stream);
    run_gemm(c, tp.g[0], FORM_CN, PATH_F64, fp.a_re, fp.a_im, ET_F64, re, im, ET_F64, fp.b_re,
             fp.b_im, ET_F64);
    centre = fp.b_re;
    centre_n = out.B.elems;
  } else {
    double* t = tmp.as<double>();
    launch_scatter_z(sdev, (int)nfac, mr, mc, ukp, fp.b_re, fp.b_im, c.stream);
    launch_scatter_z(sdev + nfac, (int)(st.size() - nfac), mr, mc, ukp, t, t + tsize, c.stream);
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
  SvdJob* jp = job.get();
  svd_eig(c, {jp});
  svd_refine(c, {jp}, {p});
  return svd_finish(c, *job, p, alloc);
}

}  // namespace tnt
