// Truncated SVD of a two-site vector (appendix B.1.2) with U(1) sectors.
//
// For every middle charge m = q_a + s1 the matrix with rows (s1, a) and
// columns (s2, b) is assembled on the device (column-major, interleaved
// complex) and decomposed in FP64 by rocSOLVER's gesvd.  The singular values
// of all sectors are pooled on the host, sorted and cut by the four
// truncation rules; the kept columns of U and rows of V^+ are scattered back
// into U(1) site blocks with the singular values absorbed left or right.
#include "svd.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <set>

#include "kernels.h"

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

namespace {
struct Sector {
  int m = 0;
  std::vector<std::pair<int, int>> rows, cols;  // (s1, q_a), (s2, q_b)
  std::vector<int> roff, coff;
  int R = 0, C = 0, K = 0;
  int64_t a_base = 0, u_base = 0, v_base = 0;  // complex offsets
  int s_base = 0, e_base = 0;
  int kept = 0, lam_base = 0;
};

// Sectors from the blocks present: rows (s1, q_a) and columns (s2, q_b), both
// ascending in s, for every middle charge m = q_a + s1.
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
    s.K = std::min(s.R, s.C);
    out.push_back(std::move(s));
  }
  return out;
}
}  // namespace

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

SvdOut svd_truncate_dev(Ctx& c, const ThetaH& th, const double* re, const double* im,
                        const tnt_trunc_params& p, int absorb, const FactorAlloc& alloc) {
  if (p.chi_max < 1) fail(TNT_E_ARG, "chi_max must be >= 1");
  if (absorb != TNT_ABSORB_RIGHT && absorb != TNT_ABSORB_LEFT) fail(TNT_E_ARG, "bad absorb");
  std::vector<Sector> secs = sectors_of(th);
  int64_t za = 0, zu = 0, zv = 0;
  int ns = 0;
  for (auto& s : secs) {
    s.a_base = za; za += (int64_t)s.R * s.C;
    s.u_base = zu; zu += (int64_t)s.R * s.K;
    s.v_base = zv; zv += (int64_t)s.K * s.C;
    s.s_base = ns; s.e_base = ns; ns += s.K;
  }
  SvdOut out;
  if (secs.empty()) fail(TNT_E_SHAPE, "theta has no sector to decompose");
  // device staging: matrices, U, V^+, S, E, info
  DevBuf mat(&c.pool, std::max<int64_t>(za, 1) * 16);
  DevBuf ubuf(&c.pool, std::max<int64_t>(zu, 1) * 16);
  DevBuf vbuf(&c.pool, std::max<int64_t>(zv, 1) * 16);
  DevBuf sbuf(&c.pool, std::max(ns, 1) * sizeof(double) * 2);
  DevBuf info(&c.pool, std::max<size_t>(secs.size(), 1) * sizeof(rocblas_int));
  launch_fill_zero(mat.ptr, ET_F64, 2 * za, c.stream);
  // gather theta blocks into the sector matrices
  std::vector<GatherTask> gt;
  int maxr = 1, maxc = 1;
  {
    std::map<int, const Sector*> bym;
    for (auto& s : secs) bym[s.m] = &s;
    for (auto& kv : th.blocks) {
      const int qa = kv.first[0], s1 = kv.first[1], s2 = kv.first[2];
      auto it = bym.find(qa + s1);
      if (it == bym.end()) continue;
      const Sector& s = *it->second;
      int ri = -1, ci = -1;
      for (size_t i = 0; i < s.rows.size(); ++i) if (s.rows[i].first == s1) ri = (int)i;
      for (size_t i = 0; i < s.cols.size(); ++i) if (s.cols[i].first == s2) ci = (int)i;
      if (ri < 0 || ci < 0) continue;
      gt.push_back(GatherTask{kv.second.off, s.a_base + (int64_t)s.coff[ci] * s.R + s.roff[ri],
                              kv.second.rows, kv.second.cols, s.R, 0});
      maxr = std::max(maxr, kv.second.rows);
      maxc = std::max(maxc, kv.second.cols);
    }
  }
  DevBuf gtab(&c.pool, std::max<size_t>(gt.size(), 1) * sizeof(GatherTask));
  if (!gt.empty())
    TNT_HIP(hipMemcpyAsync(gtab.ptr, gt.data(), gt.size() * sizeof(GatherTask),
                           hipMemcpyHostToDevice, c.stream));
  launch_gather_cm(gtab.as<GatherTask>(), (int)gt.size(), maxr, maxc, re, im, mat.as<double>(),
                   c.stream);
  // per-sector FP64 SVD
  rocblas_handle h = blas(c);
  double* S = sbuf.as<double>();
  double* E = S + ns;
  for (size_t i = 0; i < secs.size(); ++i) {
    const Sector& s = secs[i];
    auto* A = reinterpret_cast<rocblas_double_complex*>(mat.as<double>()) + s.a_base;
    auto* U = reinterpret_cast<rocblas_double_complex*>(ubuf.as<double>()) + s.u_base;
    auto* V = reinterpret_cast<rocblas_double_complex*>(vbuf.as<double>()) + s.v_base;
    rocblas_status st = rocsolver_zgesvd(h, rocblas_svect_singular, rocblas_svect_singular, s.R,
                                         s.C, A, s.R, S + s.s_base, U, s.R, V, s.K,
                                         E + s.e_base, rocblas_outofplace,
                                         info.as<rocblas_int>() + i);
    if (st != rocblas_status_success) fail(TNT_E_HIP, "rocsolver_zgesvd failed");
  }
  std::vector<double> hs(ns);
  std::vector<rocblas_int> hinfo(secs.size());
  TNT_HIP(hipMemcpyAsync(hs.data(), S, ns * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  TNT_HIP(hipMemcpyAsync(hinfo.data(), info.ptr, secs.size() * sizeof(rocblas_int),
                         hipMemcpyDeviceToHost, c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  for (auto v : hinfo)
    if (v != 0) fail(TNT_E_HIP, "SVD did not converge in a sector");
  for (double v : hs)
    if (!std::isfinite(v)) fail(TNT_E_NONFINITE, "non-finite singular value (theta not finite?)");
  // pool, sort (lambda desc, then m asc, then index asc), select
  struct Ent { double lam; int sec, idx; };
  std::vector<Ent> pool;
  pool.reserve(ns);
  for (size_t i = 0; i < secs.size(); ++i)
    for (int k = 0; k < secs[i].K; ++k) pool.push_back({hs[secs[i].s_base + k], (int)i, k});
  std::stable_sort(pool.begin(), pool.end(), [](const Ent& a, const Ent& b) {
    if (a.lam != b.lam) return a.lam > b.lam;
    if (a.sec != b.sec) return a.sec < b.sec;
    return a.idx < b.idx;
  });
  std::vector<double> sorted(pool.size());
  for (size_t i = 0; i < pool.size(); ++i) sorted[i] = pool[i].lam;
  double eps = 0;
  const int chi = trunc_select(sorted.data(), (int)sorted.size(), p, &eps);
  double nk = 0;
  for (int i = 0; i < chi; ++i) {
    nk += sorted[i] * sorted[i];
    secs[pool[i].sec].kept++;
  }
  nk = std::sqrt(nk);
  if (!(nk > 0)) fail(TNT_E_NONFINITE, "theta has zero norm");
  const double scale = p.renormalise ? 1.0 / nk : 1.0;
  out.chi = chi;
  out.eps = eps;
  out.lambda0 = sorted.empty() ? 0 : sorted[0];
  out.norm_kept = nk;
  for (auto& s : secs) {
    if (s.kept == 0) continue;
    out.bond[s.m] = s.kept;
    s.lam_base = (int)out.lam.size();
    for (int k = 0; k < s.kept; ++k) out.lam.push_back(hs[s.s_base + k] * scale);
  }
  // factor layouts: A blocks (q_a, s1) ascending, B blocks (m, s2) ascending
  {
    std::map<std::pair<int, int>, std::pair<int, int>> ablk, bblk;  // key -> (rows, cols)
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
  double *a_re = fp.a_re, *a_im = fp.a_im, *b_re = fp.b_re, *b_im = fp.b_im;
  // scatter
  std::vector<ScatterTask> st;
  int mr = 1, mc = 1;
  for (auto& s : secs) {
    if (s.kept == 0) continue;
    for (size_t i = 0; i < s.rows.size(); ++i) {
      const int s1 = s.rows[i].first, qa = s.rows[i].second;
      const BlockRef& b = out.A.blocks.at({qa, s1});
      st.push_back(ScatterTask{s.u_base + s.roff[i], b.off,
                               absorb == TNT_ABSORB_LEFT ? (int64_t)s.lam_base : -1, b.rows,
                               b.cols, s.R, 0});
      mr = std::max(mr, b.rows); mc = std::max(mc, b.cols);
    }
  }
  const size_t na = st.size();
  for (auto& s : secs) {
    if (s.kept == 0) continue;
    for (size_t i = 0; i < s.cols.size(); ++i) {
      const int s2 = s.cols[i].first;
      const BlockRef& b = out.B.blocks.at({s.m, s2});
      st.push_back(ScatterTask{s.v_base + (int64_t)s.coff[i] * s.K, b.off,
                               absorb == TNT_ABSORB_RIGHT ? (int64_t)s.lam_base : -1, b.rows,
                               b.cols, s.K, 1});
      mr = std::max(mr, b.rows); mc = std::max(mc, b.cols);
    }
  }
  DevBuf stab(&c.pool, std::max<size_t>(st.size(), 1) * sizeof(ScatterTask) +
                           std::max<size_t>(out.lam.size(), 1) * sizeof(double));
  char* base = stab.as<char>();
  double* lam_dev = reinterpret_cast<double*>(base + std::max<size_t>(st.size(), 1) * sizeof(ScatterTask));
  if (!st.empty())
    TNT_HIP(hipMemcpyAsync(base, st.data(), st.size() * sizeof(ScatterTask),
                           hipMemcpyHostToDevice, c.stream));
  if (!out.lam.empty())
    TNT_HIP(hipMemcpyAsync(lam_dev, out.lam.data(), out.lam.size() * sizeof(double),
                           hipMemcpyHostToDevice, c.stream));
  const ScatterTask* sdev = reinterpret_cast<const ScatterTask*>(base);
  launch_scatter_cm(sdev, (int)na, mr, mc, ubuf.as<double>(), lam_dev, a_re, a_im, c.stream);
  launch_scatter_cm(sdev + na, (int)(st.size() - na), mr, mc, vbuf.as<double>(), lam_dev, b_re,
                    b_im, c.stream);
  // the host vectors above must outlive the asynchronous copies
  TNT_HIP(hipStreamSynchronize(c.stream));
  return out;
}

}  // namespace tnt
