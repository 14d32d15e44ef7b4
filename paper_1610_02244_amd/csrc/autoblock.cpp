// Automatic blocking (the library's mode for tensors without known
// symmetries, Fig. fig:autoblocking, Table tab:tebdtimes): entries of
// magnitude at most `tol` are dropped, the rows and columns are grouped into
// the connected components of the bipartite graph of the remaining entries
// (row i joined to column j when a_ij survives), which is the block-diagonal
// form after a row and a column permutation, and the blocks are decomposed
// by the same block SVD as the U(1) sectors: each block is given a label of
// its own and plays the part of a charge sector (d = 1), so the blocks are
// solved together and cut together by the truncation rules.
//
// The pattern is computed on the device and read back as one byte per entry;
// the grouping (union-find, O(m n)) runs on the host, as the reordering is
// O(n^2) against the O(n^3) of the decomposition; the blocks are gathered on
// the device into packed storage and the factors scattered back to the
// caller's order.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "capi_util.h"
#include "kernels.h"
#include "svd.h"

namespace tnt {

namespace {

struct Blocks {
  std::vector<std::vector<int>> rows, cols;  // per block, ascending
};

Blocks find_blocks(const std::vector<unsigned char>& mask, int m, int n) {
  std::vector<int> parent(m + n);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int x) {
    while (parent[x] != x) {
      parent[x] = parent[parent[x]];
      x = parent[x];
    }
    return x;
  };
  std::vector<char> live_r(m, 0), live_c(n, 0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j)
      if (mask[(size_t)i * n + j]) {
        live_r[i] = live_c[j] = 1;
        const int a = find(i), b = find(m + j);
        if (a != b) parent[std::max(a, b)] = std::min(a, b);
      }
  // blocks ordered by their smallest row (the root of a component that holds
  // a row is that smallest row index, since unions keep the smaller root)
  std::vector<int> label(m + n, -1);
  Blocks B;
  for (int i = 0; i < m; ++i) {
    if (!live_r[i]) continue;
    const int r = find(i);
    if (label[r] < 0) {
      label[r] = (int)B.rows.size();
      B.rows.emplace_back();
      B.cols.emplace_back();
    }
    B.rows[label[r]].push_back(i);
  }
  for (int j = 0; j < n; ++j)
    if (live_c[j]) B.cols[label[find(m + j)]].push_back(j);
  return B;
}

}  // namespace

}  // namespace tnt

using namespace tnt;

extern "C" tnt_status tnt_auto_block_svd(tnt_ctx ctx, const double* a_re, const double* a_im,
                                         int32_t m, int32_t n, int64_t lda, double tol,
                                         const tnt_trunc_params* trunc, double* u_re,
                                         double* u_im, int64_t ldu, double* b_re, double* b_im,
                                         int64_t ldb, double* S, int32_t* chi, int32_t* nblocks,
                                         double* eps) {
  TNT_API_BEGIN(ctx)
  if (!a_re || !a_im || !trunc || !u_re || !u_im || !b_re || !b_im || !S || !chi)
    fail(TNT_E_ARG, "null argument");
  if (m < 1 || n < 1 || lda < n) fail(TNT_E_ARG, "bad matrix shape");
  if (trunc->chi_max < 1) fail(TNT_E_ARG, "chi_max < 1");
  if (ldu < trunc->chi_max || ldb < n) fail(TNT_E_ARG, "output leading dimension too small");
  if (!(tol >= 0.0) || !std::isfinite(tol)) fail(TNT_E_ARG, "tol must be finite and >= 0");
  const int cm = trunc->chi_max;
  // outputs start as zero
  TNT_HIP(hipMemsetAsync(u_re, 0, (size_t)m * ldu * sizeof(double), c.stream));
  TNT_HIP(hipMemsetAsync(u_im, 0, (size_t)m * ldu * sizeof(double), c.stream));
  TNT_HIP(hipMemsetAsync(b_re, 0, (size_t)cm * ldb * sizeof(double), c.stream));
  TNT_HIP(hipMemsetAsync(b_im, 0, (size_t)cm * ldb * sizeof(double), c.stream));
  // pattern
  DevBuf mk(&c.pool, (size_t)m * n);
  launch_nonzero_mask(a_re, a_im, m, n, lda, tol, mk.as<unsigned char>(), c.stream);
  std::vector<unsigned char> mask((size_t)m * n);
  TNT_HIP(hipMemcpyAsync(mask.data(), mk.ptr, mask.size(), hipMemcpyDeviceToHost, c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  const Blocks bl = find_blocks(mask, m, n);
  const int nb = (int)bl.rows.size();
  if (nblocks) *nblocks = nb;
  if (nb == 0) {
    *chi = 0;
    if (eps) *eps = 0.0;
    TNT_HIP(hipStreamSynchronize(c.stream));
    return TNT_OK;
  }
  // blocks as sectors: label k, rows_k x cols_k
  Bond left, right;
  for (int k = 0; k < nb; ++k) {
    left[k] = (int)bl.rows[k].size();
    right[k] = (int)bl.cols[k].size();
  }
  const ThetaH th = make_theta(left, right, 1);
  // index lists: rows of block k, then its columns
  std::vector<int32_t> idx;
  std::vector<int32_t> roff(nb), coff(nb);
  for (int k = 0; k < nb; ++k) {
    roff[k] = (int32_t)idx.size();
    idx.insert(idx.end(), bl.rows[k].begin(), bl.rows[k].end());
    coff[k] = (int32_t)idx.size();
    idx.insert(idx.end(), bl.cols[k].begin(), bl.cols[k].end());
  }
  DevBuf di(&c.pool, idx.size() * sizeof(int32_t));
  TNT_HIP(hipMemcpyAsync(di.ptr, idx.data(), idx.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, c.stream));
  auto run_copy = [&](const std::vector<IndexCopyTask>& tasks, const double* sre,
                      const double* sim, double* dre, double* dim) {
    std::vector<int2> rows;
    for (size_t t = 0; t < tasks.size(); ++t)
      for (int r = 0; r < tasks[t].rows; ++r) rows.push_back(make_int2((int)t, r));
    if (rows.empty()) return;
    DevBuf dt(&c.pool, tasks.size() * sizeof(IndexCopyTask));
    DevBuf dr(&c.pool, rows.size() * sizeof(int2));
    TNT_HIP(hipMemcpyAsync(dt.ptr, tasks.data(), tasks.size() * sizeof(IndexCopyTask),
                           hipMemcpyHostToDevice, c.stream));
    TNT_HIP(hipMemcpyAsync(dr.ptr, rows.data(), rows.size() * sizeof(int2),
                           hipMemcpyHostToDevice, c.stream));
    launch_index_copy(dt.as<IndexCopyTask>(), dr.as<int2>(), (int)rows.size(),
                      di.as<int32_t>(), sre, sim, dre, dim, c.stream);
    TNT_HIP(hipStreamSynchronize(c.stream));  // host lists released on return
  };
  // gather the blocks (entries at or below tol dropped)
  DevBuf theta(&c.pool, std::max<int64_t>(1, 2 * th.elems) * sizeof(double));
  double* tre = theta.as<double>();
  {
    std::vector<IndexCopyTask> tasks;
    for (int k = 0; k < nb; ++k) {
      const BlockRef& b = th.blocks.at({k, 0, 0});
      IndexCopyTask t{};
      t.src_off = 0;
      t.src_ld = lda;
      t.dst_off = b.off;
      t.dst_ld = b.cols;
      t.src_ridx = roff[k];
      t.src_cidx = coff[k];
      t.dst_ridx = t.dst_cidx = -1;
      t.rows = b.rows;
      t.cols = b.cols;
      t.tol2 = tol * tol;
      tasks.push_back(t);
    }
    run_copy(tasks, a_re, a_im, tre, tre + th.elems);
  }
  DevBuf fa, fb;
  SvdOut r = svd_truncate_dev(c, th, tre, tre + th.elems, *trunc, TNT_ABSORB_RIGHT,
                              [&](const SvdOut& o) {
                                fa = DevBuf(&c.pool, std::max<int64_t>(1, 2 * o.A.elems) * 8);
                                fb = DevBuf(&c.pool, std::max<int64_t>(1, 2 * o.B.elems) * 8);
                                FactorPlanes fp;
                                fp.a_re = fa.as<double>();
                                fp.a_im = fa.as<double>() + o.A.elems;
                                fp.b_re = fb.as<double>();
                                fp.b_im = fb.as<double>() + o.B.elems;
                                return fp;
                              });
  // scatter: U(rows of k, base_k + c) = A_k(r, c); B(base_k + r, cols of k) = B_k(r, c)
  {
    std::vector<IndexCopyTask> ta, tb;
    int base = 0;
    for (auto& kv : r.bond) {
      const int k = kv.first, kept = kv.second;
      const BlockRef& a = r.A.blocks.at({k, 0});
      const BlockRef& b = r.B.blocks.at({k, 0});
      IndexCopyTask t{};
      t.src_off = a.off;
      t.src_ld = a.cols;
      t.dst_off = 0;
      t.dst_ld = ldu;
      t.src_ridx = t.src_cidx = -1;
      t.dst_ridx = roff[k];
      t.dst_cidx = -1;
      t.dst_cbase = base;
      t.rows = a.rows;
      t.cols = kept;
      t.tol2 = -1.0;
      ta.push_back(t);
      IndexCopyTask u{};
      u.src_off = b.off;
      u.src_ld = b.cols;
      u.dst_off = 0;
      u.dst_ld = ldb;
      u.src_ridx = u.src_cidx = -1;
      u.dst_ridx = -1;
      u.dst_rbase = base;
      u.dst_cidx = coff[k];
      u.rows = kept;
      u.cols = b.cols;
      u.tol2 = -1.0;
      tb.push_back(u);
      base += kept;
    }
    run_copy(ta, fa.as<double>(), fa.as<double>() + r.A.elems, u_re, u_im);
    run_copy(tb, fb.as<double>(), fb.as<double>() + r.B.elems, b_re, b_im);
  }
  *chi = r.chi;
  for (int i = 0; i < r.chi; ++i) S[i] = r.lam[i];
  if (eps) *eps = r.eps;
  TNT_API_END
}
