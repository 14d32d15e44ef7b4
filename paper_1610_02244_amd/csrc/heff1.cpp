// One-site effective Hamiltonian (the contractor of Sec. 4.2, Listing
// lis:varmincontract, in its one-site form):
//   y[a', s', b'] = sum L[a', w, a] W[w, u, s', s] R[b', u, b] A[a, s, b].
// The same three steps as the two-site operator with a single MPO tensor:
// a grouped FP64 GEMM per (w, A block) for L.A, the sparse MPO combination,
// and a grouped GEMM with R whose inner dimension runs over (u, b).
#include <array>
#include <map>

#include "capi_util.h"
#include "kernels.h"

namespace tnt {
namespace {

// site tensor A[a, s, b]: labels (q_a, s, q_b), extents (dim_a, 1, dim_b)
std::map<std::pair<int, int>, BlockRef> parse_site3(const tnt_btensor* t, int d,
                                                     const char* what) {
  const std::string w(what);
  if (!t) fail(TNT_E_ARG, w + ": null descriptor");
  if (t->rank != 3) fail(TNT_E_ARG, w + ": rank must be 3");
  if (t->nblocks < 0 || (t->nblocks > 0 && (!t->qn || !t->extent || !t->offset)))
    fail(TNT_E_ARG, w + ": bad block arrays");
  if (t->dtype != TNT_DT_F64) fail(TNT_E_ARG, w + ": dtype must be TNT_DT_F64");
  if (t->nblocks > 0 && (!t->re || !t->im)) fail(TNT_E_ARG, w + ": null plane");
  std::map<std::pair<int, int>, BlockRef> out;
  for (int i = 0; i < t->nblocks; ++i) {
    const int* q = t->qn + 3 * i;
    const int* e = t->extent + 3 * i;
    if (e[1] != 1 || e[0] < 1 || e[2] < 1) fail(TNT_E_SHAPE, w + ": bad extents");
    if (q[1] < 0 || q[1] >= d) fail(TNT_E_ARG, w + ": physical label out of range");
    if (q[2] != q[0] + q[1]) fail(TNT_E_CHARGE, w + ": block violates q_b = q_a + s");
    const int64_t off = t->offset[i], sz = (int64_t)e[0] * e[2];
    if (off < 0) fail(TNT_E_ARG, w + ": negative offset");
    if (off + sz > t->capacity) fail(TNT_E_CAPACITY, w + ": block past capacity");
    if (!out.emplace(std::make_pair(q[0], q[1]), BlockRef{off, e[0], e[2]}).second)
      fail(TNT_E_ARG, w + ": duplicate block");
  }
  return out;
}

}  // namespace
}  // namespace tnt

using namespace tnt;

extern "C" tnt_status tnt_heff1_apply(tnt_ctx ctx, const tnt_btensor* L, const tnt_mpo_site* W,
                                      const tnt_btensor* R, const tnt_btensor* A,
                                      const tnt_btensor* out) {
  TNT_API_BEGIN(ctx)
  if (!L || !W || !R || !A || !out) fail(TNT_E_ARG, "null argument");
  // every operand is read (and out written) as FP64 planes
  for (const tnt_btensor* t : {L, R, A, out}) {
    if (t->dtype != TNT_DT_F64) fail(TNT_E_ARG, "L, R, A and out must be FP64 planes");
    if (!t->re || !t->im) fail(TNT_E_ARG, "null plane");
  }
  const MpoH w = parse_mpo(W, "W");
  const EnvH le = parse_env(L, w, "L");
  const EnvH re = parse_env(R, w, "R");
  const auto a = parse_site3(A, w.d, "A");
  const auto o = parse_site3(out, w.d, "out");
  if (a.size() != o.size()) fail(TNT_E_SHAPE, "out: block set differs from A");
  for (auto& kv : a) {
    auto it = o.find(kv.first);
    if (it == o.end() || it->second.rows != kv.second.rows || it->second.cols != kv.second.cols)
      fail(TNT_E_SHAPE, "out: block set or extents differ from A");
  }
  const int D = w.D, d = w.d;
  const auto& qw = w.qw;
  // X[w; a', s, b] = L(w, q_a) A(q_a, s)
  HostGemm gx;
  std::map<std::array<int, 3>, std::array<int64_t, 3>> xoff;  // -> off, rows, cols
  int64_t xs = 0;
  for (auto& kv : a) {
    const int qa = kv.first.first, s = kv.first.second;
    for (int ww = 0; ww < D; ++ww) {
      auto il = le.blocks.find({ww, qa});
      if (il == le.blocks.end()) continue;
      if (il->second.cols != kv.second.rows) fail(TNT_E_SHAPE, "L and A disagree on a sector");
      const int M = il->second.rows, N = kv.second.cols, K = kv.second.rows;
      xoff[{ww, qa + qw[ww], s}] = {xs, M, N};
      gx.add_task(xs, M, N, N);
      gx.add_seg(il->second.off, K, kv.second.off, N, K);
      xs += (int64_t)M * N;
    }
  }
  // Y[u; a', s', b] = sum_{w, s} W[w, u, s', s] X[w; a', s, b]
  std::map<std::array<int, 3>, std::vector<std::pair<int64_t, double>>> yterms;
  std::map<std::array<int, 3>, std::pair<int, int>> yshape;
  for (auto& x : xoff) {
    const int ww = x.first[0], qap = x.first[1], s = x.first[2];
    for (int u = 0; u < D; ++u)
      for (int sp = 0; sp < d; ++sp) {
        const double cf = w.at(ww, u, sp, s);
        if (cf == 0.0) continue;
        yterms[{u, qap, sp}].push_back({x.second[0], cf});
        yshape[{u, qap, sp}] = {(int)x.second[1], (int)x.second[2]};
      }
  }
  HostComb cy;
  std::map<std::array<int, 3>, int64_t> yoff;
  int64_t ys = 0;
  for (auto& y : yterms) {
    const auto shp = yshape.at(y.first);
    yoff[y.first] = ys;
    cy.add_task(ys, shp.first * shp.second);
    for (auto& t : y.second) cy.add_term(t.first, t.second);
    ys += (int64_t)shp.first * shp.second;
  }
  cy.finalize();
  // out(q_a', s') = sum_u Y[u; a', s', b] R(u, q_b)^T,  q_b = q_a' + s' - qw[u]
  HostGemm go;
  for (auto& kv : o) {
    const int qap = kv.first.first, sp = kv.first.second;
    const int M = kv.second.rows, N = kv.second.cols;
    go.add_task(kv.second.off, M, N, N);
    for (int u = 0; u < D; ++u) {
      auto iy = yoff.find({u, qap, sp});
      if (iy == yoff.end()) continue;
      auto ir = re.blocks.find({u, qap + sp - qw[u]});
      if (ir == re.blocks.end()) continue;
      const auto ysh = yshape.at({u, qap, sp});
      const int K = ysh.second;
      if (ysh.first != M) fail(TNT_E_SHAPE, "L and A disagree on a sector");
      if (ir->second.rows != N || ir->second.cols != K)
        fail(TNT_E_SHAPE, "R and A disagree on a sector");
      go.add_seg(iy->second, K, ir->second.off, ir->second.cols, K);
    }
  }
  double* ore = static_cast<double*>(out->re);
  double* oim = static_cast<double*>(out->im);
  if (!go.tasks.empty()) {
    if (!gx.tasks.empty()) gx.finalize(default_tile_cfg(gx, PATH_F64));
    go.finalize(default_tile_cfg(go, PATH_F64));
    DevTables t;
    t.upload(c, {&gx, &go}, {&cy});
    DevBuf X(&c.pool, std::max<int64_t>(1, 2 * xs) * sizeof(double));
    DevBuf Y(&c.pool, std::max<int64_t>(1, 2 * ys) * sizeof(double));
    double* x = X.as<double>();
    double* y = Y.as<double>();
    if (!gx.tasks.empty())
      run_gemm(c, t.g[0], FORM_NN, PATH_F64, L->re, L->im, ET_F64, A->re, A->im, ET_F64, x,
               x + xs, ET_F64);
    if (!cy.tasks.empty()) run_comb(c, t.c[0], x, x + xs, y, y + ys, ET_F64);
    run_gemm(c, t.g[1], FORM_NT, PATH_F64, y, y + ys, ET_F64, R->re, R->im, ET_F64, ore, oim,
             ET_F64);
    TNT_HIP(hipStreamSynchronize(c.stream));
  }
  TNT_API_END
}
