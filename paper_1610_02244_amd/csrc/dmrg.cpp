// Two-site variational sweep over a U(1) block MPS (Sec. 4.3 in two-site
// form): theta formation, Lanczos on H_eff, truncated SVD, environment
// update, for bonds 1..L-1 (right pass) then L-1..1 (left pass).  All tensor
// arithmetic runs in the grouped MFMA GEMM and combine kernels; environments,
// theta and the SVD are FP64.
#include "dmrg.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <chrono>
#include <climits>
#include <cmath>

#include "batch.h"
#include "capi_util.h"

namespace tnt {

namespace {
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
int dim_of(const Bond& b, int q) {
  auto it = b.find(q);
  return it == b.end() ? 0 : it->second;
}
}  // namespace

ThetaH form_theta(Ctx& c, MpsH& m, int j, DevBuf& out) {
  ThetaH th = make_theta(m.bonds[j - 1], m.bonds[j + 1], m.d);
  out.ensure(&c.pool, std::max<int64_t>(1, 2 * th.elems) * sizeof(double));
  HostGemm g;
  const SiteH& A = m.lay[j - 1];
  const SiteH& B = m.lay[j];
  for (auto& kv : th.blocks) {
    const int qa = kv.first[0], s1 = kv.first[1], s2 = kv.first[2];
    const BlockRef& ob = kv.second;
    g.add_task(ob.off, ob.rows, ob.cols, ob.cols);
    auto ia = A.blocks.find({qa, s1});
    auto ib = B.blocks.find({qa + s1, s2});
    if (ia != A.blocks.end() && ib != B.blocks.end())
      g.add_seg(ia->second.off, ia->second.cols, ib->second.off, ib->second.cols,
                ia->second.cols);
  }
  g.finalize(default_tile_cfg(g, PATH_F64));
  DevTables t;
  t.upload(c, {&g}, {});
  double* o = out.as<double>();
  run_gemm(c, t.g[0], FORM_NN, PATH_F64, m.re(j), m.im(j), ET_F64, m.re(j + 1), m.im(j + 1),
           ET_F64, o, o + th.elems, ET_F64);
  TNT_HIP(hipStreamSynchronize(c.stream));  // tables (host and device) released below
  return th;
}

// L_j[a', w', a] = sum conj(A[c', s', a']) L_{j-1}[c', w, c] W[w, w', s', s] A[c, s, a]
void update_left_env(Ctx& c, EnvS& e, int j) {
  MpsH& m = *e.mps;
  const MpoH& W = e.W[j - 1];
  const auto& qw = e.qw;
  const int D = W.D, d = m.d;
  const EnvH& Lp = e.Llay[j - 1];
  const SiteH& A = m.lay[j - 1];
  const Bond& bl = m.bonds[j - 1];
  const Bond& br = m.bonds[j];
  // X[w; c', s, a] = L_{j-1}(w, c) A(c, s)
  HostGemm gx;
  std::map<std::array<int, 3>, int64_t> xoff;
  int64_t off = 0;
  for (auto& lb : Lp.blocks) {
    const int w = lb.first.first, qc = lb.first.second;
    for (int s = 0; s < d; ++s) {
      auto ia = A.blocks.find({qc, s});
      if (ia == A.blocks.end()) continue;
      const int M = lb.second.rows, N = ia->second.cols, K = lb.second.cols;
      xoff[{w, qc, s}] = off;
      gx.add_task(off, M, N, N);
      gx.add_seg(lb.second.off, K, ia->second.off, N, K);
      off += (int64_t)M * N;
    }
  }
  const int64_t xs = off;
  // Y[w'; c', s', a] = sum_{w, s} W[w, w', s', s] X[w; c', s, a]
  std::map<std::array<int, 3>, std::vector<std::pair<int64_t, double>>> yterms;
  for (auto& x : xoff) {
    const int w = x.first[0], qc = x.first[1], s = x.first[2];
    const int qcp = qc + qw[w];
    for (int wp = 0; wp < D; ++wp)
      for (int sp = 0; sp < d; ++sp) {
        const double cf = W.at(w, wp, sp, s);
        if (cf != 0.0) yterms[{wp, qcp, sp}].push_back({x.second, cf});
      }
  }
  HostComb cy;
  std::map<std::array<int, 3>, int64_t> yoff;
  off = 0;
  for (auto& y : yterms) {
    const int wp = y.first[0], qcp = y.first[1], sp = y.first[2];
    const int qa = qcp + sp - qw[wp];
    const int rows = dim_of(bl, qcp), cols = dim_of(br, qa);
    if (rows == 0 || cols == 0) continue;
    yoff[y.first] = off;
    cy.add_task(off, rows * cols);
    for (auto& t : y.second) cy.add_term(t.first, t.second);
    off += (int64_t)rows * cols;
  }
  const int64_t ys = off;
  cy.finalize();
  // L_j(w', a) = sum_{s'} A(c', s')^H Y[w'; c', s', a],  c' = a + qw[w'] - s'
  EnvH Ln = make_env(br, qw);
  HostGemm gl;
  for (auto& lb : Ln.blocks) {
    const int wp = lb.first.first, qa = lb.first.second;
    const int M = lb.second.rows, N = lb.second.cols;
    gl.add_task(lb.second.off, M, N, N);
    for (int sp = 0; sp < d; ++sp) {
      const int qcp = qa + qw[wp] - sp;
      auto ia = A.blocks.find({qcp, sp});
      auto iy = yoff.find({wp, qcp, sp});
      if (ia == A.blocks.end() || iy == yoff.end()) continue;
      gl.add_seg(ia->second.off, ia->second.cols, iy->second, N, ia->second.rows);
    }
  }
  gx.finalize(default_tile_cfg(gx, PATH_F64));
  gl.finalize(default_tile_cfg(gl, PATH_F64));
  DevTables t;
  t.upload(c, {&gx, &gl}, {&cy});
  DevBuf X(&c.pool, std::max<int64_t>(1, 2 * xs) * sizeof(double));
  DevBuf Y(&c.pool, std::max<int64_t>(1, 2 * ys) * sizeof(double));
  DevBuf out(&c.pool, std::max<int64_t>(1, 2 * Ln.elems) * sizeof(double));
  double* x = X.as<double>();
  double* y = Y.as<double>();
  double* o = out.as<double>();
  run_gemm(c, t.g[0], FORM_NN, PATH_F64, e.Lre(j - 1), e.Lim(j - 1), ET_F64, m.re(j), m.im(j),
           ET_F64, x, x + xs, ET_F64);
  run_comb(c, t.c[0], x, x + xs, y, y + ys, ET_F64);
  run_gemm(c, t.g[1], FORM_CN, PATH_F64, m.re(j), m.im(j), ET_F64, y, y + ys, ET_F64, o,
           o + Ln.elems, ET_F64);
  TNT_HIP(hipStreamSynchronize(c.stream));
  e.Llay[j] = Ln;
  e.Ldat[j] = std::move(out);
}

// R_j[b', u, b] = sum conj(A[b', s', c']) W[u, u', s', s] R_{j+1}[c', u', c] A[b, s, c]
void update_right_env(Ctx& c, EnvS& e, int j) {
  MpsH& m = *e.mps;
  const MpoH& W = e.W[j - 1];
  const auto& qw = e.qw;
  const int D = W.D, d = m.d;
  const EnvH& Rn = e.Rlay[j + 1];
  const SiteH& B = m.lay[j - 1];
  const Bond& bl = m.bonds[j - 1];
  const Bond& br = m.bonds[j];
  // X[u'; b, s, c'] = B(b, s) R_{j+1}(u', c)^T
  HostGemm gx;
  std::map<std::array<int, 3>, int64_t> xoff;
  int64_t off = 0;
  for (auto& bb : B.blocks) {
    const int qb = bb.first.first, s = bb.first.second, qc = qb + s;
    for (int up = 0; up < D; ++up) {
      auto ir = Rn.blocks.find({up, qc});
      if (ir == Rn.blocks.end()) continue;
      const int M = bb.second.rows, N = ir->second.rows, K = bb.second.cols;
      xoff[{up, qb, s}] = off;
      gx.add_task(off, M, N, N);
      gx.add_seg(bb.second.off, K, ir->second.off, ir->second.cols, K);
      off += (int64_t)M * N;
    }
  }
  const int64_t xs = off;
  // Y[u; b, s', c'] = sum_{u', s} W[u, u', s', s] X[u'; b, s, c']
  std::map<std::array<int, 3>, std::vector<std::pair<int64_t, double>>> yterms;
  for (auto& x : xoff) {
    const int up = x.first[0], qb = x.first[1], s = x.first[2];
    for (int u = 0; u < D; ++u)
      for (int sp = 0; sp < d; ++sp) {
        const double cf = W.at(u, up, sp, s);
        if (cf != 0.0) yterms[{u, qb, sp}].push_back({x.second, cf});
      }
  }
  HostComb cy;
  std::map<std::array<int, 3>, int64_t> yoff;
  off = 0;
  for (auto& y : yterms) {
    const int u = y.first[0], qb = y.first[1], sp = y.first[2];
    const int rows = dim_of(bl, qb), cols = dim_of(br, qb + sp + qw[u]);
    if (rows == 0 || cols == 0) continue;
    yoff[y.first] = off;
    cy.add_task(off, rows * cols);
    for (auto& t : y.second) cy.add_term(t.first, t.second);
    off += (int64_t)rows * cols;
  }
  const int64_t ys = off;
  cy.finalize();
  // R_j(u, b) = sum_{s'} conj(B(b', s')) Y[u; b, s', c']^T,  b' = b + qw[u]
  EnvH Rj = make_env(bl, qw);
  HostGemm gr;
  for (auto& rb : Rj.blocks) {
    const int u = rb.first.first, qb = rb.first.second;
    const int M = rb.second.rows, N = rb.second.cols;
    const int qbp = qb + qw[u];
    gr.add_task(rb.second.off, M, N, N);
    for (int sp = 0; sp < d; ++sp) {
      auto ib = B.blocks.find({qbp, sp});
      auto iy = yoff.find({u, qb, sp});
      if (ib == B.blocks.end() || iy == yoff.end()) continue;
      const int K = ib->second.cols;
      gr.add_seg(ib->second.off, K, iy->second, K, K);
    }
  }
  gx.finalize(default_tile_cfg(gx, PATH_F64));
  gr.finalize(default_tile_cfg(gr, PATH_F64));
  DevTables t;
  t.upload(c, {&gx, &gr}, {&cy});
  DevBuf X(&c.pool, std::max<int64_t>(1, 2 * xs) * sizeof(double));
  DevBuf Y(&c.pool, std::max<int64_t>(1, 2 * ys) * sizeof(double));
  DevBuf out(&c.pool, std::max<int64_t>(1, 2 * Rj.elems) * sizeof(double));
  double* x = X.as<double>();
  double* y = Y.as<double>();
  double* o = out.as<double>();
  run_gemm(c, t.g[0], FORM_NT, PATH_F64, m.re(j), m.im(j), ET_F64, e.Rre(j + 1), e.Rim(j + 1),
           ET_F64, x, x + xs, ET_F64);
  run_comb(c, t.c[0], x, x + xs, y, y + ys, ET_F64);
  run_gemm(c, t.g[1], FORM_cNT, PATH_F64, m.re(j), m.im(j), ET_F64, y, y + ys, ET_F64, o,
           o + Rj.elems, ET_F64);
  TNT_HIP(hipStreamSynchronize(c.stream));
  e.Rlay[j] = Rj;
  e.Rdat[j] = std::move(out);
}

static void upload_boundary(Ctx& c, const EnvH& lay, int w, DevBuf& dst) {
  std::vector<double> h(std::max<int64_t>(1, 2 * lay.elems), 0.0);
  bool found = false;
  for (auto& kv : lay.blocks)
    if (kv.first.first == w) {
      h[kv.second.off] = 1.0;
      found = true;
    }
  if (!found) fail(TNT_E_ARG, "boundary MPO index has no charge-neutral block");
  dst = DevBuf(&c.pool, h.size() * sizeof(double));
  TNT_HIP(hipMemcpyAsync(dst.ptr, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice,
                         c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
}

void build_boundaries(Ctx& c, EnvS& e) {
  MpsH& m = *e.mps;
  if (m.bonds[0].size() != 1 || m.bonds[m.L].size() != 1)
    fail(TNT_E_STATE, "end bonds must hold exactly one sector");
  if (m.bonds[0].begin()->second != 1 || m.bonds[m.L].begin()->second != 1)
    fail(TNT_E_STATE, "end bonds must have dimension 1");
  e.Llay.assign(m.L + 1, EnvH());
  e.Rlay.assign(m.L + 2, EnvH());
  e.Ldat.clear();
  e.Rdat.clear();
  e.Ldat.resize(m.L + 1);
  e.Rdat.resize(m.L + 2);
  e.Llay[0] = make_env(m.bonds[0], e.qw);
  upload_boundary(c, e.Llay[0], e.left_index, e.Ldat[0]);
  e.Rlay[m.L + 1] = make_env(m.bonds[m.L], e.qw);
  upload_boundary(c, e.Rlay[m.L + 1], e.right_index, e.Rdat[m.L + 1]);
}

// ---------------------------------------------------------------------------
// right-canonical form by Householder QR (sites L..2), then unit norm.
// For each left sector q of site j, M_q (rows a, columns (s, b)) satisfies
// M_q^+ = Q R (reduced, rocSOLVER geqrf + ungqr); site j keeps Q^+ (a right
// isometry, k = min(rows, cols) rows) and R^+ is absorbed into site j-1.
// ---------------------------------------------------------------------------
void right_canonicalize(Ctx& c, MpsH& m) {
  rocblas_handle h = static_cast<rocblas_handle>(blas_handle(c));
  for (int j = m.L; j >= 2; --j) {
    const SiteH& S = m.lay[j - 1];
    struct Sec { int q, R, C, k; int64_t zbase, tbase, rbase; std::vector<std::pair<int, int>> cols; };
    std::map<int, Sec> secs;  // left charge -> sector
    for (auto& kv : S.blocks) {
      Sec& s = secs[kv.first.first];
      s.q = kv.first.first;
      s.R = kv.second.rows;
      s.cols.push_back({kv.first.second, kv.second.cols});
    }
    if (secs.empty()) fail(TNT_E_STATE, "site " + std::to_string(j) + " has no block");
    int64_t zs = 0, ts = 0, rs = 0;
    for (auto& kv : secs) {
      Sec& s = kv.second;
      s.C = 0;
      for (auto& cc : s.cols) s.C += cc.second;
      s.k = std::min(s.R, s.C);
      s.zbase = zs; zs += (int64_t)s.C * s.R;   // M^+ column-major (C x R)
      s.tbase = ts; ts += s.k;                  // Householder scalars
      s.rbase = rs; rs += (int64_t)s.R * s.k;   // R^+ (R x k) row-major
    }
    Bond newb;
    for (auto& kv : secs) newb[kv.first] = kv.second.k;
    // gather M^+ : Z[c + r C] = conj(M[r][c])
    std::vector<GatherTask> gt;
    int mr = 1, mc = 1;
    for (auto& kv : secs) {
      const Sec& s = kv.second;
      int64_t co = 0;
      for (auto& cc : s.cols) {
        const BlockRef& b = S.blocks.at({s.q, cc.first});
        gt.push_back(GatherTask{b.off, s.zbase + co, s.C, 1, b.rows, b.cols, 1, 0});
        mr = std::max(mr, b.rows);
        mc = std::max(mc, b.cols);
        co += cc.second;
      }
    }
    DevBuf gtab(&c.pool, gt.size() * sizeof(GatherTask));
    TNT_HIP(hipMemcpyAsync(gtab.ptr, gt.data(), gt.size() * sizeof(GatherTask),
                           hipMemcpyHostToDevice, c.stream));
    DevBuf z(&c.pool, std::max<int64_t>(1, 2 * zs) * sizeof(double));
    DevBuf tau(&c.pool, std::max<int64_t>(1, 2 * ts) * sizeof(double));
    launch_gather_z(gtab.as<GatherTask>(), (int)gt.size(), mr, mc, m.re(j), m.im(j),
                    z.as<double>(), c.stream);
    auto* Z = reinterpret_cast<rocblas_double_complex*>(z.as<double>());
    auto* T = reinterpret_cast<rocblas_double_complex*>(tau.as<double>());
    for (auto& kv : secs) {
      const Sec& s = kv.second;
      if (rocsolver_zgeqrf(h, s.C, s.R, Z + s.zbase, s.C, T + s.tbase) != rocblas_status_success)
        fail(TNT_E_HIP, "rocsolver_zgeqrf failed");
    }
    // R^+ (R x k, lower triangular) before Q overwrites the factor
    std::vector<ScatterTask> st;
    mr = mc = 1;
    for (auto& kv : secs) {
      const Sec& s = kv.second;
      st.push_back(ScatterTask{s.zbase, s.C, 1, s.rbase, s.R, s.k, 1, 1});
      mr = std::max(mr, s.R);
      mc = std::max(mc, s.k);
    }
    DevBuf rbuf(&c.pool, std::max<int64_t>(1, 2 * rs) * sizeof(double));
    double* rp = rbuf.as<double>();
    DevBuf stab(&c.pool, (st.size() + S.blocks.size()) * sizeof(ScatterTask));
    TNT_HIP(hipMemcpyAsync(stab.ptr, st.data(), st.size() * sizeof(ScatterTask),
                           hipMemcpyHostToDevice, c.stream));
    launch_scatter_z(stab.as<ScatterTask>(), (int)st.size(), mr, mc, z.as<double>(), rp, rp + rs,
                     c.stream);
    for (auto& kv : secs) {
      const Sec& s = kv.second;
      if (rocsolver_zungqr(h, s.C, s.k, s.k, Z + s.zbase, s.C, T + s.tbase) !=
          rocblas_status_success)
        fail(TNT_E_HIP, "rocsolver_zungqr failed");
    }
    // new site j = Q^+: block (q, s)[r, c] = conj(Q(coff + c, r))
    SiteH Bn = make_site(newb, m.bonds[j], m.d);
    std::vector<ScatterTask> sb;
    mr = mc = 1;
    for (auto& kv : secs) {
      const Sec& s = kv.second;
      int64_t co = 0;
      for (auto& cc : s.cols) {
        const BlockRef& b = Bn.blocks.at({s.q, cc.first});
        sb.push_back(ScatterTask{s.zbase + co, s.C, 1, b.off, b.rows, b.cols, 1, 0});
        mr = std::max(mr, b.rows);
        mc = std::max(mc, b.cols);
        co += cc.second;
      }
    }
    DevBuf site(&c.pool, std::max<int64_t>(1, 2 * Bn.elems) * sizeof(double));
    launch_fill_zero(site.ptr, ET_F64, 2 * Bn.elems, c.stream);  // blocks absent before stay zero
    ScatterTask* sdev = stab.as<ScatterTask>() + st.size();
    TNT_HIP(hipMemcpyAsync(sdev, sb.data(), sb.size() * sizeof(ScatterTask),
                           hipMemcpyHostToDevice, c.stream));
    launch_scatter_z(sdev, (int)sb.size(), mr, mc, z.as<double>(), site.as<double>(),
                     site.as<double>() + Bn.elems, c.stream);
    // absorb R^+ into site j-1: A'(q', s') = A(q', s') R^+(q' + s')
    const SiteH& Ao = m.lay[j - 2];
    SiteH An;
    int64_t off = 0;
    for (auto& kv : Ao.blocks) {
      const int qr = kv.first.first + kv.first.second;
      auto it = newb.find(qr);
      if (it == newb.end()) continue;
      An.blocks[kv.first] = BlockRef{off, kv.second.rows, it->second};
      off += (int64_t)kv.second.rows * it->second;
    }
    An.elems = off;
    HostGemm g;
    for (auto& kv : An.blocks) {
      const BlockRef& ob = Ao.blocks.at(kv.first);
      const Sec& s = secs.at(kv.first.first + kv.first.second);
      g.add_task(kv.second.off, kv.second.rows, kv.second.cols, kv.second.cols);
      g.add_seg(ob.off, ob.cols, s.rbase, s.k, ob.cols);
    }
    g.finalize(default_tile_cfg(g, PATH_F64));
    DevTables t;
    t.upload(c, {&g}, {});
    DevBuf nb(&c.pool, std::max<int64_t>(1, 2 * An.elems) * sizeof(double));
    run_gemm(c, t.g[0], FORM_NN, PATH_F64, m.re(j - 1), m.im(j - 1), ET_F64, rp, rp + rs, ET_F64,
             nb.as<double>(), nb.as<double>() + An.elems, ET_F64);
    // The state is defined up to its norm (normalised at the end): site j-1
    // is scaled to unit Frobenius norm so that the norms of the R factors,
    // ~sqrt(d chi) each, do not multiply up over the chain (a random MPS of
    // 128 sites at chi = 2048 would overflow FP64).
    {
      DevBuf pn(&c.pool, RED_BLOCKS * sizeof(double) + 64);
      double* pp = pn.as<double>();
      launch_norm2_partial(nb.as<double>(), 2 * An.elems, pp, c.stream);
      launch_reduce_partials(pp, 1, RED_BLOCKS, pp + RED_BLOCKS, c.stream);
      double n2 = 0;
      TNT_HIP(hipMemcpyAsync(&n2, pp + RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost,
                             c.stream));
      TNT_HIP(hipStreamSynchronize(c.stream));
      if (!(n2 > 0) || !std::isfinite(n2))
        fail(TNT_E_NONFINITE, "MPS norm is zero or not finite at site " + std::to_string(j - 1));
      launch_scale_host(nb.as<double>(), 2 * An.elems, 1.0 / std::sqrt(n2), c.stream);
    }
    TNT_HIP(hipStreamSynchronize(c.stream));
    m.lay[j - 1] = Bn;
    m.dat[j - 1] = std::move(site);
    m.lay[j - 2] = An;
    m.dat[j - 2] = std::move(nb);
    m.bonds[j - 1] = newb;
  }
  // normalise site 1
  const int64_t n = m.lay[0].elems;
  DevBuf part(&c.pool, RED_BLOCKS * sizeof(double) + 64);
  double* p = part.as<double>();
  launch_norm2_partial(m.re(1), 2 * n, p, c.stream);
  launch_reduce_partials(p, 1, RED_BLOCKS, p + RED_BLOCKS, c.stream);
  double nrm2 = 0;
  TNT_HIP(hipMemcpyAsync(&nrm2, p + RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  if (!(nrm2 > 0) || !std::isfinite(nrm2)) fail(TNT_E_NONFINITE, "MPS norm is zero or not finite");
  launch_scale_host(m.re(1), 2 * n, 1.0 / std::sqrt(nrm2), c.stream);
}

// ---------------------------------------------------------------------------
// sweep
// ---------------------------------------------------------------------------
void dmrg_sweep(Ctx& c, MpsH& m, EnvS& e, const tnt_sweep_params& p, SweepStats& st) {
  const double t0 = now_s();
  const int64_t retries0 = c.eig_retries;
  const int L = m.L;
  if (L < 2) fail(TNT_E_STATE, "need at least two sites");
  if (p.record_cap < 2 * (L - 1) && (p.bond_E || p.bond_eps || p.bond_chi || p.bond_steps))
    fail(TNT_E_CAPACITY, "record arrays shorter than 2(L-1)");
  DevBuf theta;
  Krylov K;
  int rec = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int step = 0; step < L - 1; ++step) {
      const int j = pass == 0 ? 1 + step : L - 1 - step;
      const double tt0 = now_s();
      ThetaH th = form_theta(c, m, j, theta);
      const double tt1 = now_s();
      st.t_theta += tt1 - tt0;
      // H_eff on (j, j+1): L_{j-1}, W_j, W_{j+1}, R_{j+2}
      HeffArgs a;
      a.w1 = e.W[j - 1];
      a.w2 = e.W[j];
      a.th = th;
      a.out = th;
      a.L = e.Llay[j - 1];
      a.R = e.Rlay[j + 2];
      auto op = cached_heff(c, a, p.lanczos.precision);
      op->bind_envs(e.Lre(j - 1), e.Lim(j - 1), e.Rre(j + 2), e.Rim(j + 2));
      K.reserve(c, p.lanczos.kmax, th.elems);
      Timers tm;
      const double tl0 = now_s();
      st.t_setup += tl0 - tt1;
      LanczosOut lo =
          lanczos_run(c, *op, K, theta.as<double>(), p.lanczos, c.graphs ? nullptr : &tm);
      const double tl1 = now_s();
      st.t_matvec += tm.matvec_s;
      st.t_lanczos += (tl1 - tl0) - tm.matvec_s;
      st.matvecs += lo.matvecs;
      st.matvec_flops += (double)op->plan.flops() * (double)lo.matvecs;
      st.gemm_flops += (double)(op->plan.flops_step1 + op->plan.flops_step4) * (double)lo.matvecs;
      st.t_gemm += tm.gemm_s;
      st.gemm_launches += tm.gemm_launches;
      // split
      const int absorb = pass == 0 ? TNT_ABSORB_RIGHT : TNT_ABSORB_LEFT;
      DevBuf na, nb;
      SvdOut r = svd_truncate_dev(c, th, theta.as<double>(), theta.as<double>() + th.elems,
                                  p.trunc, absorb, [&](const SvdOut& o) {
                                    na = DevBuf(&c.pool, std::max<int64_t>(1, 2 * o.A.elems) * 8);
                                    nb = DevBuf(&c.pool, std::max<int64_t>(1, 2 * o.B.elems) * 8);
                                    FactorPlanes fp;
                                    fp.a_re = na.as<double>();
                                    fp.a_im = na.as<double>() + o.A.elems;
                                    fp.b_re = nb.as<double>();
                                    fp.b_im = nb.as<double>() + o.B.elems;
                                    return fp;
                                  });
      const double ts = now_s();
      st.t_svd += ts - tl1;
      m.bonds[j] = r.bond;
      m.lay[j - 1] = r.A;
      m.dat[j - 1] = std::move(na);
      m.lay[j] = r.B;
      m.dat[j] = std::move(nb);
      if (pass == 0) update_left_env(c, e, j);
      else update_right_env(c, e, j + 1);
      st.t_env += now_s() - ts;
      st.energy = lo.E;
      st.max_residual = std::max(st.max_residual, lo.residual);
      st.max_eps = std::max(st.max_eps, r.eps);
      st.max_chi = std::max(st.max_chi, r.chi);
      if (p.bond_E) p.bond_E[rec] = lo.E;
      if (p.bond_eps) p.bond_eps[rec] = r.eps;
      if (p.bond_chi) p.bond_chi[rec] = r.chi;
      if (p.bond_steps) p.bond_steps[rec] = lo.steps;
      ++rec;
      st.updates++;
    }
  }
  st.t_total = now_s() - t0;
  st.eig_retries = c.eig_retries - retries0;
}

// ---------------------------------------------------------------------------
// batched sweeps: every chain advances one bond update per step, in lockstep;
// the Lanczos recurrences of all chains active at a step run as one batch
// (one grouped launch per contraction step), while theta formation, the
// truncated SVD and the environment update stay per chain.
// ---------------------------------------------------------------------------
void dmrg_sweep_batched(Ctx& c, const std::vector<MpsH*>& ms, const std::vector<EnvS*>& es,
                        const tnt_sweep_params* ps, std::vector<SweepStats>& st) {
  const double t0 = now_s();
  const int64_t retries0 = c.eig_retries;
  const int nc = (int)ms.size();
  st.assign(nc, SweepStats{});
  int T = 0;
  for (int i = 0; i < nc; ++i) {
    const int L = ms[i]->L;
    if (L < 2) fail(TNT_E_STATE, "need at least two sites");
    const tnt_sweep_params& p = ps[i];
    if (p.record_cap < 2 * (L - 1) && (p.bond_E || p.bond_eps || p.bond_chi || p.bond_steps))
      fail(TNT_E_CAPACITY, "record arrays shorter than 2(L-1)");
    T = std::max(T, 2 * (L - 1));
  }
  const tnt_lanczos_params& lp = ps[0].lanczos;
  std::vector<DevBuf> theta(nc);
  std::vector<int> rec(nc, 0);
  BatchKrylov K;
  DevBuf xall;
  RunTable gather;
  double t_matvec = 0, t_lanczos = 0, t_gemm = 0, t_svd = 0, t_env = 0, t_theta = 0, t_setup = 0;
  int64_t launches = 0;
  for (int t = 0; t < T; ++t) {
    struct Act { int i, j, pass; };
    std::vector<Act> act;
    for (int i = 0; i < nc; ++i) {
      const int steps = ms[i]->L - 1;
      if (t >= 2 * steps) continue;
      const int pass = t < steps ? 0 : 1;
      const int step = pass == 0 ? t : t - steps;
      act.push_back(Act{i, pass == 0 ? 1 + step : ms[i]->L - 1 - step, pass});
    }
    std::vector<ThetaH> ths;
    std::vector<HeffArgs> hargs;
    std::vector<int64_t> nn;
    std::vector<const double *> Lr, Li, Rr, Ri;
    for (const Act& a : act) {
      MpsH& m = *ms[a.i];
      EnvS& e = *es[a.i];
      const double tt0 = now_s();
      ThetaH th = form_theta(c, m, a.j, theta[a.i]);
      const double tt1 = now_s();
      t_theta += tt1 - tt0;
      HeffArgs h;
      h.w1 = e.W[a.j - 1];
      h.w2 = e.W[a.j];
      h.th = th;
      h.out = th;
      h.L = e.Llay[a.j - 1];
      h.R = e.Rlay[a.j + 2];
      hargs.push_back(std::move(h));
      t_setup += now_s() - tt1;
      nn.push_back(th.elems);
      ths.push_back(std::move(th));
      Lr.push_back(e.Lre(a.j - 1));
      Li.push_back(e.Lim(a.j - 1));
      Rr.push_back(e.Rre(a.j + 2));
      Ri.push_back(e.Rim(a.j + 2));
    }
    const double tp0 = now_s();
    // the chains' host plans (built on several host threads), merged into
    // one batch operator: only the merged operator gets device tables
    std::vector<const HeffArgs*> hp;
    std::vector<int64_t> Lx, Rx;
    for (const HeffArgs& h : hargs) {
      hp.push_back(&h);
      Lx.push_back(h.L.extent);
      Rx.push_back(h.R.extent);
    }
    std::vector<std::shared_ptr<HeffPlan>> plans = cached_plans(c, hp, lp.precision);
    t_setup += now_s() - tp0;
    const double tb0 = now_s();
    auto B = cached_plan_batch(c, plans, Lx, Rx, nn, lp.precision);
    bind_batch_envs(c, *B, Lr, Li, Rr, Ri);
    xall.ensure(&c.pool, std::max<int64_t>(1, 2 * B->N) * sizeof(double));
    double* x = xall.as<double>();
    {
      std::vector<CopyRun> runs;
      for (size_t a = 0; a < act.size(); ++a) {
        const int64_t n = nn[a], off = B->parts[a].x_off;
        const double* src = theta[act[a].i].as<double>();
        runs.push_back(CopyRun{src, x + off, n});
        runs.push_back(CopyRun{src + n, x + B->N + off, n});
      }
      gather.run(c, runs);
    }
    t_setup += now_s() - tb0;
    Timers tm;
    std::vector<LanczosOut> lo;
    const double tl0 = now_s();
    lanczos_run_batched(c, *B, K, x, lp, lo, c.graphs ? nullptr : &tm);
    const double tl1 = now_s();
    t_matvec += tm.matvec_s;
    t_lanczos += (tl1 - tl0) - tm.matvec_s;
    t_gemm += tm.gemm_s;
    launches += tm.gemm_launches;
    // the sector eigendecompositions of every chain of the step share one
    // set of batched calls
    const double te0 = now_s();
    std::vector<std::shared_ptr<SvdJob>> jobs;
    std::vector<SvdJob*> jp;
    for (size_t a = 0; a < act.size(); ++a) {
      if (ps[act[a].i].trunc.chi_max < 1) fail(TNT_E_ARG, "chi_max must be >= 1");
      const int64_t off = B->parts[a].x_off;
      jobs.push_back(svd_begin(c, ths[a], x + off, x + B->N + off,
                               act[a].pass == 0 ? TNT_ABSORB_RIGHT : TNT_ABSORB_LEFT));
      jp.push_back(jobs.back().get());
    }
    svd_eig(c, jp);
    {
      std::vector<tnt_trunc_params> tp;
      for (size_t a = 0; a < act.size(); ++a) tp.push_back(ps[act[a].i].trunc);
      svd_refine(c, jp, tp);
    }
    t_svd += now_s() - te0;
    for (size_t a = 0; a < act.size(); ++a) {
      const int i = act[a].i, j = act[a].j, pass = act[a].pass;
      MpsH& m = *ms[i];
      EnvS& e = *es[i];
      const tnt_sweep_params& p = ps[i];
      SweepStats& s = st[i];
      const HeffPlan& pl = *plans[a];
      s.matvecs += lo[a].matvecs;
      s.matvec_flops += (double)pl.flops() * (double)lo[a].matvecs;
      s.gemm_flops += (double)(pl.flops_step1 + pl.flops_step4) * (double)lo[a].matvecs;
      DevBuf na, nb;
      const double ts0 = now_s();
      SvdOut r = svd_finish(c, *jobs[a], p.trunc, [&](const SvdOut& o) {
        na = DevBuf(&c.pool, std::max<int64_t>(1, 2 * o.A.elems) * 8);
        nb = DevBuf(&c.pool, std::max<int64_t>(1, 2 * o.B.elems) * 8);
        FactorPlanes fp;
        fp.a_re = na.as<double>();
        fp.a_im = na.as<double>() + o.A.elems;
        fp.b_re = nb.as<double>();
        fp.b_im = nb.as<double>() + o.B.elems;
        return fp;
      });
      const double ts = now_s();
      t_svd += ts - ts0;
      m.bonds[j] = r.bond;
      m.lay[j - 1] = r.A;
      m.dat[j - 1] = std::move(na);
      m.lay[j] = r.B;
      m.dat[j] = std::move(nb);
      if (pass == 0) update_left_env(c, e, j);
      else update_right_env(c, e, j + 1);
      t_env += now_s() - ts;
      s.energy = lo[a].E;
      s.max_residual = std::max(s.max_residual, lo[a].residual);
      s.max_eps = std::max(s.max_eps, r.eps);
      s.max_chi = std::max(s.max_chi, r.chi);
      if (p.bond_E) p.bond_E[rec[i]] = lo[a].E;
      if (p.bond_eps) p.bond_eps[rec[i]] = r.eps;
      if (p.bond_chi) p.bond_chi[rec[i]] = r.chi;
      if (p.bond_steps) p.bond_steps[rec[i]] = lo[a].steps;
      ++rec[i];
      s.updates++;
    }
  }
  // batch-level timings (the chains share every launch)
  const double total = now_s() - t0;
  for (SweepStats& s : st) {
    s.t_total = total;
    s.eig_retries = c.eig_retries - retries0;
    s.t_matvec = t_matvec;
    s.t_lanczos = t_lanczos;
    s.t_gemm = t_gemm;
    s.gemm_launches = launches;
    s.t_svd = t_svd;
    s.t_env = t_env;
    s.t_theta = t_theta;
    s.t_setup = t_setup;
  }
}

}  // namespace tnt
