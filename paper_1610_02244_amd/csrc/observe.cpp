// Two-point correlations <O^dagger_i O_j> of a block MPS for every pair of
// sites: with O = b the single-particle density matrix rho_ij and, on its
// diagonal, the densities <n_j> (the outputs of the ground-state example of
// Sec. 5, Fig. fig:ground_state_results).
//
// One pass from left to right carries, at bond k, one environment channel
// per open string: channel 0 is the plain norm environment and channel i
// (i < k) holds the network of sites 1..k with O^dagger inserted at site i.
// At site k, with P[w] = S_{k-1}[w] A_k (one grouped GEMM over every
// channel and physical index):
//   - string i is closed with O at site k and the rest of the chain:
//       <O^dagger_i O_k> = sum_{s,s'} O_{s's} <P[i](s), G(s')>,
//     where G(s') = A_k(s') R_{k+1}^T is the product of the site with the
//     norm environment of sites k+1..L (Hermitian, so the conjugate of the
//     needed contraction is this NT product);
//   - the norm channel gives <psi|psi> and <(O^dagger O)_k> the same way;
//   - every string is carried on with the identity (S_k[i] = sum_s
//     A_k(s)^H P[i](s)) and string k is opened from the norm channel with
//     O^dagger.
// So a site costs two grouped GEMMs over its k live channels, one GEMM with
// the norm environment, one combine and one launch of block dot products;
// the whole pass is O(L^2 chi^3 d) flops in FP64 grouped-GEMM launches.
#include <array>
#include <complex>
#include <map>

#include "dmrg.h"
#include "kernels.h"

namespace tnt {

void correlation_matrix(Ctx& c, MpsH& m, const std::vector<double>& op, int dq,
                        std::vector<std::complex<double>>& C, double* flops) {
  const int L = m.L, d = m.d;
  auto dim = [](const Bond& b, int q) {
    auto it = b.find(q);
    return it == b.end() ? 0 : it->second;
  };
  double fl = 0.0;
  // norm environments R_j of sites j..L (j = 2..L+1): the D = 1 identity MPO
  EnvS e;
  e.mps = &m;
  MpoH I;
  I.d = d;
  I.D = 1;
  I.qw = {0};
  I.W.assign((size_t)d * d, 0.0);
  for (int s = 0; s < d; ++s) I.W[(size_t)s * d + s] = 1.0;
  e.W.assign(L, I);
  e.qw = {0};
  e.left_index = e.right_index = 0;
  build_boundaries(c, e);
  for (int j = L; j >= 2; --j) update_right_env(c, e, j);

  C.assign((size_t)L * L, std::complex<double>(0.0, 0.0));
  // string environment at bond k-1: channel charges (bra = ket + q[w])
  std::vector<int> qcur = {0};
  EnvH S = e.Llay[0];
  DevBuf Sd = std::move(e.Ldat[0]);
  std::vector<double> hout;
  for (int k = 1; k <= L; ++k) {
    const SiteH& A = m.lay[k - 1];
    const Bond& br = m.bonds[k];
    const EnvH& R = e.Rlay[k + 1];
    const double* are = m.re(k);
    const double* aim = m.im(k);
    // P[w; c', s, a] = S[w](c', c) A(c, s)(c, a)
    HostGemm gp;
    std::map<std::array<int, 3>, int64_t> poff;
    int64_t ps = 0;
    for (auto& sb : S.blocks) {
      const int w = sb.first.first, q = sb.first.second;
      for (int s = 0; s < d; ++s) {
        auto ia = A.blocks.find({q, s});
        if (ia == A.blocks.end()) continue;
        const int M = sb.second.rows, N = ia->second.cols, K = sb.second.cols;
        poff[{w, q, s}] = ps;
        gp.add_task(ps, M, N, N);
        gp.add_seg(sb.second.off, K, ia->second.off, N, K);
        ps += (int64_t)M * N;
      }
    }
    // G(c', s') = A(c', s') R_{k+1}(a', a)^T
    HostGemm gg;
    std::map<std::pair<int, int>, int64_t> goff;
    int64_t gs = 0;
    for (auto& ab : A.blocks) {
      const int qc = ab.first.first, s = ab.first.second;
      auto ir = R.blocks.find({0, qc + s});
      if (ir == R.blocks.end()) continue;
      const int M = ab.second.rows, N = ir->second.rows, K = ab.second.cols;
      goff[{qc, s}] = gs;
      gg.add_task(gs, M, N, N);
      gg.add_seg(ab.second.off, K, ir->second.off, ir->second.cols, K);
      gs += (int64_t)M * N;
    }
    // dot products, slot 0 = norm, 1 = diagonal, 1 + i = string opened at i
    std::vector<DotTask> dots;
    std::vector<int> slot;
    for (auto& p : poff) {
      const int w = p.first[0], q = p.first[1], s = p.first[2];
      const int qb = q + qcur[w];
      for (int sp = 0; sp < d; ++sp) {
        if (qb + sp != q + s) continue;  // G(qb, s') must have P's columns
        auto ig = goff.find({qb, sp});
        if (ig == goff.end()) continue;
        const int n = dim(m.bonds[k - 1], qb) * dim(br, q + s);
        if (n == 0) continue;
        if (w == 0) {
          if (sp != s) continue;
          double dd = 0.0;  // (O^dagger O)_{ss}
          for (int t = 0; t < d; ++t) dd += op[(size_t)t * d + s] * op[(size_t)t * d + s];
          dots.push_back(DotTask{p.second, ig->second, n, 0, 1.0});
          slot.push_back(0);
          if (dd != 0.0) {
            dots.push_back(DotTask{p.second, ig->second, n, 0, dd});
            slot.push_back(1);
          }
        } else {
          const double cf = op[(size_t)sp * d + s];
          if (cf == 0.0) continue;
          dots.push_back(DotTask{p.second, ig->second, n, 0, cf});
          slot.push_back(1 + w);
        }
      }
    }
    // new string k: Y(c', s') = sum_s O^dagger_{s's} P[0](c', s); O^dagger
    // moves s to s' = s - dq, so Y(c', s') has columns a = c' + s' + dq
    std::map<std::pair<int, int>, std::vector<std::pair<int64_t, double>>> yterms;
    for (auto& p : poff) {
      if (p.first[0] != 0) continue;
      const int q = p.first[1], s = p.first[2];
      for (int sp = 0; sp < d; ++sp) {
        const double cf = op[(size_t)s * d + sp];  // <s'|O^dagger|s> = O_{s s'}
        if (cf != 0.0) yterms[{q, sp}].push_back({p.second, cf});
      }
    }
    HostComb cyo;
    std::map<std::pair<int, int>, int64_t> yoff;
    int64_t ys = 0;
    for (auto& y : yterms) {
      const int q = y.first.first, sp = y.first.second;
      const int64_t size = (int64_t)dim(m.bonds[k - 1], q) * dim(br, q + sp + dq);
      if (size == 0) continue;
      yoff[y.first] = ys;
      cyo.add_task(ys, (int)size);
      for (auto& t : y.second) cyo.add_term(t.first, t.second);
      ys += size;
    }
    cyo.finalize();
    // S_k: channels 0..k-1 carried on, channel k opened
    std::vector<int> qnext = qcur;
    qnext.push_back(-dq);
    EnvH Sn = make_env(br, qnext);
    HostGemm gs2;
    for (auto& sb : Sn.blocks) {
      const int w = sb.first.first, qa = sb.first.second;
      const int M = sb.second.rows, N = sb.second.cols;
      gs2.add_task(sb.second.off, M, N, N);
      const int abra = qa + qnext[w];
      for (int sp = 0; sp < d; ++sp) {
        const int qc = abra - sp;
        auto ia = A.blocks.find({qc, sp});
        if (ia == A.blocks.end()) continue;
        int64_t boff = -1;
        if (w < k) {
          auto ip = poff.find({w, qc - qcur[w], sp});
          if (ip != poff.end()) boff = ip->second;
        } else {
          auto iy = yoff.find({qc, sp});
          if (iy != yoff.end()) boff = ps + iy->second;
        }
        if (boff < 0) continue;
        gs2.add_seg(ia->second.off, ia->second.cols, boff, N, ia->second.rows);
      }
    }
    fl += gp.flops + gg.flops + gs2.flops + cyo.flops;
    const bool has_p = !gp.tasks.empty(), has_g = !gg.tasks.empty();
    const bool has_y = !cyo.tasks.empty(), has_s = !gs2.tasks.empty();
    if (has_p) gp.finalize(default_tile_cfg(gp, PATH_F64));
    if (has_g) gg.finalize(default_tile_cfg(gg, PATH_F64));
    if (has_s) gs2.finalize(default_tile_cfg(gs2, PATH_F64));
    DevTables t;
    t.upload(c, {&gp, &gg, &gs2}, {&cyo});
    const int64_t tot = ps + ys;
    DevBuf PY(&c.pool, std::max<int64_t>(1, 2 * tot) * sizeof(double));
    DevBuf G(&c.pool, std::max<int64_t>(1, 2 * gs) * sizeof(double));
    DevBuf Sout(&c.pool, std::max<int64_t>(1, 2 * Sn.elems) * sizeof(double));
    DevBuf Dt(&c.pool, std::max<size_t>(1, dots.size()) * sizeof(DotTask));
    DevBuf Do(&c.pool, std::max<size_t>(1, 2 * dots.size()) * sizeof(double));
    double* py = PY.as<double>();
    double* g = G.as<double>();
    double* so = Sout.as<double>();
    const double* sre = Sd.as<double>();
    const double* sim = sre + S.elems;
    if (!dots.empty())
      TNT_HIP(hipMemcpyAsync(Dt.ptr, dots.data(), dots.size() * sizeof(DotTask),
                             hipMemcpyHostToDevice, c.stream));
    if (has_p)
      run_gemm(c, t.g[0], FORM_NN, PATH_F64, sre, sim, ET_F64, are, aim, ET_F64, py, py + tot,
               ET_F64);
    if (has_g)
      run_gemm(c, t.g[1], FORM_NT, PATH_F64, are, aim, ET_F64, e.Rre(k + 1), e.Rim(k + 1),
               ET_F64, g, g + gs, ET_F64);
    if (!dots.empty())
      launch_block_dots(Dt.as<DotTask>(), (int)dots.size(), py, py + tot, g, g + gs,
                        Do.as<double>(), c.stream);
    if (has_y) run_comb(c, t.c[0], py, py + tot, py + ps, py + tot + ps, ET_F64);
    if (has_s)
      run_gemm(c, t.g[2], FORM_CN, PATH_F64, are, aim, ET_F64, py, py + tot, ET_F64, so,
               so + Sn.elems, ET_F64);
    hout.assign(2 * dots.size(), 0.0);
    if (!dots.empty())
      TNT_HIP(hipMemcpyAsync(hout.data(), Do.ptr, hout.size() * sizeof(double),
                             hipMemcpyDeviceToHost, c.stream));
    TNT_HIP(hipStreamSynchronize(c.stream));
    // fixed-order sums per slot
    std::vector<std::complex<double>> acc(k + 1, std::complex<double>(0.0, 0.0));
    for (size_t i = 0; i < dots.size(); ++i)
      acc[slot[i]] += std::complex<double>(hout[2 * i], hout[2 * i + 1]);
    const double nrm = acc[0].real();
    if (!(nrm > 0.0)) fail(TNT_E_STATE, "MPS has zero norm");
    C[(size_t)(k - 1) * L + (k - 1)] = acc[1] / nrm;
    for (int i = 1; i < k; ++i) {
      const std::complex<double> v = acc[1 + i] / nrm;
      C[(size_t)(i - 1) * L + (k - 1)] = v;
      C[(size_t)(k - 1) * L + (i - 1)] = std::conj(v);
    }
    S = std::move(Sn);
    Sd = std::move(Sout);
    qcur = std::move(qnext);
  }
  if (flops) *flops = fl;
}

}  // namespace tnt
