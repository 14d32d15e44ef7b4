// Task-list construction for the grouped kernels and the two-site H_eff plan.
#include "plan.h"

#include <climits>

#include <algorithm>
#include <cstring>
#include <exception>
#include <functional>
#include <numeric>
#include <set>
#include <thread>

namespace tnt {

// ---------------------------------------------------------------------------
// tile tables
// ---------------------------------------------------------------------------
void HostGemm::finalize(int cfg) {
  tile_cfg = cfg;
  tiles = build_tiles(cfg);
  var_cfg.clear();
  var_tiles.clear();
}

void HostGemm::add_variant(int cfg) {
  if (cfg == tile_cfg) return;
  for (int v : var_cfg)
    if (v == cfg) return;
  var_cfg.push_back(cfg);
  var_tiles.push_back(build_tiles(cfg));
}

std::vector<int2> HostGemm::build_tiles(int cfg) const {
  std::vector<int2> tiles;
  int BM, BN;
  gemm_tile_dims(cfg, &BM, &BN);
  const int nt = (int)tasks.size();
  std::vector<double> cost(nt);
  std::vector<int> order(nt);
  for (int i = 0; i < nt; ++i) {
    const GemmTask& t = tasks[i];
    int64_t ksum = 0;
    for (int s = 0; s < t.nseg; ++s) ksum += segs[t.seg0 + s].K;
    const int tm = (t.M + BM - 1) / BM, tn = (t.N + BN - 1) / BN;
    // a tile's cost ~ padded K work plus a fixed overhead (prologue/epilogue)
    cost[i] = (double)tm * tn * (double)(ksum + 64);
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<std::vector<int2>> bins(8);
  double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i : order) {
    const GemmTask& t = tasks[i];
    int x = 0;
    for (int k = 1; k < 8; ++k)
      if (load[k] < load[x]) x = k;
    load[x] += cost[i];
    const int tm = (t.M + BM - 1) / BM, tn = (t.N + BN - 1) / BN;
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) bins[x].push_back(int2{i, a | (b << 16)});
  }
  // within a bin, longest tiles (largest K) first: the dispatcher hands
  // tiles out in table order, so the short ones fill the tail
  std::vector<int64_t> tk(nt);
  for (int i = 0; i < nt; ++i) {
    int64_t ksum = 0;
    for (int s = 0; s < tasks[i].nseg; ++s) ksum += segs[tasks[i].seg0 + s].K;
    tk[i] = ksum;
  }
  for (auto& b : bins)
    std::stable_sort(b.begin(), b.end(), [&](const int2& u, const int2& v) { return tk[u.x] > tk[v.x]; });
  size_t slots = 0;
  for (auto& b : bins) slots = std::max(slots, b.size());
  tiles.assign(slots * 8, int2{-1, 0});
  for (size_t s = 0; s < slots; ++s)
    for (int x = 0; x < 8; ++x)
      if (s < bins[x].size()) tiles[s * 8 + x] = bins[x][s];
  return tiles;
}

std::vector<int> tile_candidates(GemmPath path) {
  if (path != PATH_F32) return {0, 1, 2, 3};
  return {0, 1, 2, 3, 4};
}

GemmPath gemm_path(int precision) {
  return precision == TNT_FP64 ? PATH_F64 : precision == TNT_BF16X3 ? PATH_BF16X3 : PATH_F32;
}

uint64_t tune_bucket(const HostGemm& h, GemmPath path, int which) {
  double wsum = 0, dsum = 0;
  for (const GemmTask& t : h.tasks) {
    double k = 0;
    for (int s = 0; s < t.nseg; ++s) k += h.segs[t.seg0 + s].K;
    const double f = (double)t.M * t.N * k;
    wsum += f;
    dsum += f * std::min(t.M, t.N);
  }
  const int typ = wsum > 0 ? (int)std::lround(4.0 * std::log2(std::max(1.0, dsum / wsum))) : 0;
  const int lf = wsum > 0 ? (int)std::lround(std::log2(wsum)) : 0;
  return ((uint64_t)path << 48) | ((uint64_t)which << 40) | ((uint64_t)(typ & 0xffff) << 16) |
         (uint64_t)(lf & 0xffff);
}

void HostComb::finalize() {
  chunks.clear();
  for (int i = 0; i < (int)tasks.size(); ++i) {
    const int n = (tasks[i].size + COMB_CHUNK - 1) / COMB_CHUNK;
    for (int c = 0; c < n; ++c) chunks.push_back(int2{i, c});
  }
}

void HostCombP::finalize() {
  chunks.clear();
  for (int i = 0; i < (int)tasks.size(); ++i) {
    const int64_t total = (int64_t)tasks[i].rows * tasks[i].dld;
    const int n = (int)((total + COMB_CHUNK - 1) / COMB_CHUNK);
    for (int c = 0; c < n; ++c) chunks.push_back(int2{i, c});
  }
}

int64_t HostPack::add(int64_t src_off, int rows, int cols, int sld, bool trans) {
  const int dld = (int)pad8(cols);
  const int64_t off = elems;
  const int ti = (int)tasks.size();
  tasks.push_back(PackTask{src_off, off, rows, cols, sld, dld, trans ? 1 : 0, 0});
  const int tr = (rows + PACK_TILE - 1) / PACK_TILE, tc = (dld + PACK_TILE - 1) / PACK_TILE;
  for (int a = 0; a < tr; ++a)
    for (int b = 0; b < tc; ++b) tiles.push_back(int2{ti, a | (b << 16)});
  elems += (int64_t)rows * dld;  // rows * dld is a multiple of 8
  return off;
}

// GEMM steps below this many flops are not tuned: such a launch takes a few
// tens of microseconds, mostly dispatch and tail, and timing the candidates
// (with a host wait per timed launch) costs more than a better shape saves.
constexpr double kTuneMinFlops = 1e9;

// Tile shape without timing.  The rule reproduces the autotuner's choices
// over every GEMM step of a chi = 256 and a chi = 1024 sweep (about 210
// steps per path, 1e3 .. 2e10 flops): on the FP32 and FP64 paths 32 x 32
// tiles win unless the step is large in both tile count and block size
// (more tiles fill the 256 CUs; only big L.theta steps gain from 64 x 64);
// on the BF16x3 path 64 x 64 wins from a typical block size of about 48.
int default_tile_cfg(const HostGemm& h, GemmPath path) {
  // flop-weighted typical output dimension, and the 64 x 64 tile count
  double wsum = 0, dsum = 0;
  int64_t tiles64 = 0;
  for (const GemmTask& t : h.tasks) {
    double k = 0;
    for (int s = 0; s < t.nseg; ++s) k += h.segs[t.seg0 + s].K;
    const double f = (double)t.M * t.N * k;
    wsum += f;
    dsum += f * std::min(t.M, t.N);
    tiles64 += (int64_t)((t.M + 63) / 64) * ((t.N + 63) / 64);
  }
  const double typ = wsum > 0 ? dsum / wsum : 0;
  if (path == PATH_BF16X3) return typ < 48 ? 1 : 0;  // 32 x 32, else 64 x 64
  return tiles64 >= 1024 && typ >= 100 ? 0 : 1;       // 64 x 64, else 32 x 32
}

// ---------------------------------------------------------------------------
// device tables
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t DevTables::image_bytes(const std::vector<const HostGemm*>& gs,
                              const std::vector<const HostComb*>& cs,
                              const std::vector<const HostCombP*>& cps,
                              const std::vector<const HostPack*>& pks) {
  size_t total = 0;
  auto add = [&](size_t bytes) { total = align256(total + bytes); };
  for (auto* h : gs) {
    add(h->tasks.size() * sizeof(GemmTask));
    add(h->segs.size() * sizeof(GemmSeg));
    add(h->tiles.size() * sizeof(int2));
    for (auto& vt : h->var_tiles) add(vt.size() * sizeof(int2));
  }
  for (auto* h : cs) {
    add(h->tasks.size() * sizeof(CombTask));
    add(h->terms.size() * sizeof(CombTerm));
    add(h->chunks.size() * sizeof(int2));
  }
  for (auto* h : cps) {
    add(h->tasks.size() * sizeof(CombPTask));
    add(h->terms.size() * sizeof(CombTerm));
    add(h->chunks.size() * sizeof(int2));
  }
  for (auto* h : pks) {
    add(h->tasks.size() * sizeof(PackTask));
    add(h->tiles.size() * sizeof(int2));
  }
  return std::max<size_t>(total, 256);
}

void DevTables::upload(Ctx& ctx, const std::vector<const HostGemm*>& gs,
                       const std::vector<const HostComb*>& cs,
                       const std::vector<const HostCombP*>& cps,
                       const std::vector<const HostPack*>& pks, void* dst) {
  size_t total = 0;
  auto add = [&](size_t bytes) { size_t o = total; total = align256(total + bytes); return o; };
  struct GO { size_t t, s, l; std::vector<size_t> v; };
  struct CO { size_t t, m, c; };
  std::vector<GO> go;
  std::vector<CO> co;
  for (auto* h : gs) {
    GO o{add(h->tasks.size() * sizeof(GemmTask)), add(h->segs.size() * sizeof(GemmSeg)),
         add(h->tiles.size() * sizeof(int2)), {}};
    for (auto& vt : h->var_tiles) o.v.push_back(add(vt.size() * sizeof(int2)));
    go.push_back(o);
  }
  for (auto* h : cs)
    co.push_back({add(h->tasks.size() * sizeof(CombTask)),
                  add(h->terms.size() * sizeof(CombTerm)), add(h->chunks.size() * sizeof(int2))});
  std::vector<CO> cpo;
  for (auto* h : cps)
    cpo.push_back({add(h->tasks.size() * sizeof(CombPTask)),
                   add(h->terms.size() * sizeof(CombTerm)), add(h->chunks.size() * sizeof(int2))});
  struct PO { size_t t, l; };
  std::vector<PO> po;
  for (auto* h : pks)
    po.push_back({add(h->tasks.size() * sizeof(PackTask)), add(h->tiles.size() * sizeof(int2))});
  total = std::max<size_t>(total, 256);
  host.assign(total, 0);
  for (size_t i = 0; i < gs.size(); ++i) {
    auto* h = gs[i];
    if (!h->tasks.empty()) memcpy(&host[go[i].t], h->tasks.data(), h->tasks.size() * sizeof(GemmTask));
    if (!h->segs.empty()) memcpy(&host[go[i].s], h->segs.data(), h->segs.size() * sizeof(GemmSeg));
    if (!h->tiles.empty()) memcpy(&host[go[i].l], h->tiles.data(), h->tiles.size() * sizeof(int2));
    for (size_t v = 0; v < h->var_tiles.size(); ++v)
      if (!h->var_tiles[v].empty())
        memcpy(&host[go[i].v[v]], h->var_tiles[v].data(), h->var_tiles[v].size() * sizeof(int2));
  }
  for (size_t i = 0; i < cs.size(); ++i) {
    auto* h = cs[i];
    if (!h->tasks.empty()) memcpy(&host[co[i].t], h->tasks.data(), h->tasks.size() * sizeof(CombTask));
    if (!h->terms.empty()) memcpy(&host[co[i].m], h->terms.data(), h->terms.size() * sizeof(CombTerm));
    if (!h->chunks.empty()) memcpy(&host[co[i].c], h->chunks.data(), h->chunks.size() * sizeof(int2));
  }
  auto put = [&](size_t at, const void* src, size_t bytes) {
    if (bytes) memcpy(&host[at], src, bytes);
  };
  for (size_t i = 0; i < cps.size(); ++i) {
    auto* h = cps[i];
    put(cpo[i].t, h->tasks.data(), h->tasks.size() * sizeof(CombPTask));
    put(cpo[i].m, h->terms.data(), h->terms.size() * sizeof(CombTerm));
    put(cpo[i].c, h->chunks.data(), h->chunks.size() * sizeof(int2));
  }
  for (size_t i = 0; i < pks.size(); ++i) {
    put(po[i].t, pks[i]->tasks.data(), pks[i]->tasks.size() * sizeof(PackTask));
    put(po[i].l, pks[i]->tiles.data(), pks[i]->tiles.size() * sizeof(int2));
  }
  char* base;
  if (dst) {
    buf.reset();
    base = static_cast<char*>(dst);
  } else {
    buf = DevBuf(&ctx.pool, total);
    base = buf.as<char>();
  }
  TNT_HIP(hipMemcpyAsync(base, host.data(), total, hipMemcpyHostToDevice, ctx.stream));
  g.clear();
  c.clear();
  cp.clear();
  p.clear();
  for (size_t i = 0; i < gs.size(); ++i) {
    G x{};
    x.tasks = reinterpret_cast<const GemmTask*>(base + go[i].t);
    x.segs = reinterpret_cast<const GemmSeg*>(base + go[i].s);
    x.tiles[0] = reinterpret_cast<const int2*>(base + go[i].l);
    x.ntiles[0] = (int)gs[i]->tiles.size();
    x.cfg[0] = gs[i]->tile_cfg;
    x.nvar = 1;
    for (size_t v = 0; v < gs[i]->var_tiles.size() && x.nvar < 8; ++v, ++x.nvar) {
      x.tiles[x.nvar] = reinterpret_cast<const int2*>(base + go[i].v[v]);
      x.ntiles[x.nvar] = (int)gs[i]->var_tiles[v].size();
      x.cfg[x.nvar] = gs[i]->var_cfg[v];
    }
    x.sel = 0;
    g.push_back(x);
  }
  for (size_t i = 0; i < cs.size(); ++i)
    c.push_back(C{reinterpret_cast<const CombTask*>(base + co[i].t),
                  reinterpret_cast<const CombTerm*>(base + co[i].m),
                  reinterpret_cast<const int2*>(base + co[i].c), (int)cs[i]->chunks.size()});
  for (size_t i = 0; i < cps.size(); ++i)
    cp.push_back(CP{reinterpret_cast<const CombPTask*>(base + cpo[i].t),
                    reinterpret_cast<const CombTerm*>(base + cpo[i].m),
                    reinterpret_cast<const int2*>(base + cpo[i].c), (int)cps[i]->chunks.size()});
  for (size_t i = 0; i < pks.size(); ++i)
    p.push_back(P{reinterpret_cast<const PackTask*>(base + po[i].t),
                  reinterpret_cast<const int2*>(base + po[i].l), (int)pks[i]->tiles.size(),
                  pks[i]->elems});
}

void run_gemm(Ctx& ctx, const DevTables::G& g, GemmForm form, GemmPath path, const void* are,
              const void* aim, ElemType at, const void* bre, const void* bim, ElemType bt,
              void* cre, void* cim, ElemType ct) {
  run_gemm_variant(ctx, g, g.sel, form, path, are, aim, at, bre, bim, bt, cre, cim, ct);
}

void run_gemm_variant(Ctx& ctx, const DevTables::G& g, int v, GemmForm form, GemmPath path,
                      const void* are, const void* aim, ElemType at, const void* bre,
                      const void* bim, ElemType bt, void* cre, void* cim, ElemType ct) {
  if (v < 0 || v >= g.nvar) fail(TNT_E_STATE, "tile-table variant out of range");
  GemmLaunch L{g.tasks, g.segs, g.tiles[v], g.ntiles[v], g.cfg[v], are, aim, at,
               bre,     bim,    bt,         cre,         cim,        ct,  form, path};
  if (!launch_grouped_gemm(L, ctx.stream))
    fail(TNT_E_STATE, "grouped GEMM variant not available (path " + std::to_string(path) +
                          ", tile shape " + std::to_string(g.cfg[v]) + ")");
}

// index of a tile table usable by `path` (the selected one if valid)
static int valid_variant(const DevTables::G& g, GemmPath path) {
  if (gemm_cfg_valid(g.cfg[g.sel], path)) return g.sel;
  for (int v = 0; v < g.nvar; ++v)
    if (gemm_cfg_valid(g.cfg[v], path)) return v;
  fail(TNT_E_STATE, "no tile table valid for this precision");
}

void run_comb(Ctx& ctx, const DevTables::C& c, const void* sre, const void* sim, void* dre,
              void* dim, ElemType t) {
  launch_combine(c.tasks, c.terms, c.chunks, c.nchunks, sre, sim, dre, dim, t, ctx.stream);
}

// ---------------------------------------------------------------------------
// H_eff plan
// ---------------------------------------------------------------------------
HeffPlan build_heff_plan(const EnvH& L, const MpoH& W1, const MpoH& W2, const EnvH& R,
                         const ThetaH& th, const ThetaH& out, bool packed) {
  HeffPlan P;
  P.packed = packed;
  const int D = W1.D, d = th.d;
  const Bond& left = th.left;
  const Bond& right = th.right;
  // dense charge indices (the block maps are only walked, never searched)
  auto span = [](const Bond& a, const Bond& b, int& lo, int& hi) {
    lo = INT_MAX;
    hi = INT_MIN;
    for (const Bond* x : {&a, &b})
      if (!x->empty()) {
        lo = std::min(lo, x->begin()->first);
        hi = std::max(hi, x->rbegin()->first);
      }
    if (lo > hi) lo = hi = 0;
  };
  int llo, lhi, rlo, rhi;
  span(left, L.bond, llo, lhi);
  span(right, R.bond, rlo, rhi);
  const int nl = lhi - llo + 1, nr = rhi - rlo + 1;
  auto li = [&](int q) { return q < llo || q > lhi ? -1 : q - llo; };
  auto ri = [&](int q) { return q < rlo || q > rhi ? -1 : q - rlo; };
  std::vector<int> ldim(nl, 0), rdim(nr, 0);
  for (auto& kv : left) ldim[kv.first - llo] = kv.second;
  for (auto& kv : right) rdim[kv.first - rlo] = kv.second;
  std::vector<const BlockRef*> Lb((size_t)D * nl, nullptr), Rb((size_t)D * nr, nullptr),
      Tb((size_t)nl * d * d, nullptr);
  for (auto& b : L.blocks) {
    const int q = li(b.first.second);
    if (q >= 0) Lb[(size_t)b.first.first * nl + q] = &b.second;
  }
  for (auto& b : R.blocks) {
    const int q = ri(b.first.second);
    if (q >= 0) Rb[(size_t)b.first.first * nr + q] = &b.second;
  }
  auto tix = [&](int q, int s1, int s2) { return ((size_t)q * d + s1) * d + s2; };
  for (auto& b : th.blocks) {
    const int q = li(b.first[0]);
    if (q >= 0) Tb[tix(q, b.first[1], b.first[2])] = &b.second;
  }
  // packed operand copies: every L and R block as stored, theta blocks
  // transposed (K = dim(q_a) becomes the contiguous index)
  std::vector<int64_t> lp_off, rp_off, xp_off;
  if (packed) {
    lp_off.assign((size_t)D * nl, -1);
    rp_off.assign((size_t)D * nr, -1);
    xp_off.assign((size_t)nl * d * d, -1);
    for (auto& b : L.blocks) {
      const int64_t o = P.Lp.add(b.second.off, b.second.rows, b.second.cols, b.second.cols, false);
      const int q = li(b.first.second);
      if (q >= 0) lp_off[(size_t)b.first.first * nl + q] = o;
    }
    for (auto& b : R.blocks) {
      const int64_t o = P.Rp.add(b.second.off, b.second.rows, b.second.cols, b.second.cols, false);
      const int q = ri(b.first.second);
      if (q >= 0) rp_off[(size_t)b.first.first * nr + q] = o;
    }
    for (auto& b : th.blocks) {
      const int64_t o = P.Xp.add(b.second.off, b.second.cols, b.second.rows, b.second.cols, true);
      const int q = li(b.first[0]);
      if (q >= 0) xp_off[tix(q, b.first[1], b.first[2])] = o;
    }
  }
  // combined two-site MPO coefficients sum_v W1[w,v,s1',s1] W2[v,u,s2',s2],
  // kept as the list of nonzero (w, s1, s2) terms per (u, s1', s2'), in
  // ascending (w, s1, s2) order
  struct MTerm { int w, s1, s2; double c; };
  std::vector<std::vector<MTerm>> mterms((size_t)D * d * d);
  for (int u = 0; u < D; ++u)
    for (int s1p = 0; s1p < d; ++s1p)
      for (int s2p = 0; s2p < d; ++s2p)
        for (int w = 0; w < D; ++w)
          for (int s1 = 0; s1 < d; ++s1)
            for (int s2 = 0; s2 < d; ++s2) {
              double c = 0.0;
              for (int v = 0; v < D; ++v) c += W1.at(w, v, s1p, s1) * W2.at(v, u, s2p, s2);
              if (c != 0.0) mterms[((size_t)u * d + s1p) * d + s2p].push_back(MTerm{w, s1, s2, c});
            }
  // T1 slab (w, q_a, s1, s2) -> index in the dense table; the slabs are laid
  // out in ascending (w, q_a, s1, s2) order
  auto t1x = [&](int w, int q, int s1, int s2) { return (size_t)w * nl * d * d + tix(q, s1, s2); };
  struct Term { size_t t1; double c; };
  struct Slab { int u, qi, s1p, s2p, qbi; std::vector<Term> terms; };
  std::vector<Slab> live;
  constexpr int64_t kUnused = -2, kUsed = -1;
  std::vector<int64_t> t1_off((size_t)D * nl * d * d, kUnused);
  for (auto& ob : th.blocks) {
    const int qap = ob.first[0], s1p = ob.first[1], s2p = ob.first[2];
    const int qbp = qap + s1p + s2p;
    const int qpi = li(qap);
    for (int u = 0; u < D; ++u) {
      const int qbi = ri(qbp - W2.qw[u]);
      if (qbi < 0 || !Rb[(size_t)u * nr + qbi] || rdim[qbi] == 0) continue;
      Slab sl{u, qpi, s1p, s2p, qbi, {}};
      for (const MTerm& m : mterms[((size_t)u * d + s1p) * d + s2p]) {
        const int qi = li(qap - W1.qw[m.w]);
        if (qi < 0 || !Lb[(size_t)m.w * nl + qi] || !Tb[tix(qi, m.s1, m.s2)]) continue;
        sl.terms.push_back(Term{t1x(m.w, qi, m.s1, m.s2), m.c});
      }
      if (sl.terms.empty()) continue;
      for (auto& t : sl.terms) t1_off[t.t1] = kUsed;
      live.push_back(std::move(sl));
    }
  }
  // step 1 tasks: one per live T1 slab
  int64_t off = 0;
  for (int w = 0; w < D; ++w)
    for (int qi = 0; qi < nl; ++qi)
      for (int s1 = 0; s1 < d; ++s1)
        for (int s2 = 0; s2 < d; ++s2) {
          const size_t x = t1x(w, qi, s1, s2);
          if (t1_off[x] == kUnused) continue;
          const int qa = qi + llo;
          const int M = ldim[li(qa + W1.qw[w])], N = rdim[ri(qa + s1 + s2)], K = ldim[qi];
          t1_off[x] = off;
          const BlockRef& lb = *Lb[(size_t)w * nl + qi];
          const BlockRef& tb = *Tb[tix(qi, s1, s2)];
          P.step1.add_task(off, M, N, N);
          P.step1.add_seg(lb.off, lb.cols, tb.off, tb.cols, K);
          if (packed) {
            P.step1p.add_task(off, M, N, N);
            P.step1p.add_seg(lp_off[(size_t)w * nl + qi], (int)pad8(K), xp_off[tix(qi, s1, s2)],
                             (int)pad8(K), K);
          }
          P.flops_step1 += 8LL * M * N * K;
          off += (int64_t)M * N;
        }
  P.t1_elems = off;
  // MPO combination: one T3 slab per live (u, output block)
  off = 0;
  auto t3x = [&](int u, int q, int s1, int s2) { return (size_t)u * nl * d * d + tix(q, s1, s2); };
  std::vector<int64_t> t3_off((size_t)D * nl * d * d, -1), t3p_off;
  if (packed) t3p_off.assign(t3_off.size(), -1);
  int64_t offp = 0;
  for (auto& sl : live) {
    const int M = ldim[sl.qi], N = rdim[sl.qbi];
    const size_t x = t3x(sl.u, sl.qi, sl.s1p, sl.s2p);
    t3_off[x] = off;
    P.mpo.add_task(off, M * N);
    for (auto& t : sl.terms) P.mpo.add_term(t1_off[t.t1], t.c);
    if (packed) {
      t3p_off[x] = offp;
      P.mpop.add_task(offp, M, N, (int)pad8(N));
      for (auto& t : sl.terms) P.mpop.add_term(t1_off[t.t1], t.c);
      offp += (int64_t)M * pad8(N);
    }
    P.flops_mpo += 4LL * (int64_t)sl.terms.size() * M * N;
    off += (int64_t)M * N;
  }
  P.t3_elems = off;
  P.t3p_elems = offp;
  // step 4 tasks: one per output block, K concatenated over live u
  for (auto& ob : out.blocks) {
    const int qap = ob.first[0], s1p = ob.first[1], s2p = ob.first[2];
    const int qbp = qap + s1p + s2p;
    const int qpi = li(qap);
    const int M = ob.second.rows, N = ob.second.cols;
    P.step4.add_task(ob.second.off, M, N, N);
    if (packed) P.step4p.add_task(ob.second.off, M, N, N);
    P.out_keys.push_back(ob.first);
    if (qpi < 0) continue;
    for (int u = 0; u < D; ++u) {
      const size_t x = t3x(u, qpi, s1p, s2p);
      if (t3_off[x] < 0) continue;
      const int qbi = ri(qbp - W2.qw[u]);
      const BlockRef& rb = *Rb[(size_t)u * nr + qbi];
      const int K = rdim[qbi];
      P.step4.add_seg(t3_off[x], K, rb.off, rb.cols, K);
      if (packed)
        P.step4p.add_seg(t3p_off[x], (int)pad8(K), rp_off[(size_t)u * nr + qbi], (int)pad8(K), K);
      P.flops_step4 += 8LL * M * N * K;
    }
  }
  P.mpo.finalize();
  if (packed) P.mpop.finalize();
  return P;
}

// ---------------------------------------------------------------------------
// HeffOp
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// batch plans
// ---------------------------------------------------------------------------
static void append_gemm(HostGemm& d, const HostGemm& s, int64_t dc, int64_t da, int64_t db) {
  const int seg_base = (int)d.segs.size();
  for (GemmTask t : s.tasks) {
    t.c_off += dc;
    t.seg0 += seg_base;
    d.tasks.push_back(t);
  }
  for (GemmSeg g : s.segs) {
    g.a_off += da;
    g.b_off += db;
    d.segs.push_back(g);
  }
  d.flops += s.flops;
}

static void append_comb(HostComb& d, const HostComb& s, int64_t dd, int64_t ds) {
  const int term_base = (int)d.terms.size();
  for (CombTask t : s.tasks) {
    t.dst_off += dd;
    t.term0 += term_base;
    d.tasks.push_back(t);
  }
  for (CombTerm t : s.terms) {
    t.src_off += ds;
    d.terms.push_back(t);
  }
  d.flops += s.flops;
}

static void append_combp(HostCombP& d, const HostCombP& s, int64_t dd, int64_t ds) {
  const int term_base = (int)d.terms.size();
  for (CombPTask t : s.tasks) {
    t.dst_off += dd;
    t.term0 += term_base;
    d.tasks.push_back(t);
  }
  for (CombTerm t : s.terms) {
    t.src_off += ds;
    d.terms.push_back(t);
  }
}

static void append_pack(HostPack& d, const HostPack& s, int64_t dsrc) {
  const int task_base = (int)d.tasks.size();
  const int64_t dst_base = d.elems;
  for (PackTask t : s.tasks) {
    t.src_off += dsrc;
    t.dst_off += dst_base;
    d.tasks.push_back(t);
  }
  for (int2 t : s.tiles) d.tiles.push_back(int2{t.x + task_base, t.y});
  d.elems += s.elems;
}

HeffPlan merge_heff_plans(const std::vector<const HeffPlan*>& plans,
                          const std::vector<BatchPart>& where) {
  HeffPlan M;
  if (plans.empty()) return M;
  M.packed = plans[0]->packed;
  // instance i's offsets inside the merged workspaces (prefix sums)
  const size_t n = plans.size();
  std::vector<int64_t> t1(n), t3(n), t3p(n), lp(n), xp(n), rp(n);
  for (size_t i = 0; i < n; ++i) {
    const HeffPlan& P = *plans[i];
    if (P.packed != M.packed) fail(TNT_E_STATE, "batch plans disagree in precision");
    t1[i] = M.t1_elems;
    t3[i] = M.t3_elems;
    t3p[i] = M.t3p_elems;
    lp[i] = M.Lp.elems;
    xp[i] = M.Xp.elems;
    rp[i] = M.Rp.elems;
    M.t1_elems += P.t1_elems;
    M.t3_elems += P.t3_elems;
    if (M.packed) {
      M.t3p_elems += P.t3p_elems;
      M.Lp.elems += P.Lp.elems;
      M.Xp.elems += P.Xp.elems;
      M.Rp.elems += P.Rp.elems;
    }
    M.flops_step1 += P.flops_step1;
    M.flops_mpo += P.flops_mpo;
    M.flops_step4 += P.flops_step4;
  }
  M.Lp.elems = M.Xp.elems = M.Rp.elems = 0;  // the appends below recount them
  // each merged table is appended on its own host thread
  std::vector<std::function<void()>> parts;
  parts.push_back([&] {
    for (size_t i = 0; i < n; ++i)
      append_gemm(M.step1, plans[i]->step1, t1[i], where[i].L_off, where[i].x_off);
  });
  parts.push_back([&] {
    for (size_t i = 0; i < n; ++i)
      append_gemm(M.step4, plans[i]->step4, where[i].x_off, t3[i], where[i].R_off);
  });
  parts.push_back([&] {
    for (size_t i = 0; i < n; ++i) append_comb(M.mpo, plans[i]->mpo, t3[i], t1[i]);
    M.mpo.finalize();
  });
  if (M.packed) {
    parts.push_back([&] {
      for (size_t i = 0; i < n; ++i)
        append_gemm(M.step1p, plans[i]->step1p, t1[i], lp[i], xp[i]);
    });
    parts.push_back([&] {
      for (size_t i = 0; i < n; ++i)
        append_gemm(M.step4p, plans[i]->step4p, where[i].x_off, t3p[i], rp[i]);
    });
    parts.push_back([&] {
      for (size_t i = 0; i < n; ++i) append_combp(M.mpop, plans[i]->mpop, t3p[i], t1[i]);
      M.mpop.finalize();
    });
    parts.push_back([&] {
      for (size_t i = 0; i < n; ++i) {
        append_pack(M.Lp, plans[i]->Lp, where[i].L_off);
        append_pack(M.Rp, plans[i]->Rp, where[i].R_off);
        append_pack(M.Xp, plans[i]->Xp, where[i].x_off);
      }
    });
  }
  std::vector<std::exception_ptr> err(parts.size());
  std::vector<std::thread> th;
  for (size_t k = 0; k < parts.size(); ++k)
    th.emplace_back([&, k]() {
      try {
        parts[k]();
      } catch (...) {
        err[k] = std::current_exception();
      }
    });
  for (auto& t : th) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  return M;
}

void HeffOp::build(Ctx& c, const EnvH& L, const MpoH& W1, const MpoH& W2, const EnvH& R,
                   const ThetaH& th, const ThetaH& out, int prec) {
  build_plan(c, build_heff_plan(L, W1, W2, R, th, out, prec != TNT_FP64), prec);
  L_ext = L.extent;
  R_ext = R.extent;
}

void HeffOp::build_plan(Ctx& c, HeffPlan&& p, int prec, bool tunable) {
  plan_tables(c, std::move(p), prec, tunable);
  upload_tables(nullptr);
}

size_t HeffOp::table_bytes() const {
  if (plan.packed)
    return DevTables::image_bytes({&plan.step1, &plan.step4, &plan.step1p, &plan.step4p},
                                  {&plan.mpo}, {&plan.mpop}, {&plan.Lp, &plan.Rp, &plan.Xp});
  return DevTables::image_bytes({&plan.step1, &plan.step4}, {&plan.mpo});
}

void HeffOp::upload_tables(void* dst) {
  Ctx& c = *ctx;
  if (plan.packed)
    tab.upload(c, {&plan.step1, &plan.step4, &plan.step1p, &plan.step4p}, {&plan.mpo},
               {&plan.mpop}, {&plan.Lp, &plan.Rp, &plan.Xp}, dst);
  else
    tab.upload(c, {&plan.step1, &plan.step4}, {&plan.mpo}, {}, {}, dst);
}

void HeffOp::ws_bytes(int prec, int64_t out[5]) const {
  for (int i = 0; i < 5; ++i) out[i] = 0;
  if (prec == TNT_FP64 || !plan.packed) {
    out[0] = std::max<int64_t>(1, 2 * plan.t1_elems) * sizeof(double);
    out[1] = std::max<int64_t>(1, 2 * plan.t3_elems) * sizeof(double);
    return;
  }
  const PackFmt f = fmt();
  const int64_t pb = (int64_t)pack_planes(f) * pack_elem_bytes(f);
  out[0] = std::max<int64_t>(1, 2 * plan.t1_elems) * sizeof(float);
  out[1] = std::max<int64_t>(16, plan.t3p_elems * pb);
  out[2] = std::max<int64_t>(16, plan.Lp.elems * pb);
  out[3] = std::max<int64_t>(16, plan.Rp.elems * pb);
  out[4] = std::max<int64_t>(16, plan.Xp.elems * pb);
}

void HeffOp::plan_tables(Ctx& c, HeffPlan&& p, int prec, bool tunable) {
  ctx = &c;
  precision = prec;
  const bool packed = prec != TNT_FP64;
  plan = std::move(p);
  if (plan.packed != packed) fail(TNT_E_STATE, "plan built for another precision");
  // tile shape: a cached tuning decision for this shape bucket, else the
  // default, plus every candidate for the first application to time when
  // `tunable` (the operator's own precision)
  struct Job {
    HostGemm* h;
    int which;
    GemmPath path;
    bool tunable, tune;
  };
  // FP64 tables: the FP64 operator, or the FP64 refinement of a
  // reduced-precision one
  std::vector<Job> jobs = {{&plan.step1, 1, PATH_F64, tunable && !packed, false},
                           {&plan.step4, 4, PATH_F64, tunable && !packed, false}};
  if (packed) {
    jobs.push_back({&plan.step1p, 1, gemm_path(prec), tunable, false});
    jobs.push_back({&plan.step4p, 4, gemm_path(prec), tunable, false});
  }
  // the tuning cache is only read here
  auto setup = [&](Job& j) {
    auto it = c.tune_cache.find(tune_bucket(*j.h, j.path, j.which));
    j.h->finalize(it != c.tune_cache.end() ? it->second : default_tile_cfg(*j.h, j.path));
    if (j.tunable && it == c.tune_cache.end() && c.autotune && j.h->flops >= kTuneMinFlops) {
      for (int cfg : tile_candidates(j.path)) j.h->add_variant(cfg);
      j.tune = true;
    }
  };
  // tile tables of large plans (merged batch operators) on one host thread
  // per table: independent sorts over tens of thousands of tasks
  size_t ntask = 0;
  for (const Job& j : jobs) ntask += j.h->tasks.size();
  if (ntask >= 4096) {
    std::vector<std::exception_ptr> err(jobs.size());
    std::vector<std::thread> th;
    for (size_t k = 0; k < jobs.size(); ++k)
      th.emplace_back([&, k]() {
        try {
          setup(jobs[k]);
        } catch (...) {
          err[k] = std::current_exception();
        }
      });
    for (auto& t : th) t.join();
    for (auto& e : err)
      if (e) std::rethrow_exception(e);
  } else {
    for (Job& j : jobs) setup(j);
  }
  bool tune = false;
  for (const Job& j : jobs) tune = tune || j.tune;
  tuned = !tune;
}

void* HeffOp::wsp(int i) const { return ext_ws[i] ? ext_ws[i] : ctx->ws[i].ptr; }

void HeffOp::ensure_ws(int i, int64_t bytes) {
  if (ext_ws[i]) return;  // sized by the caller (ws_bytes)
  ctx->ws[i].ensure(&ctx->pool, bytes);
}

void HeffOp::bind_envs(const void* lre, const void* lim, const void* rre, const void* rim) {
  Ctx& c = *ctx;
  L_re = static_cast<const double*>(lre); L_im = static_cast<const double*>(lim);
  R_re = static_cast<const double*>(rre); R_im = static_cast<const double*>(rim);
  if (!plan.packed) return;
  const PackFmt f = fmt();
  const int64_t pb = (int64_t)pack_planes(f) * pack_elem_bytes(f);
  ensure_ws(2, std::max<int64_t>(16, plan.Lp.elems * pb));
  ensure_ws(3, std::max<int64_t>(16, plan.Rp.elems * pb));
  const DevTables::P& lp = tab.p[0];
  const DevTables::P& rp = tab.p[1];
  launch_pack(lp.tasks, lp.tiles, lp.ntiles, L_re, L_im, wsp(2), lp.elems, f, c.stream);
  launch_pack(rp.tasks, rp.tiles, rp.ntiles, R_re, R_im, wsp(3), rp.elems, f, c.stream);
}

void HeffOp::launch_step(int step, int v, bool fp64, const double* xre, const double* xim,
                         double* yre, double* yim) {
  Ctx& c = *ctx;
  if (fp64) {
    double* a = static_cast<double*>(wsp(0));
    double* b = static_cast<double*>(wsp(1));
    if (step == 1)
      run_gemm_variant(c, tab.g[0], v, FORM_NN, PATH_F64, L_re, L_im, ET_F64, xre, xim, ET_F64,
                       a, a + plan.t1_elems, ET_F64);
    else
      run_gemm_variant(c, tab.g[1], v, FORM_NT, PATH_F64, b, b + plan.t3_elems, ET_F64, R_re,
                       R_im, ET_F64, yre, yim, ET_F64);
    return;
  }
  // packed path: step 1 Lp . Xp^T -> FP32 T1 slabs; step 4 T3p . Rp^T -> y
  const DevTables::G& g = tab.g[step == 1 ? 2 : 3];
  if (v < 0 || v >= g.nvar) fail(TNT_E_STATE, "tile-table variant out of range");
  float* t1 = static_cast<float*>(wsp(0));
  PackedLaunch L{};
  L.tasks = g.tasks;
  L.segs = g.segs;
  L.tiles = g.tiles[v];
  L.ntiles = g.ntiles[v];
  L.tile_cfg = g.cfg[v];
  L.fmt = fmt();
  if (step == 1) {
    L.a = wsp(2); L.a_plane = plan.Lp.elems;
    L.b = wsp(4); L.b_plane = plan.Xp.elems;
    L.c_re = t1; L.c_im = t1 + plan.t1_elems; L.c_t = ET_F32;
  } else {
    L.a = wsp(1); L.a_plane = plan.t3p_elems;
    L.b = wsp(3); L.b_plane = plan.Rp.elems;
    L.c_re = yre; L.c_im = yim; L.c_t = ET_F64;
  }
  if (!launch_packed_gemm(L, c.stream))
    fail(TNT_E_STATE, "packed GEMM variant not available (tile shape " + std::to_string(g.cfg[v]) +
                          ")");
}

HeffOp::~HeffOp() {
  if (graph.exec) (void)hipGraphExecDestroy(graph.exec);
}

void HeffOp::prepare(const double* xre, const double* xim, double* yre, double* yim, int prec) {
  Ctx& c = *ctx;
  if (prec == TNT_FP64 || !plan.packed) {
    ensure_ws(0, std::max<int64_t>(1, 2 * plan.t1_elems) * sizeof(double));
    ensure_ws(1, std::max<int64_t>(1, 2 * plan.t3_elems) * sizeof(double));
    if (!tuned && !plan.packed) autotune(xre, xim, yre, yim, prec);
    return;
  }
  const PackFmt f = fmt();
  const int64_t pb = (int64_t)pack_planes(f) * pack_elem_bytes(f);
  ensure_ws(0, std::max<int64_t>(1, 2 * plan.t1_elems) * sizeof(float));
  ensure_ws(1, std::max<int64_t>(16, plan.t3p_elems * pb));
  ensure_ws(4, std::max<int64_t>(16, plan.Xp.elems * pb));
  if (!tuned) {
    const DevTables::P& xp = tab.p[2];
    launch_pack(xp.tasks, xp.tiles, xp.ntiles, xre, xim, wsp(4), xp.elems, f, c.stream);
    autotune(xre, xim, yre, yim, prec);
  }
}

void HeffOp::apply(const double* xre, const double* xim, double* yre, double* yim, int prec,
                   const hipEvent_t* tev) {
  Ctx& c = *ctx;
  auto mark = [&](int i) {
    if (tev) TNT_HIP(hipEventRecord(tev[i - 2], c.stream));
  };
  // FP64: the FP64 operator, or the refinement matvec of a reduced-precision
  // operator (on the FP64 environments)
  if (prec == TNT_FP64 || !plan.packed) {
    ensure_ws(0, std::max<int64_t>(1, 2 * plan.t1_elems) * sizeof(double));
    ensure_ws(1, std::max<int64_t>(1, 2 * plan.t3_elems) * sizeof(double));
    if (!tuned && !plan.packed) autotune(xre, xim, yre, yim, prec);
    const int v1 = valid_variant(tab.g[0], PATH_F64), v4 = valid_variant(tab.g[1], PATH_F64);
    mark(2);
    launch_step(1, v1, true, xre, xim, yre, yim);
    mark(3);
    run_comb(c, tab.c[0], static_cast<double*>(wsp(0)), static_cast<double*>(wsp(0)) + plan.t1_elems,
             static_cast<double*>(wsp(1)), static_cast<double*>(wsp(1)) + plan.t3_elems, ET_F64);
    mark(4);
    launch_step(4, v4, true, xre, xim, yre, yim);
    mark(5);
    return;
  }
  const PackFmt f = fmt();
  const int64_t pb = (int64_t)pack_planes(f) * pack_elem_bytes(f);
  ensure_ws(0, std::max<int64_t>(1, 2 * plan.t1_elems) * sizeof(float));
  ensure_ws(1, std::max<int64_t>(16, plan.t3p_elems * pb));
  ensure_ws(4, std::max<int64_t>(16, plan.Xp.elems * pb));
  const DevTables::P& xp = tab.p[2];
  launch_pack(xp.tasks, xp.tiles, xp.ntiles, xre, xim, wsp(4), xp.elems, f, c.stream);
  if (!tuned) autotune(xre, xim, yre, yim, prec);
  const DevTables::CP& cp = tab.cp[0];
  mark(2);
  launch_step(1, tab.g[2].sel, false, xre, xim, yre, yim);
  mark(3);
  launch_combine_packed(cp.tasks, cp.terms, cp.chunks, cp.nchunks, static_cast<float*>(wsp(0)),
                        static_cast<float*>(wsp(0)) + plan.t1_elems, wsp(1), plan.t3p_elems, f,
                        c.stream);
  mark(4);
  launch_step(4, tab.g[3].sel, false, xre, xim, yre, yim);
  mark(5);
}

void HeffOp::autotune(const double* xre, const double* xim, double* yre, double* yim, int prec) {
  Ctx& c = *ctx;
  tuned = true;
  const bool fp64 = !plan.packed;
  const GemmPath path = gemm_path(precision);
  (void)prec;
  // candidates run on the operator's real operands; step 4 reads whatever
  // the slab workspace holds (in bounds; values do not affect timing) and
  // the caller's apply overwrites every output afterwards
  for (int step : {1, 4}) {
    const int gi = (fp64 ? 0 : 2) + (step == 1 ? 0 : 1);
    DevTables::G& g = tab.g[gi];
    if (g.nvar <= 1) continue;
    // one warm-up launch per candidate, then three interleaved rounds of one
    // timed launch each; a candidate's time is its fastest round, so a
    // single disturbed launch cannot decide
    std::vector<float> t(g.nvar, 1e30f);
    for (int v = 0; v < g.nvar; ++v)
      if (gemm_cfg_valid(g.cfg[v], path)) launch_step(step, v, fp64, xre, xim, yre, yim);
    for (int round = 0; round < 3; ++round)
      for (int v = 0; v < g.nvar; ++v) {
        if (!gemm_cfg_valid(g.cfg[v], path)) continue;
        TNT_HIP(hipEventRecord(c.ev[6], c.stream));
        launch_step(step, v, fp64, xre, xim, yre, yim);
        TNT_HIP(hipEventRecord(c.ev[7], c.stream));
        TNT_HIP(hipEventSynchronize(c.ev[7]));
        float ms = 0;
        TNT_HIP(hipEventElapsedTime(&ms, c.ev[6], c.ev[7]));
        t[v] = std::min(t[v], ms);
      }
    int best = g.sel;
    for (int v = 0; v < g.nvar; ++v)
      if (t[v] < t[best] || !gemm_cfg_valid(g.cfg[best], path)) best = v;
    g.sel = best;
    const HostGemm& h = fp64 ? (step == 1 ? plan.step1 : plan.step4)
                             : (step == 1 ? plan.step1p : plan.step4p);
    c.tune_cache[tune_bucket(h, path, step)] = g.cfg[best];
  }
}

}  // namespace tnt
