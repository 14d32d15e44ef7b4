// C-ABI: context and the two-site H_eff application.
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <thread>
#include <unordered_map>

#include "capi_util.h"
#include "plan.h"

namespace tnt {

struct PlanCache {
  // batch operators by the identities of their instance operators (which
  // they keep alive)
  struct Batch {
    std::vector<std::shared_ptr<HeffOp>> ops;
    std::shared_ptr<BatchHeff> b;
  };
  std::unordered_map<uint64_t, Batch> batch;
  // batched C-ABI calls by the hash of all their raw descriptors
  std::unordered_map<uint64_t, std::shared_ptr<BatchCall>> raw_batch;
  // operators by the hash of their parsed block structures
  std::unordered_map<uint64_t, std::shared_ptr<HeffOp>> heff;
  // the same operators by the hash of the raw host descriptors they were
  // parsed and validated from (skips the parse for a repeated call)
  std::unordered_map<uint64_t, std::shared_ptr<HeffOp>> raw;
  // host plans alone (the lockstep sweep merges them into batch operators)
  // by the operators' key, and those batch operators by plan identities
  std::unordered_map<uint64_t, std::shared_ptr<HeffPlan>> plan;
  struct PlanBatch {
    std::vector<std::shared_ptr<HeffPlan>> plans;
    std::shared_ptr<BatchHeff> b;
  };
  std::unordered_map<uint64_t, PlanBatch> plan_batch;
};

// Word-wise hash of the raw host metadata of an H_eff call: every field the
// parse reads (labels, extents, offsets, capacities, dtypes, MPO arrays).
static void raw_add(uint64_t& h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  auto mix = [&](uint64_t w) {
    h ^= w + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    h *= 0xff51afd7ed558ccdULL;
  };
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    memcpy(&w, b + i, 8);
    mix(w);
  }
  uint64_t w = 0;
  if (i < n) memcpy(&w, b + i, n - i);
  mix(w ^ (uint64_t)n);
}
static void raw_btensor(uint64_t& h, const tnt_btensor* t) {
  if (!t || t->nblocks < 0 || t->rank < 0 || (t->nblocks > 0 && (!t->qn || !t->extent || !t->offset)))
    fail(TNT_E_ARG, "invalid block-tensor descriptor");
  const int32_t hdr[3] = {t->rank, t->nblocks, t->dtype};
  raw_add(h, hdr, sizeof(hdr));
  raw_add(h, &t->capacity, sizeof(t->capacity));
  raw_add(h, t->qn, sizeof(int32_t) * (size_t)t->nblocks * t->rank);
  raw_add(h, t->extent, sizeof(int32_t) * (size_t)t->nblocks * t->rank);
  raw_add(h, t->offset, sizeof(int64_t) * (size_t)t->nblocks);
}
static void raw_mpo(uint64_t& h, const tnt_mpo_site* m) {
  if (!m || !m->bond_charge || !m->W || m->d <= 0 || m->D <= 0 || m->d > 64 || m->D > 64)
    fail(TNT_E_ARG, "invalid MPO descriptor");
  const int32_t hdr[2] = {m->d, m->D};
  raw_add(h, hdr, sizeof(hdr));
  raw_add(h, m->bond_charge, sizeof(int32_t) * m->D);
  raw_add(h, m->W, sizeof(double) * (size_t)m->D * m->D * m->d * m->d);
}

void destroy_blas(void* h);                  // svd.cpp
int64_t blas_workspace_bytes(const Ctx& c);  // svd.cpp

Ctx::~Ctx() {
  if (stream) (void)hipStreamSynchronize(stream);
  else (void)hipDeviceSynchronize();
  delete plans;
  plans = nullptr;
  if (blas) destroy_blas(blas);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : step_ev)
    if (e) (void)hipEventDestroy(e);
  if (gstream) (void)hipStreamDestroy(gstream);
  for (int i = 0; i < kSide; ++i) {
    if (side[i]) (void)hipStreamSynchronize(side[i]);
    if (side_blas[i]) destroy_blas(side_blas[i]);
    if (side[i]) (void)hipStreamDestroy(side[i]);
  }
  for (auto& e : side_ev)
    if (e) (void)hipEventDestroy(e);
}

void Hasher::add(const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ULL;
  }
}

void hash_theta(Hasher& H, const ThetaH& t) {
  for (auto& kv : t.blocks) {
    H.add(kv.first.data(), sizeof(int) * 3);
    H.add(&kv.second, sizeof(BlockRef));
  }
  H.add<int64_t>(-1);
}

void hash_env(Hasher& H, const EnvH& e) {
  for (auto& kv : e.blocks) {
    H.add(&kv.first, sizeof(kv.first));
    H.add(&kv.second, sizeof(BlockRef));
  }
  H.add<int64_t>(-2);
}

void hash_mpo(Hasher& H, const MpoH& m) {
  H.add(m.W.data(), m.W.size() * sizeof(double));
  H.add(m.qw.data(), m.qw.size() * sizeof(int));
}

void check_precision(int32_t p) {
  if (p != TNT_FP64 && p != TNT_FP32 && p != TNT_BF16X3) fail(TNT_E_ARG, "unknown precision");
  if (p == TNT_BF16X3 && !bf16x3_available()) fail(TNT_E_ARG, "BF16X3 path not built");
}

// Parse and cross-check the operands of an H_eff application.
HeffArgs parse_heff_args(const tnt_btensor* L, const tnt_mpo_site* W1, const tnt_mpo_site* W2,
                         const tnt_btensor* R, const tnt_btensor* theta, const tnt_btensor* out) {
  HeffArgs a;
  a.w1 = parse_mpo(W1, "W1");
  a.w2 = parse_mpo(W2, "W2");
  if (a.w1.d != a.w2.d || a.w1.D != a.w2.D || a.w1.qw != a.w2.qw)
    fail(TNT_E_SHAPE, "W1 and W2 disagree in d, D or bond charges");
  a.th = parse_theta(theta, a.w1.d, "theta");
  a.out = out ? parse_theta(out, a.w1.d, "out") : a.th;
  if (out) check_same_structure(a.th, a.out);
  a.L = parse_env(L, a.w1, "L");
  a.R = parse_env(R, a.w2, "R");
  check_bond_match(a.L.bond, a.th.left, "L vs theta left bond");
  check_bond_match(a.R.bond, a.th.right, "R vs theta right bond");
  return a;
}

uint64_t raw_hash_batch(int n, const tnt_btensor* const* L, const tnt_mpo_site* const* W1,
                        const tnt_mpo_site* const* W2, const tnt_btensor* const* R,
                        const tnt_btensor* const* theta, const tnt_btensor* const* out,
                        int prec, uint64_t salt) {
  uint64_t rh = salt ^ ((uint64_t)(uint32_t)prec << 32) ^ (uint64_t)(uint32_t)n;
  for (int i = 0; i < n; ++i) {
    if (!L[i] || !R[i] || !theta[i] || (out && !out[i])) fail(TNT_E_ARG, "null instance operand");
    raw_btensor(rh, L[i]);
    raw_btensor(rh, R[i]);
    raw_btensor(rh, theta[i]);
    if (out) raw_btensor(rh, out[i]);
    raw_mpo(rh, W1[i]);
    raw_mpo(rh, W2[i]);
  }
  return rh;
}

std::shared_ptr<BatchCall> find_batch_call(Ctx& c, uint64_t key) {
  if (!c.plans) c.plans = new PlanCache();
  auto it = c.plans->raw_batch.find(key);
  return it == c.plans->raw_batch.end() ? nullptr : it->second;
}

void store_batch_call(Ctx& c, uint64_t key, std::shared_ptr<BatchCall> bc) {
  if (!c.plans) c.plans = new PlanCache();
  if (c.plans->raw_batch.size() >= 64) {
    TNT_HIP(hipStreamSynchronize(c.stream));
    c.plans->raw_batch.clear();
  }
  c.plans->raw_batch[key] = std::move(bc);
}

std::shared_ptr<BatchHeff> cached_batch(Ctx& c, const std::vector<std::shared_ptr<HeffOp>>& ops,
                                        const std::vector<int64_t>& n, int prec) {
  Hasher H;
  H.add(prec);
  for (size_t i = 0; i < ops.size(); ++i) {
    H.add(ops[i].get());
    H.add(n[i]);
  }
  if (!c.plans) c.plans = new PlanCache();
  auto it = c.plans->batch.find(H.h);
  if (it != c.plans->batch.end() && it->second.ops == ops) return it->second.b;
  if (c.plans->batch.size() >= 256) {
    TNT_HIP(hipStreamSynchronize(c.stream));
    c.plans->batch.clear();
    c.plans->raw_batch.clear();
  }
  auto b = std::make_shared<BatchHeff>();
  build_batch(c, *b, ops, n, prec);
  c.plans->batch[H.h] = PlanCache::Batch{ops, b};
  return b;
}

void copy_runs(Ctx& c, const std::vector<CopyRun>& runs) {
  if (runs.empty()) return;
  int64_t mx = 0;
  for (const CopyRun& r : runs) mx = std::max(mx, r.count);
  DevBuf t(&c.pool, runs.size() * sizeof(CopyRun));
  TNT_HIP(hipMemcpyAsync(t.ptr, runs.data(), runs.size() * sizeof(CopyRun),
                         hipMemcpyHostToDevice, c.stream));
  launch_copy_runs(t.as<CopyRun>(), (int)runs.size(), mx, c.stream);
  // the host run list must outlive the transfer
  TNT_HIP(hipStreamSynchronize(c.stream));
}

// Host plans of args[miss[q]]: independent host work, built on up to
// kPlanThreads threads (the planner has no shared state).
static std::vector<HeffPlan> build_plans(const std::vector<const HeffArgs*>& args,
                                         const std::vector<size_t>& miss, int prec) {
  const bool packed = prec != TNT_FP64;
  std::vector<HeffPlan> plans(miss.size());
  auto plan_one = [&](size_t q) {
    const HeffArgs& a = *args[miss[q]];
    plans[q] = build_heff_plan(a.L, a.w1, a.w2, a.R, a.th, a.out, packed);
  };
  const size_t nth = std::min<size_t>(miss.size(), kPlanThreads);
  if (nth <= 1) {
    for (size_t q = 0; q < miss.size(); ++q) plan_one(q);
    return plans;
  }
  std::vector<std::exception_ptr> err(nth);
  std::vector<std::thread> th;
  for (size_t w = 0; w < nth; ++w)
    th.emplace_back([&, w]() {
      try {
        for (size_t q = w; q < miss.size(); q += nth) plan_one(q);
      } catch (...) {
        err[w] = std::current_exception();
      }
    });
  for (auto& t : th) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  return plans;
}

static uint64_t heff_key(const HeffArgs& a, int prec) {
  Hasher H;
  H.add(prec);
  hash_mpo(H, a.w1);
  hash_mpo(H, a.w2);
  hash_env(H, a.L);
  hash_env(H, a.R);
  hash_theta(H, a.th);
  hash_theta(H, a.out);
  return H.h;
}

std::shared_ptr<HeffOp> cached_heff(Ctx& c, const HeffArgs& a, int prec) {
  return cached_heffs(c, {&a}, prec)[0];
}

std::vector<std::shared_ptr<HeffOp>> cached_heffs(Ctx& c, const std::vector<const HeffArgs*>& args,
                                                  int prec) {
  if (!c.plans) c.plans = new PlanCache();
  const size_t n = args.size();
  std::vector<uint64_t> key(n);
  std::vector<std::shared_ptr<HeffOp>> out(n);
  std::vector<size_t> miss;
  for (size_t i = 0; i < n; ++i) {
    key[i] = heff_key(*args[i], prec);
    auto it = c.plans->heff.find(key[i]);
    if (it != c.plans->heff.end()) out[i] = it->second;
    else miss.push_back(i);
  }
  if (miss.empty()) return out;
  if (c.plans->heff.size() + miss.size() > 1024) {
    TNT_HIP(hipStreamSynchronize(c.stream));
    c.plans->heff.clear();
    c.plans->raw.clear();
  }
  std::vector<HeffPlan> plans = build_plans(args, miss, prec);
  for (size_t q = 0; q < miss.size(); ++q) {
    const size_t i = miss[q];
    auto it = c.plans->heff.find(key[i]);  // an earlier miss of this call with the same key
    if (it != c.plans->heff.end()) {
      out[i] = it->second;
      continue;
    }
    auto op = std::make_shared<HeffOp>();
    op->build_plan(c, std::move(plans[q]), prec);
    op->L_ext = args[i]->L.extent;
    op->R_ext = args[i]->R.extent;
    c.plans->heff[key[i]] = op;
    out[i] = op;
  }
  return out;
}

std::vector<std::shared_ptr<HeffPlan>> cached_plans(Ctx& c,
                                                   const std::vector<const HeffArgs*>& args,
                                                   int prec) {
  if (!c.plans) c.plans = new PlanCache();
  const size_t n = args.size();
  std::vector<uint64_t> key(n);
  std::vector<std::shared_ptr<HeffPlan>> out(n);
  std::vector<size_t> miss;
  for (size_t i = 0; i < n; ++i) {
    key[i] = heff_key(*args[i], prec);
    auto it = c.plans->plan.find(key[i]);
    if (it != c.plans->plan.end()) out[i] = it->second;
    else miss.push_back(i);
  }
  if (miss.empty()) return out;
  if (c.plans->plan.size() + miss.size() > 4096) {
    TNT_HIP(hipStreamSynchronize(c.stream));
    c.plans->plan.clear();
    c.plans->plan_batch.clear();
  }
  std::vector<HeffPlan> plans = build_plans(args, miss, prec);
  for (size_t q = 0; q < miss.size(); ++q) {
    const size_t i = miss[q];
    auto it = c.plans->plan.find(key[i]);
    if (it != c.plans->plan.end()) {
      out[i] = it->second;
      continue;
    }
    auto p = std::make_shared<HeffPlan>(std::move(plans[q]));
    c.plans->plan[key[i]] = p;
    out[i] = p;
  }
  return out;
}

std::shared_ptr<BatchHeff> cached_plan_batch(Ctx& c,
                                             const std::vector<std::shared_ptr<HeffPlan>>& plans,
                                             const std::vector<int64_t>& L_ext,
                                             const std::vector<int64_t>& R_ext,
                                             const std::vector<int64_t>& n, int prec) {
  Hasher H;
  H.add(prec);
  for (size_t i = 0; i < plans.size(); ++i) {
    H.add(plans[i].get());
    H.add(n[i]);
    H.add(L_ext[i]);
    H.add(R_ext[i]);
  }
  if (!c.plans) c.plans = new PlanCache();
  auto it = c.plans->plan_batch.find(H.h);
  if (it != c.plans->plan_batch.end() && it->second.plans == plans) return it->second.b;
  if (c.plans->plan_batch.size() >= 256) {
    TNT_HIP(hipStreamSynchronize(c.stream));
    c.plans->plan_batch.clear();
  }
  auto b = std::make_shared<BatchHeff>();
  std::vector<const HeffPlan*> pp;
  for (const auto& p : plans) pp.push_back(p.get());
  // a lockstep sweep builds a new batch operator at nearly every step: the
  // tile shapes come from cached decisions or the defaults, not timing
  build_batch_plans(c, *b, pp, L_ext, R_ext, n, prec, false);
  c.plans->plan_batch[H.h] = PlanCache::PlanBatch{plans, b};
  return b;
}

}  // namespace tnt

using namespace tnt;

extern "C" {

tnt_status tnt_ctx_create(int32_t device, void* hip_stream, tnt_ctx* out) {
  if (!out) return TNT_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TNT_E_HIP;
  if (hipSetDevice(device) != hipSuccess) return TNT_E_HIP;
  Ctx* c = new (std::nothrow) Ctx();
  if (!c) return TNT_E_ALLOC;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess)
    c->num_cu = cu;
  for (auto& e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete c;
      return TNT_E_HIP;
    }
  try {
    c->scratch = scratch_address(device);
  } catch (const Error& e) {
    delete c;
    return e.code;
  }
  *out = reinterpret_cast<tnt_ctx>(c);
  return TNT_OK;
}

void tnt_ctx_destroy(tnt_ctx ctx) { delete reinterpret_cast<Ctx*>(ctx); }

const char* tnt_last_error(tnt_ctx ctx) {
  if (!ctx) return "null context";
  return reinterpret_cast<Ctx*>(ctx)->last_error.c_str();
}

tnt_status tnt_sync(tnt_ctx ctx) {
  TNT_API_BEGIN(ctx)
  TNT_HIP(hipStreamSynchronize(c.stream));
  TNT_API_END
}

int64_t tnt_pool_bytes(tnt_ctx ctx) {
  return ctx ? reinterpret_cast<Ctx*>(ctx)->pool.held() : -1;
}

tnt_status tnt_ctx_memory(tnt_ctx ctx, int64_t* out) {
  TNT_API_BEGIN(ctx)
  if (!out) fail(TNT_E_ARG, "tnt_ctx_memory: null out");
  out[0] = c.pool.held();
  out[1] = c.pool.in_use();
  out[2] = c.pool.peak_in_use();
  out[3] = blas_workspace_bytes(c);
  TNT_API_END
}

tnt_status tnt_ctx_set_autotune(tnt_ctx ctx, int32_t on) {
  TNT_API_BEGIN(ctx)
  c.autotune = on ? 1 : 0;
  if (!on) c.tune_cache.clear();
  // cached plans keep the tile tables they were built with
  if (c.plans) {
    TNT_HIP(hipStreamSynchronize(c.stream));
    c.plans->heff.clear();
    c.plans->raw.clear();
    c.plans->batch.clear();
    c.plans->raw_batch.clear();
  }
  TNT_API_END
}

tnt_status tnt_heff2_apply_batched(tnt_ctx ctx, int32_t n, const tnt_btensor* const* L,
                                   const tnt_mpo_site* const* W1, const tnt_mpo_site* const* W2,
                                   const tnt_btensor* const* R, const tnt_btensor* const* theta,
                                   tnt_btensor* const* out, int32_t precision) {
  TNT_API_BEGIN(ctx)
  check_precision(precision);
  if (n < 1 || !L || !W1 || !W2 || !R || !theta || !out) fail(TNT_E_ARG, "null or empty batch");
  const uint64_t rh = raw_hash_batch(n, L, W1, W2, R, theta, out, precision, 0x13198a2e03707344ULL);
  std::shared_ptr<BatchCall> bc = find_batch_call(c, rh);
  if (bc) {
    // the same descriptors were parsed and validated before
    for (int i = 0; i < n; ++i)
      for (const tnt_btensor* t : {L[i], R[i], theta[i], (const tnt_btensor*)out[i]})
        if (!t->re || !t->im) fail(TNT_E_ARG, "null plane");
  } else {
    bc = std::make_shared<BatchCall>();
    std::vector<int64_t> nn;
    for (int i = 0; i < n; ++i) {
      HeffArgs a = parse_heff_args(L[i], W1[i], W2[i], R[i], theta[i], out[i]);
      if (L[i]->dtype != TNT_DT_F64 || R[i]->dtype != TNT_DT_F64 ||
          theta[i]->dtype != TNT_DT_F64 || out[i]->dtype != TNT_DT_F64)
        fail(TNT_E_ARG, "L, R, theta and out must be FP64 planes");
      bc->tlay.push_back(a.th);
      bc->olay.push_back(a.out);
      // the batch vector holds every instance in its canonical packed layout
      int64_t off = 0;
      for (auto& kv : a.th.blocks) {
        kv.second.off = off;
        off += (int64_t)kv.second.rows * kv.second.cols;
      }
      a.th.elems = a.th.extent = off;
      a.out = a.th;
      nn.push_back(off);
      bc->ops.push_back(cached_heff(c, a, precision));
    }
    bc->b = cached_batch(c, bc->ops, nn, precision);
    store_batch_call(c, rh, bc);
  }
  BatchHeff& B = *bc->b;
  std::vector<const double *> Lr, Li, Rr, Ri;
  for (int i = 0; i < n; ++i) {
    Lr.push_back(static_cast<const double*>(L[i]->re));
    Li.push_back(static_cast<const double*>(L[i]->im));
    Rr.push_back(static_cast<const double*>(R[i]->re));
    Ri.push_back(static_cast<const double*>(R[i]->im));
  }
  bind_batch_envs(c, B, Lr, Li, Rr, Ri);
  bc->xy.ensure(&c.pool, std::max<int64_t>(1, 4 * B.N) * sizeof(double));
  double* x = bc->xy.as<double>();
  double* y = x + 2 * B.N;
  std::vector<CopyRun> in, back;
  for (int i = 0; i < n; ++i) {
    const int64_t base = B.parts[i].x_off;
    int64_t off = 0;
    for (auto& kv : bc->tlay[i].blocks) {
      const BlockRef& src = kv.second;
      const BlockRef& dst = bc->olay[i].blocks.at(kv.first);
      const int64_t cnt = (int64_t)src.rows * src.cols;
      in.push_back(CopyRun{static_cast<const double*>(theta[i]->re) + src.off, x + base + off, cnt});
      in.push_back(
          CopyRun{static_cast<const double*>(theta[i]->im) + src.off, x + B.N + base + off, cnt});
      back.push_back(CopyRun{y + base + off, static_cast<double*>(out[i]->re) + dst.off, cnt});
      back.push_back(CopyRun{y + B.N + base + off, static_cast<double*>(out[i]->im) + dst.off, cnt});
      off += cnt;
    }
  }
  bc->in.run(c, in);
  B.op->apply(x, x + B.N, y, y + B.N, precision);
  bc->back.run(c, back);
  TNT_HIP(hipGetLastError());
  TNT_API_END
}

tnt_status tnt_ctx_set_graphs(tnt_ctx ctx, int32_t on) {
  TNT_API_BEGIN(ctx)
  c.graphs = on ? 1 : 0;
  TNT_API_END
}

tnt_status tnt_ctx_set_eig_reduction(tnt_ctx ctx, int32_t min_order) {
  TNT_API_BEGIN(ctx)
  c.eig_trd_min = min_order < 0 ? Ctx::kEigTrdDefault : min_order;
  TNT_API_END
}

tnt_status tnt_heff2_apply(tnt_ctx ctx, const tnt_btensor* L, const tnt_mpo_site* W1,
                           const tnt_mpo_site* W2, const tnt_btensor* R,
                           const tnt_btensor* theta, tnt_btensor* out, int32_t precision) {
  TNT_API_BEGIN(ctx)
  check_precision(precision);
  if (!out) fail(TNT_E_ARG, "null out");
  uint64_t rh = 0x243f6a8885a308d3ULL ^ (uint64_t)precision;
  raw_btensor(rh, L);
  raw_btensor(rh, R);
  raw_btensor(rh, theta);
  raw_btensor(rh, out);
  raw_mpo(rh, W1);
  raw_mpo(rh, W2);
  if (!c.plans) c.plans = new PlanCache();
  std::shared_ptr<HeffOp> op;
  auto hit = c.plans->raw.find(rh);
  if (hit != c.plans->raw.end()) {
    op = hit->second;  // the same descriptors were parsed and validated before
    for (const tnt_btensor* t : {L, R, theta, (const tnt_btensor*)out})
      if (!t->re || !t->im) fail(TNT_E_ARG, "null plane");
  } else {
    HeffArgs a = parse_heff_args(L, W1, W2, R, theta, out);
    if (L->dtype != TNT_DT_F64 || R->dtype != TNT_DT_F64 || theta->dtype != TNT_DT_F64 ||
        out->dtype != TNT_DT_F64)
      fail(TNT_E_ARG, "L, R, theta and out must be FP64 planes");
    op = cached_heff(c, a, precision);
    if (c.plans->raw.size() >= 1024) c.plans->raw.clear();
    c.plans->raw[rh] = op;
  }
  op->bind_envs(L->re, L->im, R->re, R->im);
  op->apply(static_cast<const double*>(theta->re), static_cast<const double*>(theta->im),
            static_cast<double*>(out->re), static_cast<double*>(out->im), precision);
  TNT_HIP(hipGetLastError());
  TNT_API_END
}

int64_t tnt_heff2_flops(const tnt_btensor* L, const tnt_mpo_site* W1, const tnt_mpo_site* W2,
                        const tnt_btensor* R, const tnt_btensor* theta, int64_t* parts) {
  try {
    HeffArgs a = parse_heff_args(L, W1, W2, R, theta, nullptr);
    HeffPlan p = build_heff_plan(a.L, a.w1, a.w2, a.R, a.th, a.th, false);
    if (parts) {
      parts[0] = p.flops_step1;
      parts[1] = p.flops_mpo;
      parts[2] = p.flops_step4;
    }
    return p.flops();
  } catch (...) {
    return -1;
  }
}

}  // extern "C"
