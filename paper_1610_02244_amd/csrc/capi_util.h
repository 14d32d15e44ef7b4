// Helpers shared by the C-ABI translation units.
#pragma once

#include <memory>
#include <new>
#include <vector>

#include "batch.h"
#include "plan.h"

namespace tnt {

// Convert exceptions into status codes at the ABI boundary.
#define TNT_API_BEGIN(ctx_)                                   \
  if (!(ctx_)) return TNT_E_ARG;                              \
  ::tnt::Ctx& c = *reinterpret_cast<::tnt::Ctx*>(ctx_);       \
  (void)c;                                                    \
  try {
#define TNT_API_END                                           \
  return TNT_OK;                                              \
  }                                                           \
  catch (const ::tnt::Error& e) {                             \
    c.last_error = e.what();                                  \
    return e.code;                                            \
  }                                                           \
  catch (const std::bad_alloc&) {                             \
    c.last_error = "host allocation failed";                  \
    return TNT_E_ALLOC;                                       \
  }                                                           \
  catch (const std::exception& e) {                           \
    c.last_error = e.what();                                  \
    return TNT_E_ARG;                                         \
  }

struct Hasher {
  uint64_t h = 1469598103934665603ULL;
  void add(const void* p, size_t n);
  template <typename T> void add(const T& v) { add(&v, sizeof(T)); }
};

struct HeffArgs {
  MpoH w1, w2;
  ThetaH th, out;
  EnvH L, R;
};

void check_precision(int32_t p);
HeffArgs parse_heff_args(const tnt_btensor* L, const tnt_mpo_site* W1, const tnt_mpo_site* W2,
                         const tnt_btensor* R, const tnt_btensor* theta, const tnt_btensor* out);
std::shared_ptr<HeffOp> cached_heff(Ctx& c, const HeffArgs& a, int prec);
// Operators for several argument sets: cache hits as they are, the host
// plans of the misses built on up to kPlanThreads threads, then their
// device tables one after another.
constexpr size_t kPlanThreads = 8;
std::vector<std::shared_ptr<HeffOp>> cached_heffs(Ctx& c, const std::vector<const HeffArgs*>& args,
                                                  int prec);
// Host plans only (same key and threads as cached_heffs, no device tables),
// and batch operators merged from such plans (cached by plan identities).
std::vector<std::shared_ptr<HeffPlan>> cached_plans(Ctx& c,
                                                   const std::vector<const HeffArgs*>& args,
                                                   int prec);
std::shared_ptr<BatchHeff> cached_plan_batch(Ctx& c,
                                             const std::vector<std::shared_ptr<HeffPlan>>& plans,
                                             const std::vector<int64_t>& L_ext,
                                             const std::vector<int64_t>& R_ext,
                                             const std::vector<int64_t>& n, int prec);

// A batched C-ABI call remembered by the hash of all its raw descriptors:
// the parsed instance layouts, operators, batch operator, and the call's own
// batch vectors, Krylov space and gather / scatter tables (so that repeated
// calls reuse buffers at stable addresses and skip every upload).
struct BatchCall {
  std::vector<std::shared_ptr<HeffOp>> ops;
  std::shared_ptr<BatchHeff> b;
  std::vector<ThetaH> tlay, olay;
  DevBuf xy;
  BatchKrylov K;
  RunTable in, back;
};
// hash of the raw host metadata of n instances (out may be NULL)
uint64_t raw_hash_batch(int n, const tnt_btensor* const* L, const tnt_mpo_site* const* W1,
                        const tnt_mpo_site* const* W2, const tnt_btensor* const* R,
                        const tnt_btensor* const* theta, const tnt_btensor* const* out,
                        int prec, uint64_t salt);
std::shared_ptr<BatchCall> find_batch_call(Ctx& c, uint64_t key);
void store_batch_call(Ctx& c, uint64_t key, std::shared_ptr<BatchCall> bc);

// Batch operator over these (cached) instance operators, built once per
// distinct sequence of instance operators and kept in the plan cache.
std::shared_ptr<BatchHeff> cached_batch(Ctx& c, const std::vector<std::shared_ptr<HeffOp>>& ops,
                                        const std::vector<int64_t>& n, int prec);
// Copy contiguous runs between device buffers (one launch).
void copy_runs(Ctx& c, const std::vector<CopyRun>& runs);

}  // namespace tnt
