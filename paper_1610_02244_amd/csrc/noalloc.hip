// Allocation-free H_eff application for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid allocation).  Its task tables and intermediate slabs live in one
// statically sized device array owned by the library, one copy per GPU.
#include <map>
#include <mutex>

#include "capi_util.h"

namespace tnt {

// 64 MiB: the two-site operator of a chi = 256 chain (FP64 slabs ~25 MB).
constexpr size_t kScratchBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this GPU's copy of the array (the array's host-side
// name is not a device address).  Called at context creation with the
// context's device current; cached per device.
void* scratch_address(int device) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device)
    fail(TNT_E_STATE, "scratch address requested with another device current");
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    fail(TNT_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  addr[device] = p;
  return p;
}

size_t scratch_bytes() { return kScratchBytes; }

static size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace tnt

using namespace tnt;

extern "C" {

tnt_status tnt_heff2_apply_noalloc(tnt_ctx ctx, const tnt_btensor* L, const tnt_mpo_site* W1,
                                   const tnt_mpo_site* W2, const tnt_btensor* R,
                                   const tnt_btensor* theta, tnt_btensor* out,
                                   int32_t precision) {
  TNT_API_BEGIN(ctx)
  check_precision(precision);
  if (!out) fail(TNT_E_ARG, "null out");
  const HeffArgs a = parse_heff_args(L, W1, W2, R, theta, out);
  if (L->dtype != TNT_DT_F64 || R->dtype != TNT_DT_F64 || theta->dtype != TNT_DT_F64 ||
      out->dtype != TNT_DT_F64)
    fail(TNT_E_ARG, "L, R, theta and out must be FP64 planes");
  if (!c.scratch) fail(TNT_E_STATE, "no scratch array on this device");
  // host plan with the default (or cached) tile shapes, no timing launches
  HeffOp op;
  op.plan_tables(c, build_heff_plan(a.L, a.w1, a.w2, a.R, a.th, a.out, precision != TNT_FP64),
                 precision, false);
  op.L_ext = a.L.extent;
  op.R_ext = a.R.extent;
  // scratch layout: tables, then the slab and packed-operand workspaces
  int64_t ws[5];
  op.ws_bytes(precision, ws);
  char* base = static_cast<char*>(c.scratch);
  size_t off = up256(op.table_bytes());
  void* at[5] = {};
  for (int i = 0; i < 5; ++i) {
    if (ws[i] <= 0) continue;
    at[i] = base + off;
    off = up256(off + (size_t)ws[i]);
  }
  if (off > kScratchBytes)
    fail(TNT_E_CAPACITY, "this operator needs " + std::to_string(off) +
                             " bytes of scratch; the allocation-free path holds " +
                             std::to_string(kScratchBytes));
  for (int i = 0; i < 5; ++i) op.ext_ws[i] = at[i];
  op.upload_tables(base);
  op.bind_envs(L->re, L->im, R->re, R->im);
  op.apply(static_cast<const double*>(theta->re), static_cast<const double*>(theta->im),
           static_cast<double*>(out->re), static_cast<double*>(out->im), precision);
  TNT_HIP(hipGetLastError());
  // the host image of the tables is released on return
  TNT_HIP(hipStreamSynchronize(c.stream));
  TNT_API_END
}

}  // extern "C"
