// Internal shared definitions: context, device pool, error plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tnt.h"

namespace tnt {

// An error carrying a status code; converted to a return value at the C-ABI.
struct Error : std::runtime_error {
  tnt_status code;
  Error(tnt_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(tnt_status c, const std::string& m) { throw Error(c, m); }

#define TNT_HIP(call)                                                             \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      ::tnt::fail(TNT_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

// Caching device pool: allocations are rounded up to a size class and kept
// for reuse after release, so steady-state sweeps call hipMalloc only while
// bond dimensions grow.  Released blocks are reused only after the context
// stream has passed the release point (the pool is per-stream and every
// kernel runs on that stream, so stream order makes reuse safe).  Block
// sizes drift along a sweep (every bond has other dimensions), so cached
// blocks that no request fits pile up: before allocating more, the pool
// returns its cached blocks to the runtime when they exceed both
// kCacheFloor and the bytes in use.
class Pool {
 public:
  static constexpr int64_t kCacheFloor = int64_t(4) << 30;
  ~Pool();
  void* get(size_t bytes);
  void put(void* p);
  int64_t held() const { return held_; }
  int64_t in_use() const { return in_use_; }
  int64_t peak_in_use() const { return peak_; }
  void release_all();

 private:
  static size_t round(size_t b);
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> live_;
  int64_t held_ = 0, in_use_ = 0, peak_ = 0;
};

// RAII handle on pool memory.
struct DevBuf {
  Pool* pool = nullptr;
  void* ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(Pool* p, size_t b) : pool(p), ptr(b ? p->get(b) : nullptr), bytes(b) {}
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      reset();
      pool = o.pool; ptr = o.ptr; bytes = o.bytes;
      o.ptr = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { reset(); }
  void reset() {
    if (ptr && pool) pool->put(ptr);
    ptr = nullptr; bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(ptr); }
  // grow-only (contents not preserved)
  void ensure(Pool* p, size_t b) {
    if (b > bytes) { reset(); pool = p; ptr = p->get(b); bytes = b; }
  }
};

struct Ctx;
// Per-context cache of device task tables keyed by a plan signature.
struct PlanCache;

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Pool pool;
  std::string last_error;
  void* blas = nullptr;    // rocblas_handle, created on first SVD
  PlanCache* plans = nullptr;
  hipEvent_t ev[8] = {};
  // per-step timing events of the Lanczos recurrence (grown on demand)
  std::vector<hipEvent_t> step_ev;
  int num_cu = 256;
  // shared H_eff workspaces (one operator runs at a time per context):
  // 0 = L.theta slabs, 1 = MPO-combined slabs, 2 / 3 = packed L / R copies,
  // 4 = packed theta
  DevBuf ws[5];
  // side streams (default priority) with their own rocBLAS handles, used to
  // run independent per-sector dense factorizations concurrently
  // tile-shape decisions of the autotuner per shape bucket (0 = tuning off)
  int autotune = 1;
  // Lanczos recurrence replayed from a HIP graph (tnt_ctx_set_graphs); the
  // recording runs on a stream of its own (the context's stream may be the
  // null stream, which cannot be recorded)
  int graphs = 0;
  // sector eigenproblems the SVD redid with the Jacobi eigensolver because
  // divide and conquer failed or returned non-finite vectors (running count)
  int64_t eig_retries = 0;
  // sector eigenproblems whose padded order is at least this use the library's
  // divide and conquer on a tridiagonal form reduced by trd.hip; smaller ones,
  // and every one when 0, use the library's whole Hermitian eigensolver
  static constexpr int kEigTrdDefault = 0;
  int eig_trd_min = kEigTrdDefault;
  hipStream_t gstream = nullptr;
  std::map<uint64_t, int> tune_cache;
  static constexpr int kSide = 8;
  hipStream_t side[kSide] = {};
  void* side_blas[kSide] = {};
  hipEvent_t side_ev[kSide + 1] = {};
  // this device's copy of the allocation-free path's scratch array
  void* scratch = nullptr;
  ~Ctx();
};

// Device address of the scratch array on `device` (which must be current).
void* scratch_address(int device);
size_t scratch_bytes();

// Pinned host staging for small device->host reads (Lanczos scalars).
struct HostStage {
  double* p = nullptr;
  size_t n = 0;
  void ensure(size_t want) {
    if (want <= n) return;
    if (p) (void)hipHostFree(p);
    if (hipHostMalloc(reinterpret_cast<void**>(&p), want * sizeof(double)) != hipSuccess) {
      p = nullptr; n = 0;
      fail(TNT_E_ALLOC, "hipHostMalloc failed");
    }
    n = want;
  }
  ~HostStage() { if (p) (void)hipHostFree(p); }
};

}  // namespace tnt
