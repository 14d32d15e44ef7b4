// Caching device pool and context lifetime.
#include <algorithm>

#include "common.h"

namespace tnt {

size_t Pool::round(size_t b) {
  if (b <= (size_t(1) << 20)) {
    size_t r = 256;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t g = size_t(2) << 20;  // 2 MiB granules above 1 MiB
  return (b + g - 1) / g * g;
}

void* Pool::get(size_t bytes) {
  const size_t r = round(std::max<size_t>(bytes, 1));
  // smallest cached block that fits without wasting more than half of it
  auto it = free_.lower_bound(r);
  if (it != free_.end() && it->first <= 2 * r) {
    void* p = it->second;
    live_[p] = it->first;
    in_use_ += (int64_t)it->first;
    peak_ = std::max(peak_, in_use_);
    free_.erase(it);
    return p;
  }
  // cached blocks that no request fits: hand them back before growing
  const int64_t cached = held_ - in_use_;
  if (cached > kCacheFloor && cached > in_use_) release_all();
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, r);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_all();  // return cached blocks to the runtime and retry once
    e = hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(TNT_E_ALLOC, "device allocation of " + std::to_string(r) + " bytes failed");
    }
  }
  live_[p] = r;
  held_ += (int64_t)r;
  in_use_ += (int64_t)r;
  peak_ = std::max(peak_, in_use_);
  return p;
}

void Pool::put(void* p) {
  auto it = live_.find(p);
  if (it == live_.end()) return;
  free_.insert({it->second, p});
  in_use_ -= (int64_t)it->second;
  live_.erase(it);
}

void Pool::release_all() {
  // hipFree synchronises the device, so blocks still read by queued kernels
  // are not returned early.
  for (auto& kv : free_) {
    (void)hipFree(kv.second);
    held_ -= (int64_t)kv.first;
  }
  free_.clear();
}

Pool::~Pool() {
  release_all();
  for (auto& kv : live_) (void)hipFree(kv.first);
  live_.clear();
  in_use_ = 0;
}

}  // namespace tnt
