// Two-site gate on theta: theta'(qa, s1', s2') = sum_{s1 + s2 = s1' + s2'}
// G[(s1' s2'), (s1 s2)] theta(qa, s1, s2), complex coefficients on
// split-complex FP64 planes.  The gate conserves the charge, so every source
// block of a destination block has its shape and the sum is elementwise;
// a workgroup takes GATE_CHUNK consecutive elements of one destination
// block and reads each of its (at most d) source blocks once, coalesced.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace tnt {

constexpr int GATE_THREADS = 256;

__global__ __launch_bounds__(GATE_THREADS) void gate_apply_kernel(
    const GateTask* __restrict__ tasks, const GateTerm* __restrict__ terms,
    const int2* __restrict__ chunks, const double* __restrict__ sre,
    const double* __restrict__ sim, double* __restrict__ dre, double* __restrict__ dim) {
  const int2 ch = chunks[blockIdx.x];
  const GateTask t = tasks[ch.x];
  const int base = ch.y * GATE_CHUNK;
  const int end = min(t.size, base + GATE_CHUNK);
  for (int e = base + (int)threadIdx.x; e < end; e += GATE_THREADS) {
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < t.nterm; ++k) {
      const GateTerm g = terms[t.term0 + k];
      const double xr = sre[g.src_off + e], xi = sim[g.src_off + e];
      ar += g.cr * xr - g.ci * xi;
      ai += g.cr * xi + g.ci * xr;
    }
    dre[t.dst_off + e] = ar;
    dim[t.dst_off + e] = ai;
  }
}

void launch_gate_apply(const GateTask* tasks, const GateTerm* terms, const int2* chunks,
                       int nchunks, const double* sre, const double* sim, double* dre,
                       double* dim, hipStream_t s) {
  if (nchunks <= 0) return;
  gate_apply_kernel<<<nchunks, GATE_THREADS, 0, s>>>(tasks, terms, chunks, sre, sim, dre, dim);
}

}  // namespace tnt
