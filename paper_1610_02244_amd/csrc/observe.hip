// Block dot products of the observables pass: out[t] = coef_t * sum_e x[e]
// conj(y[e]) over the n_t elements of task t (split-complex FP64 planes).
// One workgroup per task; each lane sums a strided slice, then the lanes of
// a wave and the waves of the workgroup are combined in a fixed order, so a
// result does not depend on timing.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace tnt {

constexpr int DOT_THREADS = 256;

__global__ __launch_bounds__(DOT_THREADS) void block_dot_kernel(
    const DotTask* __restrict__ tasks, const double* __restrict__ xre,
    const double* __restrict__ xim, const double* __restrict__ yre,
    const double* __restrict__ yim, double* __restrict__ out) {
  const DotTask t = tasks[blockIdx.x];
  double sr = 0.0, si = 0.0;
  for (int e = threadIdx.x; e < t.n; e += DOT_THREADS) {
    const double ar = xre[t.x_off + e], ai = xim[t.x_off + e];
    const double br = yre[t.y_off + e], bi = yim[t.y_off + e];
    sr += ar * br + ai * bi;
    si += ai * br - ar * bi;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o, 64);
    si += __shfl_xor(si, o, 64);
  }
  __shared__ double red[2][DOT_THREADS / 64];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    red[0][wave] = sr;
    red[1][wave] = si;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0, i = 0.0;
    for (int w = 0; w < DOT_THREADS / 64; ++w) {
      r += red[0][w];
      i += red[1][w];
    }
    out[2 * blockIdx.x] = t.coef * r;
    out[2 * blockIdx.x + 1] = t.coef * i;
  }
}

void launch_block_dots(const DotTask* tasks, int ntask, const double* xre, const double* xim,
                       const double* yre, const double* yim, double* out, hipStream_t s) {
  if (ntask <= 0) return;
  block_dot_kernel<<<ntask, DOT_THREADS, 0, s>>>(tasks, xre, xim, yre, yim, out);
}

}  // namespace tnt
