// Device-side building blocks shared by the grouped-GEMM kernels: MFMA
// wrappers with their gfx950 lane layouts and the K-chunk walker.
//
// gfx950 MFMA lane layouts (64 lanes, slot = lane / 16):
//   16x16x4 f32 / f64: A lane l holds A[l % 16][slot], B lane l holds
//     B[slot][l % 16];
//   16x16x32 bf16: A lane l holds A[l % 16][8 slot + e], B lane l holds
//     B[8 slot + e][l % 16], e = 0..7;
//   f32 result register r of lane l: C[4 slot + r][l % 16] (both shapes);
//   f64 result register r of lane l: C[4 r + slot][l % 16].
#pragma once

#include "kernels.h"

namespace tnt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<float> {
  typedef f32x4 acc_t;
  typedef f32x4 quad_t;
  __device__ static inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mma<double> {
  typedef f64x4 acc_t;
  typedef f64x4 quad_t;
  __device__ static inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int NT = 256;  // threads per workgroup: 4 waves, 2 x 2 over the output tile

// Walks the K-chunks (segment, k0) of one task in summation order.  The
// next chunk is fetched into registers (load) while the current LDS stage is
// consumed (compute); store moves the registers into a stage.  With two
// stages the chunks alternate between them and one barrier per chunk
// suffices; with one stage the store waits for every wave's compute.
template <int BK, int STAGES, typename Load, typename Store, typename Compute>
__device__ inline void walk_chunks(const GemmSeg* __restrict__ segs, int seg0, int nseg,
                                   Load& load, Store& store, Compute& compute) {
  int s = 0;
  GemmSeg cur;
  if (nseg > 0) {
    cur = segs[seg0];
    while (cur.K <= 0 && ++s < nseg) cur = segs[seg0 + s];
  }
  if (s < nseg) {
    load(cur, 0);
    store(0);
    __syncthreads();
  }
  int k0 = 0, st = 0;
  while (s < nseg) {
    const int kvalid = min(BK, cur.K - k0);
    int ns = s, nk0 = k0 + BK;
    GemmSeg nxt = cur;
    if (nk0 >= cur.K) {
      nk0 = 0;
      ++ns;
      while (ns < nseg) {
        nxt = segs[seg0 + ns];
        if (nxt.K > 0) break;
        ++ns;
      }
    }
    const bool more = ns < nseg;
    if (more) load(nxt, nk0);
    compute(st, kvalid);
    if (STAGES == 1) {
      __syncthreads();
      if (more) store(0);
      __syncthreads();
    } else {
      if (more) store(st ^ 1);
      __syncthreads();
      st ^= 1;
    }
    s = ns;
    k0 = nk0;
    cur = nxt;
  }
}

}  // namespace tnt
