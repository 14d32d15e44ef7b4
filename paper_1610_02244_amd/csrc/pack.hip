// Producers of packed operands (kernels.h): copies of FP64 blocks (the
// environments once per bond, theta once per matvec, transposed so that its
// contracted index is contiguous) and the MPO combination writing the
// step-4 slabs directly in packed form.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace tnt {

// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), both rounded to
// nearest even (x - hi is exact in FP32)
__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

template <int FMT>
__device__ inline void put_packed(char* __restrict__ dst, int64_t plane, int64_t idx, float re,
                                  float im) {
  if constexpr (FMT == PK_F32) {
    float* d = reinterpret_cast<float*>(dst);
    d[idx] = re;
    d[plane + idx] = im;
  } else {
    __bf16* d = reinterpret_cast<__bf16*>(dst);
    __bf16 h, l;
    split_bf16(re, h, l);
    d[idx] = h;
    d[plane + idx] = l;
    split_bf16(im, h, l);
    d[2 * plane + idx] = h;
    d[3 * plane + idx] = l;
  }
}

// One 32 x 32 destination tile per workgroup (256 threads = 32 x 8).  A
// transposed copy goes through LDS so that both the source reads and the
// destination writes are row-contiguous.
template <int FMT>
__global__ __launch_bounds__(256) void pack_kernel(const PackTask* __restrict__ tasks,
                                                   const int2* __restrict__ tiles,
                                                   const double* __restrict__ sre,
                                                   const double* __restrict__ sim,
                                                   char* __restrict__ dst, int64_t plane) {
  __shared__ double tr[2][PACK_TILE][PACK_TILE + 1];
  const int2 tl = tiles[blockIdx.x];
  const PackTask t = tasks[tl.x];
  const int r0 = (tl.y & 0xffff) * PACK_TILE, c0 = (tl.y >> 16) * PACK_TILE;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  if (t.trans) {
    // source rows are destination columns
#pragma unroll
    for (int i = 0; i < PACK_TILE / 8; ++i) {
      const int sr = c0 + ty + 8 * i, sc = r0 + tx;
      double a = 0, b = 0;
      if (sr < t.cols && sc < t.rows) {
        const int64_t k = t.src_off + (int64_t)sr * t.sld + sc;
        a = sre[k];
        b = sim[k];
      }
      tr[0][ty + 8 * i][tx] = a;
      tr[1][ty + 8 * i][tx] = b;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PACK_TILE / 8; ++i) {
      const int r = r0 + ty + 8 * i, c = c0 + tx;
      if (r < t.rows && c < t.dld)
        put_packed<FMT>(dst, plane, t.dst_off + (int64_t)r * t.dld + c,
                        (float)tr[0][tx][ty + 8 * i], (float)tr[1][tx][ty + 8 * i]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < PACK_TILE / 8; ++i) {
      const int r = r0 + ty + 8 * i, c = c0 + tx;
      if (r < t.rows && c < t.dld) {
        float a = 0, b = 0;
        if (c < t.cols) {
          const int64_t k = t.src_off + (int64_t)r * t.sld + c;
          a = (float)sre[k];
          b = (float)sim[k];
        }
        put_packed<FMT>(dst, plane, t.dst_off + (int64_t)r * t.dld + c, a, b);
      }
    }
  }
}

void launch_pack(const PackTask* tasks, const int2* tiles, int ntiles, const double* sre,
                 const double* sim, void* dst, int64_t plane, PackFmt f, hipStream_t s) {
  if (ntiles <= 0) return;
  if (f == PK_F32)
    hipLaunchKernelGGL(pack_kernel<PK_F32>, dim3(ntiles), dim3(256), 0, s, tasks, tiles, sre,
                       sim, static_cast<char*>(dst), plane);
  else
    hipLaunchKernelGGL(pack_kernel<PK_BF16X3>, dim3(ntiles), dim3(256), 0, s, tasks, tiles, sre,
                       sim, static_cast<char*>(dst), plane);
}

template <int FMT>
__global__ __launch_bounds__(256) void combine_packed_kernel(
    const CombPTask* __restrict__ tasks, const CombTerm* __restrict__ terms,
    const int2* __restrict__ chunks, const float* __restrict__ sre,
    const float* __restrict__ sim, char* __restrict__ dst, int64_t plane) {
  const int2 c = chunks[blockIdx.x];
  const CombPTask tk = tasks[c.x];
  const int total = tk.rows * tk.dld;
  const int base = c.y * COMB_CHUNK;
#pragma unroll
  for (int e = 0; e < COMB_CHUNK / 256; ++e) {
    const int i = base + e * 256 + threadIdx.x;
    if (i >= total) break;
    const int r = i / tk.dld, col = i - r * tk.dld;
    float ar = 0, ai = 0;
    if (col < tk.cols) {
      const int si = r * tk.cols + col;
      for (int t = 0; t < tk.nterm; ++t) {
        const CombTerm tm = terms[tk.term0 + t];
        const float cf = (float)tm.coef;
        ar += cf * sre[tm.src_off + si];
        ai += cf * sim[tm.src_off + si];
      }
    }
    put_packed<FMT>(dst, plane, tk.dst_off + i, ar, ai);
  }
}

void launch_combine_packed(const CombPTask* tasks, const CombTerm* terms, const int2* chunks,
                           int32_t nchunks, const float* src_re, const float* src_im, void* dst,
                           int64_t plane, PackFmt f, hipStream_t s) {
  if (nchunks <= 0) return;
  if (f == PK_F32)
    hipLaunchKernelGGL(combine_packed_kernel<PK_F32>, dim3(nchunks), dim3(256), 0, s, tasks,
                       terms, chunks, src_re, src_im, static_cast<char*>(dst), plane);
  else
    hipLaunchKernelGGL(combine_packed_kernel<PK_BF16X3>, dim3(nchunks), dim3(256), 0, s, tasks,
                       terms, chunks, src_re, src_im, static_cast<char*>(dst), plane);
}

}  // namespace tnt
