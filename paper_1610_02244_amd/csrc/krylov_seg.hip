// Segmented Krylov-vector kernels of the batched Lanczos recurrence.
//
// A batch vector holds the vectors of several independent problems: complex
// entries [off_i, off_i + n_i) of instance i, stored as a re plane of N
// doubles followed by an im plane (N = sum of n_i).  Each workgroup owns one
// contiguous range inside one instance (SegBlock), so reductions are
// per-block partial sums added per instance in block order (deterministic),
// and per-instance scalars are read at base + inst * stride.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace tnt {

__device__ inline double seg_block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;  // valid in thread 0
}

constexpr int SEG_MAXK = 32;

// out[inst * out_stride + j] = sum over the instance's blocks of
// partial[b * k2 + j], in block order
__global__ void seg_reduce_kernel(const double* __restrict__ partial, int k2,
                                  const int2* __restrict__ inst_blk,
                                  double* __restrict__ out, int out_stride) {
  __shared__ double sh[4];
  const int j = blockIdx.x, inst = blockIdx.y;
  const int2 r = inst_blk[inst];
  double v = 0;
  for (int b = r.x + threadIdx.x; b < r.y; b += blockDim.x) v += partial[b * k2 + j];
  const double t = seg_block_sum(v, sh);
  if (threadIdx.x == 0) out[inst * out_stride + j] = t;
}

void launch_seg_reduce(const double* partial, int k2, const int2* inst_blk, int ninst,
                       double* out, int out_stride, hipStream_t s) {
  hipLaunchKernelGGL(seg_reduce_kernel, dim3(k2, ninst), dim3(256), 0, s, partial, k2, inst_blk,
                     out, out_stride);
}

// w -= a_i v1 + b_i v0 on instance i's entries (v0 may be NULL)
__global__ __launch_bounds__(RED_THREADS) void seg_axpy2_kernel(
    const double* __restrict__ v1, const double* __restrict__ a, int a_stride,
    const double* __restrict__ v0, const double* __restrict__ b, int b_stride,
    double* __restrict__ w, int64_t N, const SegBlock* __restrict__ blk) {
  const SegBlock sb = blk[blockIdx.x];
  const double ai = a[sb.inst * a_stride];
  const double bi = v0 ? b[sb.inst * b_stride] : 0.0;
  for (int64_t x = sb.lo + threadIdx.x; x < sb.hi; x += RED_THREADS) {
    double r = w[x] - ai * v1[x], m = w[N + x] - ai * v1[N + x];
    if (v0) {
      r -= bi * v0[x];
      m -= bi * v0[N + x];
    }
    w[x] = r;
    w[N + x] = m;
  }
}

void launch_seg_axpy2(const double* v1, const double* a, int a_stride, const double* v0,
                      const double* b, int b_stride, double* w, int64_t N, const SegBlock* blk,
                      int nblk, hipStream_t s) {
  hipLaunchKernelGGL(seg_axpy2_kernel, dim3(nblk), dim3(RED_THREADS), 0, s, v1, a, a_stride, v0,
                     b, b_stride, w, N, blk);
}

// |x|^2 partials per block
__global__ __launch_bounds__(RED_THREADS) void seg_norm2_kernel(const double* __restrict__ x,
                                                                int64_t N,
                                                                const SegBlock* __restrict__ blk,
                                                                double* __restrict__ part) {
  __shared__ double sh[4];
  const SegBlock sb = blk[blockIdx.x];
  double acc = 0;
  for (int64_t i = sb.lo + threadIdx.x; i < sb.hi; i += RED_THREADS)
    acc += x[i] * x[i] + x[N + i] * x[N + i];
  const double r = seg_block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

void launch_seg_norm2(const double* x, int64_t N, const SegBlock* blk, int nblk, double* part,
                      hipStream_t s) {
  hipLaunchKernelGGL(seg_norm2_kernel, dim3(nblk), dim3(RED_THREADS), 0, s, x, N, blk, part);
}

// dst = src * f_i with f_i = scale[i * stride] (mode 0) or
// 1 / sqrt(scale[i * stride]) (mode 1, zero for a non-positive norm)
__global__ __launch_bounds__(RED_THREADS) void seg_scale_copy_kernel(
    const double* __restrict__ src, double* __restrict__ dst, int64_t N,
    const SegBlock* __restrict__ blk, const double* __restrict__ scale, int stride, int mode) {
  const SegBlock sb = blk[blockIdx.x];
  const double v = scale[sb.inst * stride];
  const double f = mode == 0 ? v : (v > 0 ? 1.0 / sqrt(v) : 0.0);
  for (int64_t x = sb.lo + threadIdx.x; x < sb.hi; x += RED_THREADS) {
    dst[x] = src[x] * f;
    dst[N + x] = src[N + x] * f;
  }
}

void launch_seg_scale_copy(const double* src, double* dst, int64_t N, const SegBlock* blk,
                           int nblk, const double* scale, int stride, int mode, hipStream_t s) {
  hipLaunchKernelGGL(seg_scale_copy_kernel, dim3(nblk), dim3(RED_THREADS), 0, s, src, dst, N,
                     blk, scale, stride, mode);
}

// out = sum_{i < k} y_{inst,i} V_i (real y at y + inst * y_stride)
__global__ __launch_bounds__(RED_THREADS) void seg_combine_basis_kernel(
    const double* __restrict__ V, int64_t ld, int k, const double* __restrict__ y, int y_stride,
    double* __restrict__ out, int64_t N, const SegBlock* __restrict__ blk) {
  __shared__ double ys[SEG_MAXK];
  const SegBlock sb = blk[blockIdx.x];
  if (threadIdx.x < k) ys[threadIdx.x] = y[sb.inst * y_stride + threadIdx.x];
  __syncthreads();
  for (int64_t x = sb.lo + threadIdx.x; x < sb.hi; x += RED_THREADS) {
    double r = 0, m = 0;
    for (int i = 0; i < k; ++i) {
      r += ys[i] * V[i * ld + x];
      m += ys[i] * V[i * ld + N + x];
    }
    out[x] = r;
    out[N + x] = m;
  }
}

void launch_seg_combine_basis(const double* V, int64_t ld, int k, const double* y, int y_stride,
                              double* out, int64_t N, const SegBlock* blk, int nblk,
                              hipStream_t s) {
  hipLaunchKernelGGL(seg_combine_basis_kernel, dim3(nblk), dim3(RED_THREADS), 0, s, V, ld, k, y,
                     y_stride, out, N, blk);
}

// ---------------------------------------------------------------------------
// Fused steps of the re-orthogonalised recurrence.  Each kernel leaves
// per-workgroup partial sums part[b * W + o] (W values per workgroup) and
// the next kernel starts by adding up its instance's partials, every
// workgroup on its own in the same fixed order: all workgroups obtain
// bitwise the same coefficients without a separate reduction launch and
// without any communication inside a launch.  The basis size K is a
// template parameter, so the loads of all K vectors for one entry are
// issued together.
// ---------------------------------------------------------------------------

// sum over the instance's workgroups [b0, b1) of part[b * W + o], o < W,
// into out[o] (LDS); every thread of the workgroup must call it
template <int W>
__device__ inline void instance_sums(const double* __restrict__ part, int b0, int b1,
                                     double* red, double* out) {
  constexpr int NSUB = RED_THREADS / W;  // workgroup subsets, each over every NSUB-th partial
  const int t = threadIdx.x;
  if constexpr (W == 1) {
    double v = 0;
    for (int b = b0 + t; b < b1; b += RED_THREADS) v += part[b];
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    if (t == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return;
  }
  if (t < NSUB * W) {
    const int o = t % W, sub = t / W;
    double v = 0;
    for (int b = b0 + sub; b < b1; b += NSUB) v += part[(size_t)b * W + o];
    red[sub * W + o] = v;
  }
  __syncthreads();
  if (t < W) {
    double v = 0;
    for (int sub = 0; sub < NSUB; ++sub) v += red[sub * W + t];
    out[t] = v;
  }
  __syncthreads();
}

// Two forms of each basis pass.  "lanes": every lane carries all K basis
// entries and 2K projection sums of its entries; for small K this streams
// at 5-7 TB/s.  "waves": the basis is split over the workgroup's waves
// (below); fewer registers per lane, so from about ten vectors on it keeps
// its occupancy where the lanes form drops to two waves per SIMD
// (K = 20 update pass on a 2.9M-entry vector: 291 us against 489 us).

// --- lanes form ------------------------------------------------------------

// smallest power of two >= n
constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }

// P values per lane in (P a power of two <= 64); lane L < P out with the
// wave total of value L.  Recursive halving, stage by stage over all
// values so the shuffles of one stage are independent: each stage sends
// half of the remaining values to the partner lane (P - 1 shuffles for
// P = 64, plus one full exchange per lane bit above P).
template <int P>
__device__ inline double wave_reduce_scatter(double* v) {
  static_assert(P >= 1 && P <= 64 && (P & (P - 1)) == 0, "P must be a power of two <= 64");
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 32; o >= P; o >>= 1) {
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] += __shfl_xor(v[i], o, 64);
  }
#pragma unroll
  for (int o = P / 2; o >= 1; o >>= 1) {
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < o; ++i) {
      const double lo = v[i], hi = v[i + o];
      v[i] = (up ? hi : lo) + __shfl_xor(up ? lo : hi, o, 64);
    }
  }
  return v[0];
}

// workgroup totals of the first W of P per-thread values (P =
// pow2_at_least(W), the rest zero) into part[blockIdx.x * W + o]; red
// holds 4 * P doubles
template <int W, int P>
__device__ inline void block_partials(double* v, double* red, double* part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double r = wave_reduce_scatter<P>(v);
  if (lane < P) red[wv * P + lane] = r;
  __syncthreads();
  if (threadIdx.x < W) {
    const int o = threadIdx.x;
    part[(size_t)blockIdx.x * W + o] = (red[o] + red[P + o]) + (red[2 * P + o] + red[3 * P + o]);
  }
}

// partials of c = V^H w over V_0 .. V_{K-1}, as (re, im) pairs
template <int K>
__global__ __launch_bounds__(RED_THREADS) void seg_cgs_dot_lanes(
    const double* __restrict__ V, int64_t ld, const double* __restrict__ w, int64_t N,
    const SegBlock* __restrict__ blk, double* __restrict__ part) {
  constexpr int P = pow2_at_least(2 * K);
  __shared__ double red[4 * P];
  const SegBlock sb = blk[blockIdx.x];
  double acc[P];
#pragma unroll
  for (int o = 0; o < P; ++o) acc[o] = 0;
  for (int64_t x = sb.lo + threadIdx.x; x < sb.hi; x += RED_THREADS) {
    const double wr = w[x], wi = w[N + x];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const double vr = V[i * ld + x], vi = V[i * ld + N + x];
      acc[2 * i] += vr * wr + vi * wi;
      acc[2 * i + 1] += vr * wi - vi * wr;
    }
  }
  block_partials<2 * K, P>(acc, red, part);
}

// c = the instance's sum of part_in (2K values); w -= V c; partials of
// V^H w into part_out.  The instance's first workgroup writes the pair of
// V_{K-1} to pair_dst + inst * S (the recurrence's alpha_j).
template <int K>
__global__ __launch_bounds__(RED_THREADS) void seg_cgs_update_dot_lanes(
    const double* __restrict__ V, int64_t ld, const double* __restrict__ part_in,
    double* __restrict__ w, int64_t N, const SegBlock* __restrict__ blk,
    const int2* __restrict__ inst_blk, double* __restrict__ part_out,
    double* __restrict__ pair_dst, int S) {
  constexpr int P = pow2_at_least(2 * K);
  __shared__ double red[RED_THREADS > 4 * P ? RED_THREADS : 4 * P];
  __shared__ double cs[2 * K];
  const SegBlock sb = blk[blockIdx.x];
  const int2 r = inst_blk[sb.inst];
  instance_sums<2 * K>(part_in, r.x, r.y, red, cs);
  if (pair_dst && blockIdx.x == r.x && threadIdx.x < 2)
    pair_dst[(size_t)sb.inst * S + threadIdx.x] = cs[2 * (K - 1) + threadIdx.x];
  double acc[P];
#pragma unroll
  for (int o = 0; o < P; ++o) acc[o] = 0;
  for (int64_t x = sb.lo + threadIdx.x; x < sb.hi; x += RED_THREADS) {
    double wr = w[x], wi = w[N + x];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const double vr = V[i * ld + x], vi = V[i * ld + N + x];
      const double cr = cs[2 * i], ci = cs[2 * i + 1];
      wr -= cr * vr - ci * vi;
      wi -= cr * vi + ci * vr;
    }
    w[x] = wr;
    w[N + x] = wi;
    // read the basis again (from cache) rather than holding 2K values in
    // registers across the update: half the registers, twice the occupancy
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const double vr = V[i * ld + x], vi = V[i * ld + N + x];
      acc[2 * i] += vr * wr + vi * wi;
      acc[2 * i + 1] += vr * wi - vi * wr;
    }
  }
  __syncthreads();  // red is reused
  block_partials<2 * K, P>(acc, red, part_out);
}

// c = the instance's sum of part_in; w -= V c; partials of |w|^2 into
// part_out (one value per workgroup)
template <int K>
__global__ __launch_bounds__(RED_THREADS) void seg_cgs_update_norm_lanes(
    const double* __restrict__ V, int64_t ld, const double* __restrict__ part_in,
    double* __restrict__ w, int64_t N, const SegBlock* __restrict__ blk,
    const int2* __restrict__ inst_blk, double* __restrict__ part_out) {
  __shared__ double red[RED_THREADS];
  __shared__ double cs[2 * K];
  const SegBlock sb = blk[blockIdx.x];
  const int2 r = inst_blk[sb.inst];
  instance_sums<2 * K>(part_in, r.x, r.y, red, cs);
  double acc[1] = {0};
  for (int64_t x = sb.lo + threadIdx.x; x < sb.hi; x += RED_THREADS) {
    double wr = w[x], wi = w[N + x];
    double vr[K], vi[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      vr[i] = V[i * ld + x];
      vi[i] = V[i * ld + N + x];
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const double cr = cs[2 * i], ci = cs[2 * i + 1];
      wr -= cr * vr[i] - ci * vi[i];
      wi -= cr * vi[i] + ci * vr[i];
    }
    w[x] = wr;
    w[N + x] = wi;
    acc[0] += wr * wr + wi * wi;
  }
  __syncthreads();
  block_partials<1, 1>(acc, red, part_out);
}

// --- waves form ------------------------------------------------------------
// The basis is split over the workgroup's four waves:
// wave v owns vectors i = v, v + 4, v + 8, ... (KW = ceil(K / 4) of them),
// and all four waves walk the same entries, SEG_U per lane per tile.  A
// lane then holds only its wave's share of the basis entries and of the
// projection sums (at most 2 * 8 of each for K <= 32), so the kernels run
// at high occupancy with every basis entry read from memory once; the
// update's partial sums meet in LDS.
constexpr int SEG_WAVES = RED_THREADS / 64;
constexpr int SEG_U = 2;                         // entries per lane per tile
constexpr int SEG_TILE = RED_THREADS / SEG_WAVES * SEG_U;   // 128 entries
static_assert(SEG_WAVES == 4, "the basis passes assume four waves per workgroup");

// sum over the wave's 64 lanes of each of M values; every lane gets the totals
template <int M>
__device__ inline void wave_sum_all(double* v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
    for (int i = 0; i < M; ++i) v[i] += __shfl_xor(v[i], o, 64);
  }
}

// loads the wave's basis entries of one tile (zero beyond hi)
template <int K, int KW>
__device__ inline void load_tile(const double* __restrict__ V, int64_t ld, int64_t N,
                                 int64_t x0, int64_t hi, int wv, double (&vr)[KW][SEG_U],
                                 double (&vi)[KW][SEG_U]) {
#pragma unroll
  for (int q = 0; q < KW; ++q) {
    const int i = wv + SEG_WAVES * q;
#pragma unroll
    for (int u = 0; u < SEG_U; ++u) {
      const int64_t x = x0 + 64 * u;
      const bool ok = i < K && x < hi;
      vr[q][u] = ok ? V[i * ld + x] : 0.0;
      vi[q][u] = ok ? V[i * ld + N + x] : 0.0;
    }
  }
}

// w_new = w - V c for one tile: each wave's share of V c (its vectors, in
// order) goes to LDS, every wave adds the four shares in the same fixed
// order and subtracts them from w.  Two barriers per tile keep `sh`
// single-buffered.
template <int K, int KW>
__device__ inline void tile_update(const double* __restrict__ w, int64_t N, int64_t x0,
                                   int64_t hi, int wv, int lane, const double* cs,
                                   const double (&vr)[KW][SEG_U], const double (&vi)[KW][SEG_U],
                                   double* sh, double (&wr)[SEG_U], double (&wi)[SEG_U]) {
#pragma unroll
  for (int u = 0; u < SEG_U; ++u) {
    double pr = 0, pi = 0;
#pragma unroll
    for (int q = 0; q < KW; ++q) {
      const int i = wv + SEG_WAVES * q;
      if (i < K) {
        const double cr = cs[2 * i], ci = cs[2 * i + 1];
        pr += cr * vr[q][u] - ci * vi[q][u];
        pi += cr * vi[q][u] + ci * vr[q][u];
      }
    }
    sh[(wv * SEG_U + u) * 128 + lane] = pr;
    sh[(wv * SEG_U + u) * 128 + 64 + lane] = pi;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < SEG_U; ++u) {
    const int64_t x = x0 + 64 * u;
    const double* s0 = sh + u * 128 + lane;
    constexpr int WS = SEG_U * 128;  // stride between the waves' shares
    const double pr = (s0[0] + s0[WS]) + (s0[2 * WS] + s0[3 * WS]);
    const double pi = (s0[64] + s0[WS + 64]) + (s0[2 * WS + 64] + s0[3 * WS + 64]);
    wr[u] = x < hi ? w[x] - pr : 0.0;
    wi[u] = x < hi ? w[N + x] - pi : 0.0;
  }
  __syncthreads();
}

// the wave's 2 * KW projection sums (one wave per vector, no cross-wave
// sum) into part[blockIdx.x * 2K + 2i + {0, 1}]
template <int K, int KW>
__device__ inline void store_projections(double (&acc)[2 * KW], int wv, int lane,
                                         double* __restrict__ part) {
  wave_sum_all<2 * KW>(acc);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < KW; ++q) {
      const int i = wv + SEG_WAVES * q;
      if (i < K) {
        part[(size_t)blockIdx.x * 2 * K + 2 * i] = acc[2 * q];
        part[(size_t)blockIdx.x * 2 * K + 2 * i + 1] = acc[2 * q + 1];
      }
    }
  }
}

// partials of c = V^H w over V_0 .. V_{K-1}, as (re, im) pairs
template <int K>
__global__ __launch_bounds__(RED_THREADS) void seg_cgs_dot_waves(
    const double* __restrict__ V, int64_t ld, const double* __restrict__ w, int64_t N,
    const SegBlock* __restrict__ blk, double* __restrict__ part) {
  constexpr int KW = (K + SEG_WAVES - 1) / SEG_WAVES;
  const SegBlock sb = blk[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[2 * KW];
#pragma unroll
  for (int o = 0; o < 2 * KW; ++o) acc[o] = 0;
  for (int64_t t = sb.lo; t < sb.hi; t += SEG_TILE) {
    double vr[KW][SEG_U], vi[KW][SEG_U];
    load_tile<K, KW>(V, ld, N, t + lane, sb.hi, wv, vr, vi);
#pragma unroll
    for (int u = 0; u < SEG_U; ++u) {
      const int64_t x = t + lane + 64 * u;
      const double wr = x < sb.hi ? w[x] : 0.0, wi = x < sb.hi ? w[N + x] : 0.0;
#pragma unroll
      for (int q = 0; q < KW; ++q) {
        acc[2 * q] += vr[q][u] * wr + vi[q][u] * wi;
        acc[2 * q + 1] += vr[q][u] * wi - vi[q][u] * wr;
      }
    }
  }
  store_projections<K, KW>(acc, wv, lane, part);
}

// c = the instance's sum of part_in (2K values); w -= V c; partials of
// V^H w into part_out.  The instance's first workgroup writes the pair of
// V_{K-1} to pair_dst + inst * S (the recurrence's alpha_j).
template <int K>
__global__ __launch_bounds__(RED_THREADS) void seg_cgs_update_dot_waves(
    const double* __restrict__ V, int64_t ld, const double* __restrict__ part_in,
    double* __restrict__ w, int64_t N, const SegBlock* __restrict__ blk,
    const int2* __restrict__ inst_blk, double* __restrict__ part_out,
    double* __restrict__ pair_dst, int S) {
  constexpr int KW = (K + SEG_WAVES - 1) / SEG_WAVES;
  __shared__ double red[RED_THREADS > 4 * SEG_U * 128 ? RED_THREADS : 4 * SEG_U * 128];
  __shared__ double cs[2 * K];
  const SegBlock sb = blk[blockIdx.x];
  const int2 r = inst_blk[sb.inst];
  instance_sums<2 * K>(part_in, r.x, r.y, red, cs);
  if (pair_dst && blockIdx.x == r.x && threadIdx.x < 2)
    pair_dst[(size_t)sb.inst * S + threadIdx.x] = cs[2 * (K - 1) + threadIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[2 * KW];
#pragma unroll
  for (int o = 0; o < 2 * KW; ++o) acc[o] = 0;
  for (int64_t t = sb.lo; t < sb.hi; t += SEG_TILE) {
    double vr[KW][SEG_U], vi[KW][SEG_U], wr[SEG_U], wi[SEG_U];
    load_tile<K, KW>(V, ld, N, t + lane, sb.hi, wv, vr, vi);
    tile_update<K, KW>(w, N, t + lane, sb.hi, wv, lane, cs, vr, vi, red, wr, wi);
#pragma unroll
    for (int u = 0; u < SEG_U; ++u) {
      const int64_t x = t + lane + 64 * u;
      if (wv == 0 && x < sb.hi) {
        w[x] = wr[u];
        w[N + x] = wi[u];
      }
#pragma unroll
      for (int q = 0; q < KW; ++q) {
        acc[2 * q] += vr[q][u] * wr[u] + vi[q][u] * wi[u];
        acc[2 * q + 1] += vr[q][u] * wi[u] - vi[q][u] * wr[u];
      }
    }
  }
  store_projections<K, KW>(acc, wv, lane, part_out);
}

// c = the instance's sum of part_in; w -= V c; partials of |w|^2 into
// part_out (one value per workgroup)
template <int K>
__global__ __launch_bounds__(RED_THREADS) void seg_cgs_update_norm_waves(
    const double* __restrict__ V, int64_t ld, const double* __restrict__ part_in,
    double* __restrict__ w, int64_t N, const SegBlock* __restrict__ blk,
    const int2* __restrict__ inst_blk, double* __restrict__ part_out) {
  constexpr int KW = (K + SEG_WAVES - 1) / SEG_WAVES;
  __shared__ double red[RED_THREADS > 4 * SEG_U * 128 ? RED_THREADS : 4 * SEG_U * 128];
  __shared__ double cs[2 * K];
  const SegBlock sb = blk[blockIdx.x];
  const int2 r = inst_blk[sb.inst];
  instance_sums<2 * K>(part_in, r.x, r.y, red, cs);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[1] = {0};
  for (int64_t t = sb.lo; t < sb.hi; t += SEG_TILE) {
    double vr[KW][SEG_U], vi[KW][SEG_U], wr[SEG_U], wi[SEG_U];
    load_tile<K, KW>(V, ld, N, t + lane, sb.hi, wv, vr, vi);
    tile_update<K, KW>(w, N, t + lane, sb.hi, wv, lane, cs, vr, vi, red, wr, wi);
    if (wv == 0) {
#pragma unroll
      for (int u = 0; u < SEG_U; ++u) {
        const int64_t x = t + lane + 64 * u;
        if (x < sb.hi) {
          w[x] = wr[u];
          w[N + x] = wi[u];
        }
        acc[0] += wr[u] * wr[u] + wi[u] * wi[u];
      }
    }
  }
  // wave 0 holds the sums; one value per workgroup
  wave_sum_all<1>(acc);
  if (threadIdx.x == 0) part_out[blockIdx.x] = acc[0];
}

// nrm2 = the instance's sum of part_in; beta_j = sqrt(nrm2); scale_j =
// 1 / beta_j unless j >= kmax_i - 1, beta_j <= tol * max(1, |alpha_0|) or
// beta_j is not finite (then 0); dst = w * scale_j when dst is set.  The
// instance's first workgroup stores nrm2, beta_j and scale_j in its scalar
// block sc + inst * S.
__global__ __launch_bounds__(RED_THREADS) void seg_cgs_next_kernel(
    const double* __restrict__ part_in, const double* __restrict__ w, double* __restrict__ dst,
    int64_t N, const SegBlock* __restrict__ blk, const int2* __restrict__ inst_blk,
    double* __restrict__ sc, int S, int nrm2_slot, int alpha0_slot, int beta_slot,
    int scale_slot, double tol, int j, const int* __restrict__ kmax) {
  __shared__ double red[RED_THREADS];
  __shared__ double tot[1];
  const SegBlock sb = blk[blockIdx.x];
  const int2 r = inst_blk[sb.inst];
  instance_sums<1>(part_in, r.x, r.y, red, tot);
  double* si = sc + (size_t)sb.inst * S;
  const double n2 = tot[0];
  const double b = sqrt(n2);
  const double thr = tol * fmax(1.0, fabs(si[alpha0_slot]));
  const double f = (j < kmax[sb.inst] - 1 && b > thr && b < INFINITY) ? 1.0 / b : 0.0;
  if (blockIdx.x == r.x && threadIdx.x == 0) {
    si[nrm2_slot] = n2;
    si[beta_slot] = b;
    si[scale_slot] = f;
  }
  if (!dst) return;
  for (int64_t x = sb.lo + threadIdx.x; x < sb.hi; x += RED_THREADS) {
    dst[x] = w[x] * f;
    dst[N + x] = w[N + x] * f;
  }
}

// K = 1 .. 32 dispatch
#define TNT_K_CASES(M) \
  M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16) \
  M(17) M(18) M(19) M(20) M(21) M(22) M(23) M(24) M(25) M(26) M(27) M(28) M(29) M(30) M(31) M(32)

// Smallest basis size at which each pass takes the waves form (measured on
// a 2.9M-entry vector: dot 5.5 vs 5.8 TB/s at K = 15; update-and-dot 2.9 vs
// 3.5 TB/s at K = 10; update-and-norm 3.5 vs 3.6 TB/s at K = 15).
constexpr int kDotWavesFrom = 12, kUpdateDotWavesFrom = 8, kUpdateNormWavesFrom = 12;

void launch_seg_cgs_dot(const double* V, int64_t ld, int k, const double* w, int64_t N,
                        const SegBlock* blk, int nblk, double* part, hipStream_t s) {
  switch (k) {
#define TNT_CASE(KK)                                                                              \
  case KK:                                                                                        \
    if constexpr (KK >= kDotWavesFrom)                                                            \
      hipLaunchKernelGGL(seg_cgs_dot_waves<KK>, dim3(nblk), dim3(RED_THREADS), 0, s, V, ld,       \
                         w, N, blk, part);                                                        \
    else                                                                                          \
      hipLaunchKernelGGL(seg_cgs_dot_lanes<KK>, dim3(nblk), dim3(RED_THREADS), 0, s, V, ld,       \
                         w, N, blk, part);                                                        \
    break;
    TNT_K_CASES(TNT_CASE)
#undef TNT_CASE
    default: break;
  }
}

void launch_seg_cgs_update_dot(const double* V, int64_t ld, int k, const double* part_in,
                               double* w, int64_t N, const SegBlock* blk, const int2* inst_blk,
                               int nblk, double* part_out, double* pair_dst, int S,
                               hipStream_t s) {
  switch (k) {
#define TNT_CASE(KK)                                                                              \
  case KK:                                                                                        \
    if constexpr (KK >= kUpdateDotWavesFrom)                                                      \
      hipLaunchKernelGGL(seg_cgs_update_dot_waves<KK>, dim3(nblk), dim3(RED_THREADS), 0, s,       \
                         V, ld, part_in, w, N, blk, inst_blk, part_out, pair_dst, S);             \
    else                                                                                          \
      hipLaunchKernelGGL(seg_cgs_update_dot_lanes<KK>, dim3(nblk), dim3(RED_THREADS), 0, s,       \
                         V, ld, part_in, w, N, blk, inst_blk, part_out, pair_dst, S);             \
    break;
    TNT_K_CASES(TNT_CASE)
#undef TNT_CASE
    default: break;
  }
}

void launch_seg_cgs_update_norm(const double* V, int64_t ld, int k, const double* part_in,
                                double* w, int64_t N, const SegBlock* blk, const int2* inst_blk,
                                int nblk, double* part_out, hipStream_t s) {
  switch (k) {
#define TNT_CASE(KK)                                                                              \
  case KK:                                                                                        \
    if constexpr (KK >= kUpdateNormWavesFrom)                                                     \
      hipLaunchKernelGGL(seg_cgs_update_norm_waves<KK>, dim3(nblk), dim3(RED_THREADS), 0, s,      \
                         V, ld, part_in, w, N, blk, inst_blk, part_out);                          \
    else                                                                                          \
      hipLaunchKernelGGL(seg_cgs_update_norm_lanes<KK>, dim3(nblk), dim3(RED_THREADS), 0, s,      \
                         V, ld, part_in, w, N, blk, inst_blk, part_out);                          \
    break;
    TNT_K_CASES(TNT_CASE)
#undef TNT_CASE
    default: break;
  }
}
#undef TNT_K_CASES

void launch_seg_cgs_next(const double* part_in, const double* w, double* dst, int64_t N,
                         const SegBlock* blk, const int2* inst_blk, int nblk, double* sc, int S,
                         int nrm2_slot, int alpha0_slot, int beta_slot, int scale_slot, double tol,
                         int j, const int* kmax, hipStream_t s) {
  hipLaunchKernelGGL(seg_cgs_next_kernel, dim3(nblk), dim3(RED_THREADS), 0, s, part_in, w, dst, N,
                     blk, inst_blk, sc, S, nrm2_slot, alpha0_slot, beta_slot, scale_slot, tol, j,
                     kmax);
}

// Gather / scatter of contiguous runs between separate buffers and a batch
// buffer: dst[i] = src[i] for each task's `count` doubles (one task per
// workgroup row, chunks of the run per workgroup column).
__global__ __launch_bounds__(256) void copy_runs_kernel(const CopyRun* __restrict__ runs) {
  const CopyRun r = runs[blockIdx.y];
  const int64_t chunk = (int64_t)gridDim.x * 256;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < r.count; i += chunk)
    r.dst[i] = r.src[i];
}

void launch_copy_runs(const CopyRun* runs, int nruns, int64_t max_count, hipStream_t s) {
  if (nruns <= 0 || max_count <= 0) return;
  int64_t gx = (max_count + 255) / 256;
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(copy_runs_kernel, dim3((unsigned)gx, nruns), dim3(256), 0, s, runs);
}

}  // namespace tnt
