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

// partial[b * 2k + 2i + {0,1}] = block b's share of <V_i, w> (re, im)
__global__ __launch_bounds__(RED_THREADS) void seg_multidot_kernel(
    const double* __restrict__ V, int64_t ld, int k, const double* __restrict__ w, int64_t N,
    const SegBlock* __restrict__ blk, double* __restrict__ partial) {
  __shared__ double sh[4];
  const SegBlock sb = blk[blockIdx.x];
  for (int i0 = 0; i0 < k; i0 += 8) {
    double accr[8], acci[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) { accr[u] = 0; acci[u] = 0; }
    for (int64_t x = sb.lo + threadIdx.x; x < sb.hi; x += RED_THREADS) {
      const double wr = w[x], wi = w[N + x];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (i0 + u < k) {
          const double vr = V[(i0 + u) * ld + x], vi = V[(i0 + u) * ld + N + x];
          accr[u] += vr * wr + vi * wi;
          acci[u] += vr * wi - vi * wr;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (i0 + u < k) {
        const double r = seg_block_sum(accr[u], sh);
        const double m = seg_block_sum(acci[u], sh);
        if (threadIdx.x == 0) {
          partial[blockIdx.x * 2 * k + 2 * (i0 + u)] = r;
          partial[blockIdx.x * 2 * k + 2 * (i0 + u) + 1] = m;
        }
      }
    }
  }
}

void launch_seg_multidot(const double* V, int64_t ld, int k, const double* w, int64_t N,
                         const SegBlock* blk, int nblk, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(seg_multidot_kernel, dim3(nblk), dim3(RED_THREADS), 0, s, V, ld, k, w, N,
                     blk, partial);
}

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

// w -= sum_i c_{inst,i} V_i (complex c at c + inst * c_stride), then |w|^2
// partials per block
__global__ __launch_bounds__(RED_THREADS) void seg_multiaxpy_norm_kernel(
    const double* __restrict__ V, int64_t ld, int k, const double* __restrict__ c, int c_stride,
    double* __restrict__ w, int64_t N, const SegBlock* __restrict__ blk,
    double* __restrict__ nrm_partial) {
  __shared__ double sh[4];
  __shared__ double cs[2 * SEG_MAXK];
  const SegBlock sb = blk[blockIdx.x];
  if (threadIdx.x < 2 * k) cs[threadIdx.x] = c[sb.inst * c_stride + threadIdx.x];
  __syncthreads();
  double acc = 0;
  for (int64_t x = sb.lo + threadIdx.x; x < sb.hi; x += RED_THREADS) {
    double wr = w[x], wi = w[N + x];
    for (int i = 0; i < k; ++i) {
      const double vr = V[i * ld + x], vi = V[i * ld + N + x];
      const double cr = cs[2 * i], ci = cs[2 * i + 1];
      wr -= cr * vr - ci * vi;
      wi -= cr * vi + ci * vr;
    }
    w[x] = wr;
    w[N + x] = wi;
    acc += wr * wr + wi * wi;
  }
  const double r = seg_block_sum(acc, sh);
  if (threadIdx.x == 0) nrm_partial[blockIdx.x] = r;
}

void launch_seg_multiaxpy_norm(const double* V, int64_t ld, int k, const double* c,
                               int c_stride, double* w, int64_t N, const SegBlock* blk,
                               int nblk, double* nrm_partial, hipStream_t s) {
  hipLaunchKernelGGL(seg_multiaxpy_norm_kernel, dim3(nblk), dim3(RED_THREADS), 0, s, V, ld, k, c,
                     c_stride, w, N, blk, nrm_partial);
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

// Per instance (one thread each): beta = sqrt(|w|^2); scale = 1 / beta when
// step j is not the instance's last (j < kmax_i - 1) and beta is above the
// breakdown tolerance tol * max(1, |alpha_0|) and finite, else 0.
__global__ void seg_lanczos_beta_kernel(const double* __restrict__ nrm2, int nrm_stride,
                                        const double* __restrict__ alpha0, int a_stride,
                                        double tol, int j, const int* __restrict__ kmax,
                                        double* __restrict__ beta, int b_stride,
                                        double* __restrict__ scale, int s_stride, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  const double b = sqrt(nrm2[i * nrm_stride]);
  beta[i * b_stride] = b;
  const double thr = tol * fmax(1.0, fabs(alpha0[i * a_stride]));
  scale[i * s_stride] = (j < kmax[i] - 1 && b > thr && b < INFINITY) ? 1.0 / b : 0.0;
}

void launch_seg_lanczos_beta(const double* nrm2, int nrm_stride, const double* alpha0,
                             int a_stride, double tol, int j, const int* kmax, double* beta,
                             int b_stride, double* scale, int s_stride, int ninst,
                             hipStream_t s) {
  hipLaunchKernelGGL(seg_lanczos_beta_kernel, dim3((ninst + 63) / 64), dim3(64), 0, s, nrm2,
                     nrm_stride, alpha0, a_stride, tol, j, kmax, beta, b_stride, scale, s_stride,
                     ninst);
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
