// Kernels of the automatic blocking of a matrix (no known symmetry): the
// pattern of entries above a tolerance, and an index-mapped block copy used
// both to gather the discovered blocks into packed storage and to scatter
// the factors back to the caller's row and column order.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace tnt {

constexpr int AB_THREADS = 256;

__global__ __launch_bounds__(AB_THREADS) void nonzero_mask_kernel(
    const double* __restrict__ re, const double* __restrict__ im, int m, int n, int64_t ld,
    double tol2, unsigned char* __restrict__ mask) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = (int64_t)blockIdx.x * AB_THREADS + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * AB_THREADS) {
    const int64_t i = e / n, j = e % n;
    const double x = re[i * ld + j], y = im[i * ld + j];
    mask[e] = (x * x + y * y > tol2) ? 1 : 0;
  }
}

// one workgroup per (task, row): dst(r, c) = src(r, c), each side addressed
// through an optional row / column index list
__global__ __launch_bounds__(AB_THREADS) void index_copy_kernel(
    const IndexCopyTask* __restrict__ tasks, const int2* __restrict__ rows,
    const int32_t* __restrict__ idx, const double* __restrict__ sre,
    const double* __restrict__ sim, double* __restrict__ dre, double* __restrict__ dim) {
  const int2 tr = rows[blockIdx.x];
  const IndexCopyTask t = tasks[tr.x];
  const int r = tr.y;
  const int64_t sr = t.src_ridx >= 0 ? idx[t.src_ridx + r] : r;
  const int64_t dr = t.dst_ridx >= 0 ? idx[t.dst_ridx + r] : t.dst_rbase + r;
  for (int col = threadIdx.x; col < t.cols; col += AB_THREADS) {
    const int64_t sc = t.src_cidx >= 0 ? idx[t.src_cidx + col] : col;
    const int64_t dc = t.dst_cidx >= 0 ? idx[t.dst_cidx + col] : t.dst_cbase + col;
    double x = sre[t.src_off + sr * t.src_ld + sc];
    double y = sim[t.src_off + sr * t.src_ld + sc];
    if (x * x + y * y <= t.tol2) x = y = 0.0;
    dre[t.dst_off + dr * t.dst_ld + dc] = x;
    dim[t.dst_off + dr * t.dst_ld + dc] = y;
  }
}

void launch_nonzero_mask(const double* re, const double* im, int m, int n, int64_t ld,
                         double tol, unsigned char* mask, hipStream_t s) {
  const int64_t total = (int64_t)m * n;
  if (total <= 0) return;
  const int64_t want = (total + AB_THREADS - 1) / AB_THREADS;
  const int grid = (int)(want < 8192 ? want : 8192);
  nonzero_mask_kernel<<<grid, AB_THREADS, 0, s>>>(re, im, m, n, ld, tol * tol, mask);
}

void launch_index_copy(const IndexCopyTask* tasks, const int2* rows, int nrows,
                       const int32_t* idx, const double* sre, const double* sim, double* dre,
                       double* dim, hipStream_t s) {
  if (nrows <= 0) return;
  index_copy_kernel<<<nrows, AB_THREADS, 0, s>>>(tasks, rows, idx, sre, sim, dre, dim);
}

}  // namespace tnt
