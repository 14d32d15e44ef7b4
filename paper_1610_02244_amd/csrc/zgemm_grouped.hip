// Grouped FP64 complex GEMM over interleaved, column-major operands: one
// launch computes the 64 x 64 output tiles of many independent products
//   C = op(A) B   or   C -= op(A) B,   op(A) = A or A^H,
// as used by the deflated SVD's per-sector products (re-orthogonalisation of
// a cluster against the resolved directions, the cluster's Gram matrix, the
// products with the cluster's eigenvectors and the kept singular vectors).
// One library call per sector and product made those steps bound by the
// host's enqueue rate when hundreds of sectors are active; here the host
// lists the tiles and one launch runs them all.
//
// Each workgroup (256 threads) owns one tile: K runs in chunks of 16 through
// LDS (64 x 16 of op(A), 16 x 64 of B), each thread accumulates a 4 x 4
// block (rows tr + 16 a, columns tc + 16 b) in registers, with K summed in
// increasing order, so results do not depend on the grouping.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace tnt {
namespace {

constexpr int kT = 64;   // tile rows and columns
constexpr int kK = 16;   // K chunk

__global__ __launch_bounds__(256) void zgemm_grouped_kernel(const ZTask* __restrict__ tasks) {
  __shared__ double2 As[kK][kT + 1];
  __shared__ double2 Bs[kK][kT + 1];
  const ZTask t = tasks[blockIdx.x];
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const double2* __restrict__ A = reinterpret_cast<const double2*>(t.A);
  const double2* __restrict__ B = reinterpret_cast<const double2*>(t.B);
  double2* __restrict__ C = reinterpret_cast<double2*>(t.C);
  const double2 zero = make_double2(0.0, 0.0);
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero;
  for (int p0 = 0; p0 < t.k; p0 += kK) {
    // op(A) tile: rows i0 .. i0 + 63, K columns p0 .. p0 + 15
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int i, p;
      double2 v = zero;
      if (t.opa == 0) {  // A(i, p) at A[i + p lda]: threads along i
        i = tid & 63;
        p = (tid >> 6) + 4 * q;
        const int gi = t.i0 + i, gp = p0 + p;
        if (gi < t.m && gp < t.k) v = A[gi + (int64_t)gp * t.lda];
      } else {  // conj(A(p, i)) at A[p + i lda]: threads along p
        p = tid & 15;
        i = (tid >> 4) + 16 * q;
        const int gi = t.i0 + i, gp = p0 + p;
        if (gi < t.m && gp < t.k) {
          v = A[gp + (int64_t)gi * t.lda];
          v.y = -v.y;
        }
      }
      As[p][i] = v;
    }
    // B tile: K rows p0 .. p0 + 15, columns j0 .. j0 + 63 (threads along p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = tid & 15, j = (tid >> 4) + 16 * q;
      const int gp = p0 + p, gj = t.j0 + j;
      Bs[p][j] = gp < t.k && gj < t.n ? B[gp + (int64_t)gj * t.ldb] : zero;
    }
    __syncthreads();
#pragma unroll 4
    for (int p = 0; p < kK; ++p) {
      double2 av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[p][tr + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[p][tc + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b].x = fma(av[a].x, bv[b].x, acc[a][b].x);
          acc[a][b].x = fma(-av[a].y, bv[b].y, acc[a][b].x);
          acc[a][b].y = fma(av[a].x, bv[b].y, acc[a][b].y);
          acc[a][b].y = fma(av[a].y, bv[b].x, acc[a][b].y);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int gi = t.i0 + tr + 16 * a;
    if (gi >= t.m) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int gj = t.j0 + tc + 16 * b;
      if (gj >= t.n) continue;
      double2* c = C + gi + (int64_t)gj * t.ldc;
      if (t.sub) {
        const double2 o = *c;
        *c = make_double2(o.x - acc[a][b].x, o.y - acc[a][b].y);
      } else {
        *c = acc[a][b];
      }
    }
  }
}

}  // namespace

void launch_zgemm_grouped(const ZTask* tasks, int ntask, hipStream_t s) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(zgemm_grouped_kernel, dim3(ntask), dim3(256), 0, s, tasks);
}

}  // namespace tnt
