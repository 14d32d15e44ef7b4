// Householder reduction of a batch of Hermitian matrices to real symmetric
// tridiagonal form, for the Gram eigenproblems of the SVD (the library
// eigensolver's reduction is a chain of five to six launches per column;
// this one is two).  Used for the padded orders the context selects
// (tnt_ctx_set_eig_reduction, off by default): the library offers its
// tridiagonal divide and conquer and back-transformation only one matrix per
// call, and those calls cost more than the launches saved here.
//
// Convention (LAPACK's lower form): Q = H_0 H_1 ... H_{n-2}, H_k = I - tau_k
// v_k v_k^H with v_k zero above row k+1, v_k(k+1) = 1 and v_k(k+2:) stored in
// A(k+2:, k); Q^H A Q = T with diagonal d and real off-diagonal e.  The
// library's back-transformation (unmtr, lower) and tridiagonal divide and
// conquer (stedc) take these arrays as they stand.
//
// Panels of TRD_NB columns (the blocked reduction of Dongarra, Sorensen and
// Hammarling): inside a panel the matrix is not updated; column k is first
// corrected by the panel's earlier reflectors through
//   A(k:, k) -= V(k:, :) W(k, :)^H + W(k:, :) V(k, :)^H,
// then its reflector is generated, and
//   w = tau (A v - V (W^H v) - W (V^H v)),  w += -(tau / 2) (w^H v) v
// is the panel's next W column.  After the panel the trailing block takes
// A -= V W^H + W V^H in one complex GEMM (the host side).
//
// Matrices are stored in full (both triangles, column-major, ld = np), so
// the product A v over the trailing block reads whole columns (coalesced)
// and the trailing update writes both triangles.
//
// Per column: trd_column_kernel (one workgroup per matrix: finishes the
// previous W column, corrects column k, makes reflector k) and
// trd_gemv_kernel (many workgroups per matrix: the trailing-block product
// A v in 64 x 64 tiles and the dot products W^H v, V^H v per 64 rows, as
// partial sums that the next column kernel adds in a fixed order).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace tnt {
namespace {

__device__ inline double2 zmul(double2 x, double2 y) {
  return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}
// conj(x) * y
__device__ inline double2 zcmul(double2 x, double2 y) {
  return make_double2(x.x * y.x + x.y * y.y, x.x * y.y - x.y * y.x);
}
__device__ inline double2 zadd(double2 x, double2 y) { return make_double2(x.x + y.x, x.y + y.y); }
__device__ inline double2 zsub(double2 x, double2 y) { return make_double2(x.x - y.x, x.y - y.y); }

constexpr int kColThreads = 1024;
constexpr int kColRows = TRD_MAX_N / kColThreads;  // rows per thread
constexpr int kTile = 64;                            // rows and columns of a gemv tile

__device__ inline double2 wave_sum2(double2 v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

// sum over the block of one complex value per thread, returned to all threads
// (fixed order: lanes by butterfly, waves in index order)
template <int NT>
__device__ double2 block_sum2(double2 v, double2* sh) {
  v = wave_sum2(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();  // sh may still be read by a previous call
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  for (int q = 0; q < NT / 64; ++q) s = zadd(s, sh[q]);
  return s;
}

__global__ __launch_bounds__(kColThreads) void trd_column_kernel(TrdBatch b, int j0, int nbp,
                                                                  int i, int do_col) {
  __shared__ double2 red[kColThreads / 64];
  __shared__ double2 tdot[2 * TRD_NB];
  __shared__ double2 vk[TRD_NB], wk[TRD_NB];
  __shared__ double2 alpha_bc, wk_last;
  const int np = b.np, k = j0 + i, tid = threadIdx.x;
  const int64_t mb = blockIdx.x;
  double2* __restrict__ A = b.A + mb * b.sA;
  double2* __restrict__ X = b.X + mb * b.sX;
  const double2* __restrict__ yp = b.yp + mb * b.sY;
  const double2* __restrict__ tp = b.tp + mb * b.sT;
  const int64_t ld = np;
  const int m = np - k, nt = (m + kTile - 1) / kTile;
  const int nd = i > 0 ? i - 1 : 0;  // finished W columns before the one being finished
  const double2 zero = make_double2(0.0, 0.0);
  // (W^H v)_j and (V^H v)_j of reflector k-1 from the per-64-row partial sums:
  // 16 threads per value, then a fixed butterfly over the 16
  if (i > 0) {
    const int q = tid >> 4, sub = tid & 15;
    double2 acc = zero;
    if (q < 2 * nd)
      for (int rb = sub; rb < nt; rb += 16) acc = zadd(acc, tp[rb * (2 * TRD_NB) + q]);
    for (int o = 8; o > 0; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, 64);
      acc.y += __shfl_xor(acc.y, o, 64);
    }
    if (sub == 0 && q < 2 * nd) tdot[q] = acc;  // q < nd: W^H v; else V^H v
  }
  // row k of the panel's finished columns
  if (do_col)
    for (int j = tid; j < nd; j += kColThreads) {
      vk[j] = X[k + j * ld];
      wk[j] = X[k + (nbp + j) * ld];
    }
  __syncthreads();
  double2 wv[kColRows], vr[kColRows], a[kColRows];
  const double2 tau = i > 0 ? b.tau[mb * b.stau + k - 1] : zero;
  double2 part = zero;
#pragma unroll
  for (int u = 0; u < kColRows; ++u) {
    const int r = k + tid + u * kColThreads;
    wv[u] = vr[u] = a[u] = zero;
    if (r >= np) continue;
    double2 y = zero, x = do_col ? A[r + k * ld] : zero;
    if (i > 0) {
      vr[u] = X[r + (i - 1) * ld];
      // partial products of A v, eight loads in flight, summed in chunk order
      int c = 0;
      for (; c + 8 <= nt; c += 8) {
        double2 t[8];
#pragma unroll
        for (int h = 0; h < 8; ++h) t[h] = yp[(c + h) * ld + r];
#pragma unroll
        for (int h = 0; h < 8; ++h) y = zadd(y, t[h]);
      }
      for (; c < nt; ++c) y = zadd(y, yp[c * ld + r]);
    }
    // corrections by the finished columns j < nd, four columns per batch
    int j = 0;
    for (; j + 4 <= nd; j += 4) {
      double2 vj[4], wj[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        vj[h] = X[r + (j + h) * ld];
        wj[h] = X[r + (nbp + j + h) * ld];
      }
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        y = zsub(y, zmul(vj[h], tdot[j + h]));
        y = zsub(y, zmul(wj[h], tdot[nd + j + h]));
        if (do_col) {
          x = zsub(x, zmul(vj[h], make_double2(wk[j + h].x, -wk[j + h].y)));
          x = zsub(x, zmul(wj[h], make_double2(vk[j + h].x, -vk[j + h].y)));
        }
      }
    }
    for (; j < nd; ++j) {
      const double2 vj = X[r + j * ld], wj = X[r + (nbp + j) * ld];
      y = zsub(y, zmul(vj, tdot[j]));
      y = zsub(y, zmul(wj, tdot[nd + j]));
      if (do_col) {
        x = zsub(x, zmul(vj, make_double2(wk[j].x, -wk[j].y)));
        x = zsub(x, zmul(wj, make_double2(vk[j].x, -vk[j].y)));
      }
    }
    a[u] = x;
    if (i > 0) {
      wv[u] = zmul(tau, y);
      part = zadd(part, zcmul(wv[u], vr[u]));
    }
  }
  if (i > 0) {
    // finish W(:, i-1): w += -(tau / 2) (w^H v) v over rows k..
    const double2 s = block_sum2<kColThreads>(part, red);
    const double2 al = zmul(make_double2(-0.5 * tau.x, -0.5 * tau.y), s);
#pragma unroll
    for (int u = 0; u < kColRows; ++u) {
      const int r = k + tid + u * kColThreads;
      if (r >= np) continue;
      wv[u] = zadd(wv[u], zmul(al, vr[u]));
      X[r + (nbp + i - 1) * ld] = wv[u];
    }
    if (!do_col) return;
    if (tid == 0) wk_last = wv[0];  // row k
    __syncthreads();
    // the finished column's own term: V(k, i-1) = 1, W(k, i-1) = w(k)
    const double2 wc = make_double2(wk_last.x, -wk_last.y);
#pragma unroll
    for (int u = 0; u < kColRows; ++u) {
      const int r = k + tid + u * kColThreads;
      if (r >= np) continue;
      a[u] = zsub(a[u], zmul(vr[u], wc));
      a[u] = zsub(a[u], wv[u]);
    }
  }
  double xs = 0.0;
#pragma unroll
  for (int u = 0; u < kColRows; ++u) {
    const int r = k + tid + u * kColThreads;
    if (r >= np) continue;
    if (r == k) a[u].y = 0.0;
    if (r == k + 1) alpha_bc = a[u];
    if (r >= k + 2) xs += a[u].x * a[u].x + a[u].y * a[u].y;
  }
  if (tid == 0) b.d[mb * b.sd + k] = a[0].x;
  if (k == np - 1) {
    if (tid == 0) A[k + k * ld] = a[0];
    return;
  }
  const double xn2 = block_sum2<kColThreads>(make_double2(xs, 0.0), red).x;  // syncs alpha_bc
  const double2 al = alpha_bc;
  double2 tk = zero, scal = make_double2(1.0, 0.0);
  double beta = al.x;
  if (xn2 != 0.0 || al.y != 0.0) {
    beta = -copysign(sqrt(al.x * al.x + al.y * al.y + xn2), al.x);
    tk = make_double2((beta - al.x) / beta, -al.y / beta);
    const double2 den = make_double2(al.x - beta, al.y);  // scal = 1 / (alpha - beta)
    const double dd = den.x * den.x + den.y * den.y;
    scal = make_double2(den.x / dd, -den.y / dd);
  }
#pragma unroll
  for (int u = 0; u < kColRows; ++u) {
    const int r = k + tid + u * kColThreads;
    if (r >= np) continue;
    if (r == k) {
      A[r + k * ld] = a[u];
      continue;
    }
    const double2 v = r == k + 1 ? make_double2(1.0, 0.0) : zmul(a[u], scal);
    A[r + k * ld] = v;
    X[r + i * ld] = v;
    X[r + (2 * nbp + i) * ld] = v;
  }
  if (tid == 0) {
    b.e[mb * b.se + k] = beta;
    b.tau[mb * b.stau + k] = tk;
  }
}

// Trailing-block product for reflector k (in-panel index i): tiles of 64 rows
// x 64 columns of A(k+1:, k+1:) v, then, in the last nt workgroups, the dot
// products W(:, j)^H v and V(:, j)^H v (j < i) over 64 rows each.
__global__ __launch_bounds__(256) void trd_gemv_kernel(TrdBatch b, int k, int i, int nbp) {
  __shared__ double2 sh[4][kTile];
  __shared__ double2 sv[kTile];
  const int np = b.np, base = k + 1, m = np - base, nt = (m + kTile - 1) / kTile;
  const int64_t mb = blockIdx.y;
  const double2* __restrict__ A = b.A + mb * b.sA;
  const double2* __restrict__ X = b.X + mb * b.sX;
  const int64_t ld = np;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int blk = blockIdx.x;
  const double2 zero = make_double2(0.0, 0.0);
  if (blk < nt * nt) {
    const int rb = blk % nt, cb = blk / nt;
    const int r = base + rb * kTile + lane;
    const int cbase = base + cb * kTile;
    if (threadIdx.x < kTile) {
      const int c = cbase + threadIdx.x;
      sv[threadIdx.x] = c < np ? X[c + i * ld] : zero;
    }
    __syncthreads();
    double2 acc = zero;
    if (r < np) {
      const int c0 = cbase + wv * (kTile / 4);
#pragma unroll
      for (int h0 = 0; h0 < kTile / 4; h0 += 8) {
        double2 t[8];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const int c = c0 + h0 + h;
          t[h] = c < np ? A[r + c * ld] : zero;
        }
#pragma unroll
        for (int h = 0; h < 8; ++h) acc = zadd(acc, zmul(t[h], sv[wv * (kTile / 4) + h0 + h]));
      }
    }
    sh[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && r < np) {
      double2 s = sh[0][lane];
      for (int q = 1; q < 4; ++q) s = zadd(s, sh[q][lane]);
      b.yp[mb * b.sY + cb * ld + r] = s;
    }
    return;
  }
  const int rb = blk - nt * nt;
  if (rb >= nt) return;
  const int r = base + rb * kTile + lane;
  const double2 v = r < np ? X[r + i * ld] : zero;
  double2* __restrict__ tp = b.tp + mb * b.sT + rb * (2 * TRD_NB);
  for (int q = wv; q < 2 * i; q += 4) {
    const int col = q < i ? nbp + q : q - i;  // W columns first, then V columns
    const double2 x = r < np ? X[r + col * ld] : zero;
    const double2 s = wave_sum2(zcmul(x, v));
    if (lane == 0) tp[q] = s;
  }
}

}  // namespace

void launch_trd_column(const TrdBatch& b, int cnt, int j0, int nbp, int i, int do_col,
                       hipStream_t s) {
  hipLaunchKernelGGL(trd_column_kernel, dim3(cnt), dim3(kColThreads), 0, s, b, j0, nbp, i,
                     do_col);
}

void launch_trd_gemv(const TrdBatch& b, int cnt, int k, int i, int nbp, hipStream_t s) {
  const int m = b.np - k - 1;
  if (m <= 0) return;
  const int nt = (m + kTile - 1) / kTile;
  hipLaunchKernelGGL(trd_gemv_kernel, dim3(nt * nt + nt, cnt), dim3(256), 0, s, b, k, i, nbp);
}

}  // namespace tnt
