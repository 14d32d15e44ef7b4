// Eigen-decomposition of small Hermitian matrices (the Gram matrices of the
// small sectors of an SVD) by cyclic Jacobi rotations, one workgroup per
// matrix with the matrix and its eigenvector matrix resident in LDS.
//
// A batched library eigensolve of small matrices (order <= 64) costs about
// one small launch chain per matrix (its run time grows linearly with the
// batch), so the sectors of order <= 32 are taken out of the library calls
// and solved here in a single launch that runs beside them.  (At order 64
// the LDS traffic of the rotations makes this kernel take a few
// milliseconds, longer than the library's chain for a typical bond.)
//
// Method (two-sided cyclic Jacobi, parallel round-robin ordering): each
// sweep visits every index pair once in n' - 1 rounds of n'/2 disjoint
// pairs (n' = n rounded up to even; the extra index is idle).  For a pair
// (p, q) with a = A_pp, d = A_qq, b = A_pq = |b| u:
//   tau = (d - a) / (2|b|),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1 / sqrt(1 + t^2),   s = t c,
//   J = [[c, s u], [-s conj(u), c]] on columns (p, q),
// which is diag(1, conj u) R diag(1, u) with R the real rotation that
// diagonalises the real symmetric matrix [[a, |b|], [|b|, d]]; so
// J^H A J has a zero (p, q) entry.  A <- J^H A J (columns, then rows) and
// V <- V J.  An entry below the rounding of its diagonal pair,
// |b| <= eps sqrt(|a d|), or below eps times the sum of |A_ii|, is set to
// zero instead; a sweep without any rotation ends the iteration.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace tnt {

constexpr int JAC_THREADS = 256;
constexpr int JAC_MAX_SWEEPS = 40;

__device__ inline double2 cmul(double2 x, double2 y) {
  return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}
__device__ inline double2 cconj(double2 x) { return make_double2(x.x, -x.y); }
__device__ inline double2 cscale(double f, double2 x) { return make_double2(f * x.x, f * x.y); }
__device__ inline double2 cadd(double2 x, double2 y) { return make_double2(x.x + y.x, x.y + y.y); }
__device__ inline double2 csub(double2 x, double2 y) { return make_double2(x.x - y.x, x.y - y.y); }

// player at position i of round k in the round-robin of m (even) players
__device__ inline int rr_player(int i, int k, int m) {
  return i == 0 ? 0 : (i - 1 + k) % (m - 1) + 1;
}

// NMAX: the largest order the instance holds in LDS (2 NMAX^2 complex)
template <int NMAX>
__global__ __launch_bounds__(JAC_THREADS) void jacobi_eig_kernel(const PadTask* __restrict__ tasks,
                                                                 int* __restrict__ info) {
  __shared__ double2 A[NMAX * NMAX];  // column-major: A[c * n + r]
  __shared__ double2 V[NMAX * NMAX];
  __shared__ int pp[NMAX / 2], pq[NMAX / 2];
  __shared__ double rc[NMAX / 2], rs[NMAX / 2];
  __shared__ double2 ru[NMAX / 2];
  __shared__ double red[JAC_THREADS / 64];
  __shared__ int rotations;
  const PadTask t = tasks[blockIdx.x];
  const int n = t.n;
  const int tid = threadIdx.x;
  if (n > NMAX || n < 0) {  // does not fit this instance (the host never asks)
    if (tid == 0) info[blockIdx.x] = 2;
    return;
  }
  const double* src = t.z + 2 * t.src_off;
  // the upper triangle (column-major) defines the matrix, as for the
  // library eigensolver; the diagonal is taken as real
  for (int e = tid; e < n * n; e += JAC_THREADS) {
    const int r = e % n, c = e / n;
    double2 v;
    if (r < c) v = make_double2(src[2 * e], src[2 * e + 1]);
    else if (r == c) v = make_double2(src[2 * e], 0.0);
    else v = make_double2(src[2 * (r * n + c)], -src[2 * (r * n + c) + 1]);
    A[e] = v;
    V[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  // sum of |A_ii| (the trace of a Gram matrix) sets the absolute floor
  double dsum = 0;
  for (int i = tid; i < n; i += JAC_THREADS) dsum += fabs(src[2 * (i * n + i)]);
  for (int o = 32; o > 0; o >>= 1) dsum += __shfl_xor(dsum, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = dsum;
  __syncthreads();
  dsum = 0;
  for (int w = 0; w < JAC_THREADS / 64; ++w) dsum += red[w];
  const int m = n + (n & 1);  // even number of players; index n is idle when n is odd
  const int npair = m / 2;
  const double eps = 1.1102230246251565e-16;  // unit roundoff of double
  // below this an off-diagonal entry is dropped whatever its diagonal pair:
  // changes the eigenvalues by at most about eps times the largest
  const double floor_abs = eps * dsum;
  int converged = n <= 1;
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS && !converged; ++sweep) {
    if (tid == 0) rotations = 0;
    __syncthreads();
    for (int k = 0; k < m - 1; ++k) {
      // 1. rotation parameters of the round's pairs
      if (tid < npair) {
        int p = rr_player(tid, k, m), q = rr_player(m - 1 - tid, k, m);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        double c = 1.0, s = 0.0;
        double2 u = make_double2(1.0, 0.0);
        if (q < n) {
          const double a = A[p * n + p].x, d = A[q * n + q].x;
          const double2 b = A[q * n + p];
          const double ab = hypot(b.x, b.y);
          if (ab > floor_abs && ab > eps * sqrt(fabs(a) * fabs(d))) {
            const double tau = (d - a) / (2.0 * ab);
            const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            u = make_double2(b.x / ab, b.y / ab);
            atomicAdd(&rotations, 1);
          } else {
            A[q * n + p] = make_double2(0.0, 0.0);
            A[p * n + q] = make_double2(0.0, 0.0);
          }
        }
        pp[tid] = p;
        pq[tid] = q;
        rc[tid] = c;
        rs[tid] = s;
        ru[tid] = u;
      }
      __syncthreads();
      // 2. columns: A <- A J, V <- V J
      for (int e = tid; e < npair * n; e += JAC_THREADS) {
        const int i = e / n, r = e % n;
        const double s = rs[i];
        if (s == 0.0) continue;
        const int p = pp[i], q = pq[i];
        const double c = rc[i];
        const double2 u = ru[i];
        const double2 ap = A[p * n + r], aq = A[q * n + r];
        A[p * n + r] = csub(cscale(c, ap), cscale(s, cmul(cconj(u), aq)));
        A[q * n + r] = cadd(cscale(s, cmul(u, ap)), cscale(c, aq));
        const double2 vp = V[p * n + r], vq = V[q * n + r];
        V[p * n + r] = csub(cscale(c, vp), cscale(s, cmul(cconj(u), vq)));
        V[q * n + r] = cadd(cscale(s, cmul(u, vp)), cscale(c, vq));
      }
      __syncthreads();
      // 3. rows: A <- J^H A; the rotated pair's off-diagonal entries are
      //    zero and its diagonal entries real by construction
      for (int e = tid; e < npair * n; e += JAC_THREADS) {
        const int i = e / n, col = e % n;
        const double s = rs[i];
        if (s == 0.0) continue;
        const int p = pp[i], q = pq[i];
        const double c = rc[i];
        const double2 u = ru[i];
        const double2 ap = A[col * n + p], aq = A[col * n + q];
        double2 np_ = csub(cscale(c, ap), cscale(s, cmul(u, aq)));
        double2 nq_ = cadd(cscale(s, cmul(cconj(u), ap)), cscale(c, aq));
        if (col == q) np_ = make_double2(0.0, 0.0);
        if (col == p) nq_ = make_double2(0.0, 0.0);
        if (col == p) np_.y = 0.0;
        if (col == q) nq_.y = 0.0;
        A[col * n + p] = np_;
        A[col * n + q] = nq_;
      }
      __syncthreads();
    }
    converged = rotations == 0;
    __syncthreads();  // every thread has read the count before the next reset
  }
  // ascending order (ties by index) and write back
  double* out = t.z + 2 * t.src_off;
  for (int i = tid; i < n; i += JAC_THREADS) {
    const double li = A[i * n + i].x;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j * n + j].x;
      rank += (lj < li) || (lj == li && j < i);
    }
    t.w[t.w_dst + rank] = li;
    for (int r = 0; r < n; ++r) {
      const double2 v = V[i * n + r];
      out[2 * ((int64_t)rank * n + r)] = v.x;
      out[2 * ((int64_t)rank * n + r) + 1] = v.y;
    }
  }
  if (tid == 0) info[blockIdx.x] = converged ? 0 : 1;
}

void launch_eig_small(const PadTask* t, int ntask, int max_n, int* info, hipStream_t s) {
  if (ntask <= 0) return;
  if (max_n <= 16)
    hipLaunchKernelGGL(jacobi_eig_kernel<16>, dim3(ntask), dim3(JAC_THREADS), 0, s, t, info);
  else
    hipLaunchKernelGGL(jacobi_eig_kernel<EIG_SMALL_MAX>, dim3(ntask), dim3(JAC_THREADS), 0, s, t,
                       info);
}

}  // namespace tnt
