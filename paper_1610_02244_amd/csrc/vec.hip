// Bandwidth-bound kernels: sparse MPO slab combinations, precision
// conversions, FP64 Krylov-vector algebra with deterministic two-stage
// reductions, and the gather/scatter between U(1) blocks and the dense
// sector matrices of the SVD.
#include "kernels.h"

namespace tnt {

// ---------------------------------------------------------------------------
// dst slab = sum_t coef_t src_t (one workgroup per COMB_CHUNK elements)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void combine_kernel(const CombTask* __restrict__ tasks,
                                                      const CombTerm* __restrict__ terms,
                                                      const int2* __restrict__ chunks,
                                                      const T* __restrict__ sre,
                                                      const T* __restrict__ sim,
                                                      T* __restrict__ dre, T* __restrict__ dim_) {
  const int2 c = chunks[blockIdx.x];
  const CombTask tk = tasks[c.x];
  const int base = c.y * COMB_CHUNK;
#pragma unroll
  for (int e = 0; e < COMB_CHUNK / 256; ++e) {
    const int i = base + e * 256 + threadIdx.x;
    if (i >= tk.size) break;
    T ar = 0, ai = 0;
    for (int t = 0; t < tk.nterm; ++t) {
      const CombTerm tm = terms[tk.term0 + t];
      const T cf = (T)tm.coef;
      ar += cf * sre[tm.src_off + i];
      ai += cf * sim[tm.src_off + i];
    }
    dre[tk.dst_off + i] = ar;
    dim_[tk.dst_off + i] = ai;
  }
}

void launch_combine(const CombTask* tasks, const CombTerm* terms, const int2* chunks,
                    int32_t nchunks, const void* src_re, const void* src_im, void* dst_re,
                    void* dst_im, ElemType t, hipStream_t s) {
  if (nchunks <= 0) return;
  if (t == ET_F64)
    hipLaunchKernelGGL(combine_kernel<double>, dim3(nchunks), dim3(256), 0, s, tasks, terms,
                       chunks, (const double*)src_re, (const double*)src_im, (double*)dst_re,
                       (double*)dst_im);
  else
    hipLaunchKernelGGL(combine_kernel<float>, dim3(nchunks), dim3(256), 0, s, tasks, terms,
                       chunks, (const float*)src_re, (const float*)src_im, (float*)dst_re,
                       (float*)dst_im);
}

// ---------------------------------------------------------------------------
// conversions and fills
// ---------------------------------------------------------------------------
template <typename S, typename D>
__global__ void convert_kernel(const S* __restrict__ s, D* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (D)s[i];
}

static int grid_for(int64_t n, int threads = 256, int cap = 4096) {
  int64_t g = (n + threads - 1) / threads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

void launch_convert(const void* src, ElemType st, void* dst, ElemType dt, int64_t n,
                    hipStream_t s) {
  if (n <= 0) return;
  const int g = grid_for(n);
  if (st == ET_F64 && dt == ET_F32)
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(g), dim3(256), 0, s,
                       (const double*)src, (float*)dst, n);
  else if (st == ET_F32 && dt == ET_F64)
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(g), dim3(256), 0, s,
                       (const float*)src, (double*)dst, n);
  else if (st == ET_F64)
    hipLaunchKernelGGL((convert_kernel<double, double>), dim3(g), dim3(256), 0, s,
                       (const double*)src, (double*)dst, n);
  else
    hipLaunchKernelGGL((convert_kernel<float, float>), dim3(g), dim3(256), 0, s,
                       (const float*)src, (float*)dst, n);
}

template <typename T>
__global__ void fill_zero_kernel(T* d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = 0;
}

void launch_fill_zero(void* dst, ElemType t, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int g = grid_for(n);
  if (t == ET_F64)
    hipLaunchKernelGGL(fill_zero_kernel<double>, dim3(g), dim3(256), 0, s, (double*)dst, n);
  else
    hipLaunchKernelGGL(fill_zero_kernel<float>, dim3(g), dim3(256), 0, s, (float*)dst, n);
}

__global__ void scale_dev_kernel(double* x, int64_t n, const double* sc) {
  const double f = *sc;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= f;
}
void launch_scale(double* x, int64_t n, const double* scale_dev, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_dev_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, scale_dev);
}
__global__ void scale_host_kernel(double* x, int64_t n, double f) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= f;
}
void launch_scale_host(double* x, int64_t n, double scale, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_host_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, scale);
}

// ---------------------------------------------------------------------------
// Krylov vectors: [re (n) | im (n)] doubles.  Block partial sums are
// reduced in a fixed order (deterministic).
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* sh) {
  // 256 threads: wave reduction by shuffles, then across the 4 waves
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;  // valid in thread 0
}

// out[j] = sum_b partial[b * k2 + j], j < k2, summed in block order
__global__ void reduce_partials_kernel(const double* __restrict__ partial, int k2, int nblk,
                                       double* __restrict__ out) {
  const int j = blockIdx.x;
  __shared__ double sh[4];
  double v = 0;
  // fixed assignment of blocks to threads, then a fixed tree
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += partial[b * k2 + j];
  const double r = block_sum(v, sh);
  if (threadIdx.x == 0) out[j] = r;
}

void launch_reduce_partials(const double* partial, int k2, int nblk, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(k2), dim3(256), 0, s, partial, k2, nblk, out);
}

__global__ __launch_bounds__(RED_THREADS) void norm2_partial_kernel(const double* __restrict__ x,
                                                                    int64_t n2,
                                                                    double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  for (int64_t i = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x; i < n2; i += stride)
    acc += x[i] * x[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

void launch_norm2_partial(const double* x, int64_t n2, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(norm2_partial_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, n2,
                     partial);
}

__global__ void check_finite_kernel(const double* __restrict__ x, int64_t n, int* flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) bad = true;
  if (bad) flag[0] = 1;  // benign race: every writer stores the same value
}

void launch_check_finite(const double* x, int64_t n, int* flag, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, flag);
}

// one task per grid row, chunks of its range per grid column
__global__ __launch_bounds__(256) void check_finite_batch_kernel(
    const FiniteTask* __restrict__ tasks, int* __restrict__ flags) {
  const FiniteTask t = tasks[blockIdx.y];
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < t.n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(t.x[i])) bad = true;
  if (bad) flags[t.slot] = 1;  // benign race: every writer stores the same value
}

void launch_check_finite_batch(const FiniteTask* t, int ntask, int64_t max_n, int* flags,
                               hipStream_t s) {
  if (ntask <= 0 || max_n <= 0) return;
  int64_t gx = (max_n + 255) / 256;
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(check_finite_batch_kernel, dim3((unsigned)gx, ntask), dim3(256), 0, s, t,
                     flags);
}

// ---------------------------------------------------------------------------
// SVD staging: split planes <-> interleaved complex (the eigensolver's format)
// ---------------------------------------------------------------------------
__global__ void scatter_z_kernel(const ScatterTask* __restrict__ tasks,
                                 const double* __restrict__ z, double* __restrict__ re,
                                 double* __restrict__ im) {
  const ScatterTask t = tasks[blockIdx.z];
  for (int r = blockIdx.y; r < t.rows; r += gridDim.y)
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < t.cols;
         c += gridDim.x * blockDim.x) {
      const int64_t dst = t.dst_off + (int64_t)r * t.cols + c;
      if (t.lower && c > r) {
        re[dst] = 0.0;
        im[dst] = 0.0;
        continue;
      }
      const int64_t src = t.src_off + (int64_t)r * t.rs + (int64_t)c * t.cs;
      re[dst] = z[2 * src];
      im[dst] = t.conj ? -z[2 * src + 1] : z[2 * src + 1];
    }
}

__global__ void gather_z_kernel(const GatherTask* __restrict__ tasks,
                                const double* __restrict__ re, const double* __restrict__ im,
                                double* __restrict__ z) {
  const GatherTask t = tasks[blockIdx.z];
  for (int r = blockIdx.y; r < t.rows; r += gridDim.y)
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < t.cols;
         c += gridDim.x * blockDim.x) {
      const int64_t src = t.src_off + (int64_t)r * t.cols + c;
      const int64_t dst = t.dst_off + (int64_t)r * t.drs + (int64_t)c * t.dcs;
      z[2 * dst] = re[src];
      z[2 * dst + 1] = t.conj ? -im[src] : im[src];
    }
}

void launch_gather_z(const GatherTask* t, int ntask, int maxrows, int maxcols,
                     const double* re, const double* im, double* z, hipStream_t s) {
  if (ntask <= 0) return;
  dim3 grid((maxcols + 63) / 64, maxrows < 256 ? maxrows : 256, ntask);
  hipLaunchKernelGGL(gather_z_kernel, grid, dim3(64), 0, s, t, re, im, z);
}

void launch_scatter_z(const ScatterTask* t, int ntask, int maxrows, int maxcols,
                      const double* src_z, double* re, double* im, hipStream_t s) {
  if (ntask <= 0) return;
  dim3 grid((maxcols + 63) / 64, maxrows < 256 ? maxrows : 256, ntask);
  hipLaunchKernelGGL(scatter_z_kernel, grid, dim3(64), 0, s, t, src_z, re, im);
}

__global__ void zcopy_kernel(const ZCopyTask* __restrict__ tasks) {
  const ZCopyTask t = tasks[blockIdx.y];
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 2 * t.n;
       k += (int64_t)gridDim.x * blockDim.x)
    t.dst[k] = t.scale * t.src[k];
}

void launch_zcopy(const ZCopyTask* t, int ntask, int64_t max_n, hipStream_t s) {
  if (ntask <= 0 || max_n <= 0) return;
  const int64_t gx = (2 * max_n + 255) / 256;
  hipLaunchKernelGGL(zcopy_kernel, dim3((unsigned)(gx < 64 ? gx : 64), ntask), dim3(256), 0, s,
                     t);
}

__global__ __launch_bounds__(256) void znorm2_kernel(const ZNormTask* __restrict__ tasks) {
  const ZNormTask t = tasks[blockIdx.x];
  __shared__ double part[256];
  double acc = 0;
  for (int64_t k = threadIdx.x; k < 2 * t.n; k += 256) acc += t.src[k] * t.src[k];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *t.out = part[0];
}

void launch_znorm2(const ZNormTask* t, int ntask, hipStream_t s) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(znorm2_kernel, dim3(ntask), dim3(256), 0, s, t);
}

__global__ void interleave_kernel(const double* __restrict__ re, const double* __restrict__ im,
                                  double* __restrict__ z, int64_t n, int conj) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    z[2 * k] = re[k];
    z[2 * k + 1] = conj ? -im[k] : im[k];
  }
}

void launch_interleave(const double* re, const double* im, double* z, int64_t n, int conj,
                       hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(interleave_kernel, dim3(grid_for(n)), dim3(256), 0, s, re, im, z, n, conj);
}

// ---------------------------------------------------------------------------
// padded Hermitian batches
//
// A sector's n x n Gram matrix G goes into an npad x npad slot as
// M = Q A Q / s with A = diag(G, D), D = -s diag(1 + j/m) (m = npad - n,
// s = trace G, or 1 if that is zero) and Q = I - 2 u u^T / (u^T u) for a
// fixed irregular positive u.  Dividing by s puts every slot at unit scale:
// the library's eigensolver uses absolute tolerances (its eigenvalue errors
// grow to ~1e-8 |G| for |G| ~ 1e-9), and the deflated SVD decomposes Gram
// matrices of any scale.  The eigenvalues are multiplied back by s.  A alone would make the tridiagonal reduction
// split exactly at the block boundary and at every padding row, and the
// divide-and-conquer solver returns non-finite vectors for such splits; Q
// mixes the blocks so M has no exact split while sharing A's spectrum.  D's
// distinct values lie below G's (positive semidefinite) spectrum, so G's
// eigenpairs are the last n of the ascending ones, with vectors Q v.
// ---------------------------------------------------------------------------
__device__ inline double pad_u(int i) { return 1.0 + 0.5 * sin(0.7 + 2.3 * (double)i); }

// broadcast of block_sum to every thread (256 threads)
__device__ inline double block_sum_all(double v, double* sh, double* out) {
  const double r = block_sum(v, sh);
  if (threadIdx.x == 0) *out = r;
  __syncthreads();
  return *out;
}

// vec[2 (w_src + i)] = (G u)_i for i < n: one wave per row, using column i
// of G (G Hermitian: row i of G is the conjugate of column i).
__global__ __launch_bounds__(256) void pad_gvec_kernel(const PadTask* __restrict__ tasks,
                                                       double* __restrict__ vec) {
  const PadTask t = tasks[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= t.n) return;  // whole wave leaves together
  const double* col = t.z + 2 * (t.src_off + (int64_t)i * t.n);
  double ar = 0, ai = 0;
  for (int k = lane; k < t.n; k += 64) {
    const double u = pad_u(k);
    ar += col[2 * k] * u;
    ai -= col[2 * k + 1] * u;
  }
  for (int o = 32; o > 0; o >>= 1) {
    ar += __shfl_down(ar, o, 64);
    ai += __shfl_down(ai, o, 64);
  }
  if (lane == 0) {
    vec[2 * (t.w_src + i)] = ar;
    vec[2 * (t.w_src + i) + 1] = ai;
  }
}

__global__ __launch_bounds__(256) void pad_embed_kernel(const PadTask* __restrict__ tasks,
                                                        const double* __restrict__ vec,
                                                        double* __restrict__ dst) {
  __shared__ double sh[4];
  __shared__ double bc;
  const PadTask t = tasks[blockIdx.y];
  const double* __restrict__ src = t.z;
  const int n = t.n, np = t.npad, m = np - n;
  // scalars of the slot (every block computes them: O(npad) from cache)
  double tr = 0, nu = 0, bg = 0, p0 = 0, p1 = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const double u = pad_u(i);
    nu += u * u;
    if (i < n) {
      tr += src[2 * (t.src_off + i + (int64_t)i * n)];
      bg += u * vec[2 * (t.w_src + i)];
    } else {
      p0 += u * u;
      p1 += u * u * (double)(i - n);
    }
  }
  tr = block_sum_all(tr, sh, &bc);
  nu = block_sum_all(nu, sh, &bc);
  bg = block_sum_all(bg, sh, &bc);
  p0 = block_sum_all(p0, sh, &bc);
  p1 = block_sum_all(p1, sh, &bc);
  const double sc = tr > 0 ? tr : 1.0;
  const double inv = 1.0 / sc;
  if (blockIdx.x == 0 && threadIdx.x == 0) *t.scale = sc;
  const double rm = m > 0 ? 1.0 / m : 0.0;
  // beta = u^T A u; d_i = -sc (1 + (i - n) / m) on the padding rows
  const double beta = bg - sc * (p0 + p1 * rm);
  const double f1 = 2.0 / nu, f2 = 4.0 * beta / (nu * nu);
  const int64_t tot = (int64_t)np * np;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % np), c = (int)(e / np);
    double ar = 0, ai = 0;
    if (r < n && c < n) {
      const int64_t k = t.src_off + r + (int64_t)c * n;
      ar = src[2 * k];
      ai = src[2 * k + 1];
    } else if (r == c) {
      ar = -sc * (1.0 + (r - n) * rm);
    }
    const double ur = pad_u(r), uc = pad_u(c);
    double wrr, wri, wcr, wci;  // (A u)_r and (A u)_c
    if (r < n) {
      wrr = vec[2 * (t.w_src + r)];
      wri = vec[2 * (t.w_src + r) + 1];
    } else {
      wrr = -sc * (1.0 + (r - n) * rm) * ur;
      wri = 0;
    }
    if (c < n) {
      wcr = vec[2 * (t.w_src + c)];
      wci = vec[2 * (t.w_src + c) + 1];
    } else {
      wcr = -sc * (1.0 + (c - n) * rm) * uc;
      wci = 0;
    }
    // M = A - f1 (u w^H + w u^T) + f2 u u^T
    dst[2 * (t.dst_off + e)] = inv * (ar - f1 * (ur * wcr + wrr * uc) + f2 * ur * uc);
    dst[2 * (t.dst_off + e) + 1] = inv * (ai - f1 * (-ur * wci + wri * uc));
  }
}

void launch_pad_embed(const PadTask* t, int ntask, int max_n, int max_npad, double* vec,
                      double* dst_z, hipStream_t s) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(pad_gvec_kernel, dim3((max_n + 3) / 4, ntask), dim3(256), 0, s, t, vec);
  const int gx = grid_for((int64_t)max_npad * max_npad, 256, 512);
  hipLaunchKernelGGL(pad_embed_kernel, dim3(gx, ntask), dim3(256), 0, s, t, vec, dst_z);
}

// One block per kept column c < n: v = slot column npad - n + c, rho = u^T v,
// z[:, c] = (v - 2 u rho / (u^T u)) restricted to the first n rows.
__global__ __launch_bounds__(256) void pad_extract_kernel(const PadTask* __restrict__ tasks,
                                                          const double* __restrict__ slot_z,
                                                          const double* __restrict__ slot_w) {
  __shared__ double sh[4];
  __shared__ double bc;
  const PadTask t = tasks[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= t.n) return;  // uniform over the block
  const int np = t.npad, sft = np - t.n;
  const double* v = slot_z + 2 * (t.dst_off + (int64_t)(sft + c) * np);
  double rr = 0, ri = 0, nu = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const double u = pad_u(i);
    rr += u * v[2 * i];
    ri += u * v[2 * i + 1];
    nu += u * u;
  }
  rr = block_sum_all(rr, sh, &bc);
  ri = block_sum_all(ri, sh, &bc);
  nu = block_sum_all(nu, sh, &bc);
  const double f = 2.0 / nu;
  double* out = t.z + 2 * (t.src_off + (int64_t)c * t.n);
  for (int r = threadIdx.x; r < t.n; r += blockDim.x) {
    const double u = pad_u(r);
    out[2 * r] = v[2 * r] - f * u * rr;
    out[2 * r + 1] = v[2 * r + 1] - f * u * ri;
  }
  if (threadIdx.x == 0) t.w[t.w_dst + c] = *t.scale * slot_w[t.w_src + sft + c];
}

void launch_pad_extract(const PadTask* t, int ntask, int max_n, const double* slot_z,
                        const double* slot_w, hipStream_t s) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(pad_extract_kernel, dim3(max_n, ntask), dim3(256), 0, s, t, slot_z, slot_w);
}

}  // namespace tnt
