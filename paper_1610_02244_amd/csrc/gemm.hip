// Grouped split-complex GEMM on CDNA4 matrix cores.
//
// Every tensor contraction of the two-site DMRG step (H_eff . theta, the
// environment updates, theta formation) is a list of independent complex
// block products C[M x N] = sum_seg op(A_seg) op(B_seg) whose sizes follow
// the U(1) sectors (1 .. ~300 per side at chi = 1024).  One launch covers a
// whole list: each workgroup owns one BM x BN output tile of one task and
// walks that task's K-segments in order, so every output element is written
// by exactly one workgroup with a fixed summation order (bitwise
// reproducible, no atomics).
//
// Complex data live in separate re/im planes.  A complex tile product is four
// real MFMA products accumulated into two real accumulators:
//   Cr += Ar Br - Ai Bi ,  Ci += Ar Bi + Ai Br.
// Operand permutes (row- or column-major blocks, conjugation) are folded
// into the global->LDS loaders; LDS holds both operands K-major so every
// MFMA fragment read is 16 consecutive elements per k row.
//
// gfx950 MFMA lane layouts used (16x16x4, 64 lanes):
//   A operand: lane l holds A[l % 16][l / 16];  B: B[l / 16][l % 16];
//   f32 result register r of lane l: C[4 (l / 16) + r][l % 16];
//   f64 result register r of lane l: C[4 r + l / 16][l % 16].
#include "kernels.h"

namespace tnt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<float> {
  typedef f32x4 acc_t;
  __device__ static inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mma<double> {
  typedef f64x4 acc_t;
  __device__ static inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

constexpr int NT = 256;  // 4 waves, arranged 2 x 2 over the output tile

template <typename T, typename TA, typename TB, typename TC, int FORM, int BM, int BN, int BK>
__global__ __launch_bounds__(NT) void grouped_gemm_kernel(
    const GemmTask* __restrict__ tasks, const GemmSeg* __restrict__ segs,
    const int2* __restrict__ tiles, int ntiles, const TA* __restrict__ Are,
    const TA* __restrict__ Aim, const TB* __restrict__ Bre, const TB* __restrict__ Bim,
    TC* __restrict__ Cre, TC* __restrict__ Cim) {
  constexpr bool TRANS_A = (FORM == FORM_CN);
  constexpr bool CONJ_A = (FORM == FORM_CN || FORM == FORM_cNT);
  constexpr bool TRANS_B = (FORM == FORM_NT || FORM == FORM_cNT);
  constexpr int PAD = 16 / sizeof(T) * 4;  // 16 floats / 8 doubles of row padding
  constexpr int EA = BM * BK / NT;         // A elements per thread per chunk
  constexpr int EB = BK * BN / NT;
  constexpr int FM = BM / 32, FN = BN / 32;  // 16x16 fragments per wave
  static_assert(EA >= 1 && EB >= 1 && NT % BK == 0 && NT % BM == 0 && NT % BN == 0, "tile");
  using acc_t = typename Mma<T>::acc_t;

  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);

  // The tile table is laid out by the planner so that block b (which the
  // dispatcher places on XCD b % 8) takes slot b / 8 of that XCD's bin: tasks
  // are balanced over the 8 XCDs and all tiles of one task share an L2.
  if ((int)blockIdx.x >= ntiles) return;
  const int2 td = tiles[blockIdx.x];
  if (td.x < 0) return;
  const GemmTask tk = tasks[td.x];
  const int m0 = (td.y & 0xffff) * BM, n0 = (td.y >> 16) * BN;
  const int M = tk.M, N = tk.N;

  acc_t accR[FM][FN], accI[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) { accR[i][j][r] = 0; accI[i][j][r] = 0; }

  T ra[2][EA], rb[2][EB];  // register staging of the next chunk (re, im)

  // load one BK-chunk of segment `sg` starting at k0 into registers
  auto load = [&](const GemmSeg& sg, int k0) {
    const int K = sg.K;
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int m, k;
      if (TRANS_A) { m = tid % BM; k = tid / BM + e * (NT / BM); }
      else { k = tid % BK; m = tid / BK + e * (NT / BK); }
      const int gm = m0 + m, gk = k0 + k;
      T vr = 0, vi = 0;
      if (gm < M && gk < K) {
        const int64_t idx = TRANS_A ? sg.a_off + (int64_t)gk * sg.lda + gm
                                    : sg.a_off + (int64_t)gm * sg.lda + gk;
        vr = (T)Are[idx];
        vi = (T)Aim[idx];
        if (CONJ_A) vi = -vi;
      }
      ra[0][e] = vr; ra[1][e] = vi;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int n, k;
      if (TRANS_B) { k = tid % BK; n = tid / BK + e * (NT / BK); }
      else { n = tid % BN; k = tid / BN + e * (NT / BN); }
      const int gn = n0 + n, gk = k0 + k;
      T vr = 0, vi = 0;
      if (gn < N && gk < K) {
        const int64_t idx = TRANS_B ? sg.b_off + (int64_t)gn * sg.ldb + gk
                                    : sg.b_off + (int64_t)gk * sg.ldb + gn;
        vr = (T)Bre[idx];
        vi = (T)Bim[idx];
      }
      rb[0][e] = vr; rb[1][e] = vi;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int m, k;
      if (TRANS_A) { m = tid % BM; k = tid / BM + e * (NT / BM); }
      else { k = tid % BK; m = tid / BK + e * (NT / BK); }
      As[0][k][m] = ra[0][e];
      As[1][k][m] = ra[1][e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int n, k;
      if (TRANS_B) { k = tid % BK; n = tid / BK + e * (NT / BK); }
      else { n = tid % BN; k = tid / BN + e * (NT / BN); }
      Bs[0][k][n] = rb[0][e];
      Bs[1][k][n] = rb[1][e];
    }
  };

  // walk the chunks (segment, k0) of this task in order
  int s = 0, k0 = 0;
  const int nseg = tk.nseg;
  GemmSeg cur;
  if (nseg > 0) {
    cur = segs[tk.seg0];
    // skip empty segments
    while (cur.K <= 0 && ++s < nseg) cur = segs[tk.seg0 + s];
  }
  if (s < nseg) load(cur, 0);
  while (s < nseg) {
    const int kvalid = min(BK, cur.K - k0);
    store();
    __syncthreads();
    // advance to the next chunk and prefetch it while this one computes
    int ns = s, nk0 = k0 + BK;
    GemmSeg nxt = cur;
    if (nk0 >= cur.K) {
      nk0 = 0;
      ++ns;
      while (ns < nseg) {
        nxt = segs[tk.seg0 + ns];
        if (nxt.K > 0) break;
        ++ns;
      }
    }
    if (ns < nseg) load(nxt, nk0);

    const int nkk = (kvalid + 3) >> 2;
    for (int kk = 0; kk < nkk; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      T ar[FM], ai[FM], nai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = As[0][kr][wm + i * 16 + (lane & 15)];
        ai[i] = As[1][kr][wm + i * 16 + (lane & 15)];
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = Bs[0][kr][wn + j * 16 + (lane & 15)];
        bi[j] = Bs[1][kr][wn + j * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          accR[i][j] = Mma<T>::run(ar[i], br[j], accR[i][j]);
          accR[i][j] = Mma<T>::run(nai[i], bi[j], accR[i][j]);
          accI[i][j] = Mma<T>::run(ar[i], bi[j], accI[i][j]);
          accI[i][j] = Mma<T>::run(ai[i], br[j], accI[i][j]);
        }
    }
    __syncthreads();
    s = ns; k0 = nk0; cur = nxt;
  }

  // epilogue: write the tile (zeros for a task without segments)
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + Mma<T>::row(lane, r);
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          const int64_t idx = tk.c_off + (int64_t)gm * tk.ldc + gn;
          Cre[idx] = (TC)accR[i][j][r];
          Cim[idx] = (TC)accI[i][j][r];
        }
      }
}

// ---------------------------------------------------------------------------

static const int kTileDims[][2] = {{64, 64}, {32, 32}, {128, 64}, {64, 128}, {128, 128}};

void gemm_tile_dims(int cfg, int* bm, int* bn) {
  *bm = kTileDims[cfg][0];
  *bn = kTileDims[cfg][1];
}
int gemm_num_tile_cfgs() { return 5; }

template <typename T, typename TA, typename TB, typename TC, int FORM, int BM, int BN>
static void launch_t(const GemmLaunch& g, hipStream_t s) {
  constexpr int BK = 16;
  hipLaunchKernelGGL((grouped_gemm_kernel<T, TA, TB, TC, FORM, BM, BN, BK>), dim3(g.ntiles),
                     dim3(NT), 0, s, g.tasks, g.segs, g.tiles, g.ntiles,
                     static_cast<const TA*>(g.a_re), static_cast<const TA*>(g.a_im),
                     static_cast<const TB*>(g.b_re), static_cast<const TB*>(g.b_im),
                     static_cast<TC*>(g.c_re), static_cast<TC*>(g.c_im));
}

// Launch with the tile shape the tile table was built for; a shape the
// element type does not provide is refused (false), never substituted.
template <typename T, typename TA, typename TB, typename TC, int FORM>
static bool launch_tiles(const GemmLaunch& g, hipStream_t s) {
  switch (g.tile_cfg) {
    case 0: launch_t<T, TA, TB, TC, FORM, 64, 64>(g, s); return true;
    case 1: launch_t<T, TA, TB, TC, FORM, 32, 32>(g, s); return true;
    case 2: launch_t<T, TA, TB, TC, FORM, 128, 64>(g, s); return true;
    case 3: launch_t<T, TA, TB, TC, FORM, 64, 128>(g, s); return true;
    case 4:
      if constexpr (sizeof(T) == 4) {
        launch_t<T, TA, TB, TC, FORM, 128, 128>(g, s);
        return true;
      }
      return false;
    default: return false;
  }
}

bool gemm_cfg_valid(int cfg, GemmPath path) { return cfg >= 0 && cfg <= (path == PATH_F64 ? 3 : 4); }

bool bf16x3_available() { return false; }

bool launch_grouped_gemm(const GemmLaunch& g, hipStream_t s) {
  if (g.ntiles <= 0) return true;
  if (g.path == PATH_F64) {
    if (g.a_t != ET_F64 || g.b_t != ET_F64 || g.c_t != ET_F64) return false;
    switch (g.form) {
      case FORM_NN: return launch_tiles<double, double, double, double, FORM_NN>(g, s);
      case FORM_NT: return launch_tiles<double, double, double, double, FORM_NT>(g, s);
      case FORM_CN: return launch_tiles<double, double, double, double, FORM_CN>(g, s);
      case FORM_cNT: return launch_tiles<double, double, double, double, FORM_cNT>(g, s);
    }
    return false;
  }
  if (g.path != PATH_F32) return false;
  // FP32 path: step 1 (NN: A f32 env copy, B f64 Krylov vector, C f32 slab)
  // and step 4 (NT: A f32 slab, B f32 env copy, C f64 Krylov vector).
  if (g.form == FORM_NN && g.a_t == ET_F32 && g.b_t == ET_F64 && g.c_t == ET_F32)
    return launch_tiles<float, float, double, float, FORM_NN>(g, s);
  if (g.form == FORM_NT && g.a_t == ET_F32 && g.b_t == ET_F32 && g.c_t == ET_F64)
    return launch_tiles<float, float, float, double, FORM_NT>(g, s);
  if (g.form == FORM_NN && g.a_t == ET_F32 && g.b_t == ET_F32 && g.c_t == ET_F32)
    return launch_tiles<float, float, float, float, FORM_NN>(g, s);
  return false;
}

}  // namespace tnt
