// Grouped split-complex FP64 GEMM on CDNA4 matrix cores, any operand form.
//
// Every tensor contraction of the two-site DMRG step (H_eff . theta, the
// environment updates, theta formation, Gram matrices of the SVD step) is a
// list of independent complex block products C[M x N] = sum_seg op(A_seg)
// op(B_seg) whose sizes follow the U(1) sectors (1 .. ~300 per side at
// chi = 1024).  One launch covers a whole list: each workgroup owns one
// BM x BN output tile of one task and walks that task's K-segments in order,
// so every output element is written by exactly one workgroup with a fixed
// summation order (bitwise reproducible, no atomics).  This kernel serves
// the FP64 path in all four operand forms; the reduced-precision H_eff
// paths run on packed operands (gemm_packed.hip).
//
// Complex data live in separate re/im planes.  A complex tile product takes
// three real MFMA products (Gauss's form) accumulated separately over K:
//   P1 += Ar Br,  P2 += Ai Bi,  P3 += (Ar + Ai)(Br + Bi),
// and the epilogue forms Cr = P1 - P2, Ci = P3 - P1 - P2.  This issues 3/4
// of the MFMA work of the schoolbook form; the error stays of the order of
// the working precision times |A||B| (normwise).
// Operand permutes (row- or column-major blocks, conjugation) are folded
// into the global->LDS loaders.
//
// LDS layout: each operand row (an m of A or an n of B) holds one K-chunk of
// 16 elements in the permuted order pos(k) = 4 (k mod 4) + k / 4, plus 4
// elements of padding.  MFMA number kk of a chunk takes k = 4 kk + slot for
// the operand slot held by lane group slot = lane / 16, so the four values a
// lane needs for the chunk's four MFMAs are contiguous: one LDS read per
// operand row and plane.  A loader thread owns a (row, k mod 4) residue and
// writes its four values with one LDS store.  The k order of the
// accumulation is the natural one (chunk by chunk, k = 0, 1, 2, ...).
#include "mfma.h"

namespace tnt {

constexpr int BK = 16;   // K per chunk
constexpr int KP = 20;   // LDS row length: 16 permuted k + 4 padding

// Loader of one operand: rows = BR (BM for A, BN for B), residues j = k mod 4.
// CONTIG: consecutive k are adjacent in memory (then consecutive threads take
// consecutive residues of a row); otherwise consecutive threads take
// consecutive rows (k is strided and rows are adjacent).
template <typename T, typename TS, int BR, bool CONTIG, bool CONJ>
struct Loader {
  static constexpr int ITEMS = 4 * BR;
  static constexpr int PER = (ITEMS + NT - 1) / NT;
  T v[PER][2][4];
  // ld_row: element distance between rows; ld_k: between consecutive k
  __device__ inline void load(const TS* __restrict__ re, const TS* __restrict__ im, int64_t off,
                              int64_t ld_row, int64_t ld_k, int r0, int rows, int k0, int K,
                              int tid) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int item = tid + e * NT;
      const int r = CONTIG ? item / 4 : item % BR;
      const int j = CONTIG ? item % 4 : item / BR;
      const bool rv = item < ITEMS && r0 + r < rows;
      const int64_t base = off + (int64_t)(r0 + r) * ld_row;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + j + 4 * i;
        T a = 0, b = 0;
        if (rv && k < K) {
          const int64_t idx = base + (int64_t)k * ld_k;
          a = (T)re[idx];
          b = (T)im[idx];
          if (CONJ) b = -b;
        }
        v[e][0][i] = a;
        v[e][1][i] = b;
      }
    }
  }
  __device__ inline void store(T (*S)[BR][KP], int tid) const {
    using quad_t = typename Mma<T>::quad_t;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int item = tid + e * NT;
      if (item >= ITEMS) continue;
      const int r = CONTIG ? item / 4 : item % BR;
      const int j = CONTIG ? item % 4 : item / BR;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        quad_t q;
        q[0] = v[e][p][0]; q[1] = v[e][p][1]; q[2] = v[e][p][2]; q[3] = v[e][p][3];
        *reinterpret_cast<quad_t*>(&S[p][r][4 * j]) = q;
      }
    }
  }
};

template <typename T, typename TA, typename TB, typename TC, int FORM, int BM, int BN>
__global__ __launch_bounds__(NT) void grouped_gemm_kernel(
    const GemmTask* __restrict__ tasks, const GemmSeg* __restrict__ segs,
    const int2* __restrict__ tiles, int ntiles, const TA* __restrict__ Are,
    const TA* __restrict__ Aim, const TB* __restrict__ Bre, const TB* __restrict__ Bim,
    TC* __restrict__ Cre, TC* __restrict__ Cim) {
  constexpr bool TRANS_A = (FORM == FORM_CN);
  constexpr bool CONJ_A = (FORM == FORM_CN || FORM == FORM_cNT);
  constexpr bool TRANS_B = (FORM == FORM_NT || FORM == FORM_cNT);
  // FP32 tiles double-buffer the LDS (one barrier per chunk); FP64 tiles
  // would not fit two stages at useful occupancy and use one
  constexpr int STAGES = sizeof(T) == 4 ? 2 : 1;
  constexpr int FM = BM / 32, FN = BN / 32;  // 16x16 fragments per wave
  using acc_t = typename Mma<T>::acc_t;
  using quad_t = typename Mma<T>::quad_t;

  __shared__ __attribute__((aligned(32))) T As[STAGES][2][BM][KP];
  __shared__ __attribute__((aligned(32))) T Bs[STAGES][2][BN][KP];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int frow = lane & 15, slot = lane >> 4;

  // The tile table is laid out by the planner so that block b (which the
  // dispatcher places on XCD b % 8) takes slot b / 8 of that XCD's bin: tasks
  // are balanced over the 8 XCDs and all tiles of one task share an L2.
  if ((int)blockIdx.x >= ntiles) return;
  const int2 td = tiles[blockIdx.x];
  if (td.x < 0) return;
  const GemmTask tk = tasks[td.x];
  const int m0 = (td.y & 0xffff) * BM, n0 = (td.y >> 16) * BN;
  const int M = tk.M, N = tk.N;

  // three real products per complex product (Gauss):
  //   P1 = Ar Br,  P2 = Ai Bi,  P3 = (Ar + Ai)(Br + Bi);
  //   Cr = P1 - P2,  Ci = P3 - P1 - P2
  acc_t acc1[FM][FN], acc2[FM][FN], acc3[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) { acc1[i][j][r] = 0; acc2[i][j][r] = 0; acc3[i][j][r] = 0; }

  // A (M x K): stored row-major M x K (k contiguous), or K x M for FORM_CN
  // B (K x N): stored row-major K x N (rows n strided), or N x K (k contiguous)
  Loader<T, TA, BM, !TRANS_A, CONJ_A> la;
  Loader<T, TB, BN, TRANS_B, false> lb;
  auto load = [&](const GemmSeg& sg, int k0) {
    la.load(Are, Aim, sg.a_off, TRANS_A ? 1 : sg.lda, TRANS_A ? sg.lda : 1, m0, M, k0, sg.K, tid);
    lb.load(Bre, Bim, sg.b_off, TRANS_B ? sg.ldb : 1, TRANS_B ? 1 : sg.ldb, n0, N, k0, sg.K, tid);
  };
  auto store = [&](int st) {
    la.store(As[st], tid);
    lb.store(Bs[st], tid);
  };
  // 16x16 fragments lying wholly outside the block are skipped (uniform per
  // wave), so ragged edges cost 16-granular padding, not tile-granular
  const int fm_live = min(FM, max(0, (M - m0 - wm + 15) >> 4));
  const int fn_live = min(FN, max(0, (N - n0 - wn + 15) >> 4));
  auto compute = [&](int st, int kvalid) {
    quad_t ar[FM], ai[FM], as[FM], br[FN], bi[FN], bs[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      if (i < fm_live) {
        ar[i] = *reinterpret_cast<const quad_t*>(&As[st][0][wm + 16 * i + frow][4 * slot]);
        ai[i] = *reinterpret_cast<const quad_t*>(&As[st][1][wm + 16 * i + frow][4 * slot]);
        as[i] = ar[i] + ai[i];
      }
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      if (j < fn_live) {
        br[j] = *reinterpret_cast<const quad_t*>(&Bs[st][0][wn + 16 * j + frow][4 * slot]);
        bi[j] = *reinterpret_cast<const quad_t*>(&Bs[st][1][wn + 16 * j + frow][4 * slot]);
        bs[j] = br[j] + bi[j];
      }
    }
    const int nkk = (kvalid + 3) >> 2;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      if (kk < nkk) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if (i < fm_live && j < fn_live) {
              acc1[i][j] = Mma<T>::run(ar[i][kk], br[j][kk], acc1[i][j]);
              acc2[i][j] = Mma<T>::run(ai[i][kk], bi[j][kk], acc2[i][j]);
              acc3[i][j] = Mma<T>::run(as[i][kk], bs[j][kk], acc3[i][j]);
            }
          }
      }
    }
  };

  walk_chunks<BK, STAGES>(segs, tk.seg0, tk.nseg, load, store, compute);

  // epilogue: write the tile (zeros for a task without segments)
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + Mma<T>::row(lane, r);
        const int gn = n0 + wn + j * 16 + frow;
        if (gm < M && gn < N) {
          const int64_t idx = tk.c_off + (int64_t)gm * tk.ldc + gn;
          const T p1 = acc1[i][j][r], p2 = acc2[i][j][r];
          Cre[idx] = (TC)(p1 - p2);
          Cim[idx] = (TC)(acc3[i][j][r] - p1 - p2);
        }
      }
}

static const int kTileDims[][2] = {{64, 64}, {32, 32}, {128, 64}, {64, 128}, {128, 128}};

void gemm_tile_dims(int cfg, int* bm, int* bn) {
  *bm = kTileDims[cfg][0];
  *bn = kTileDims[cfg][1];
}
int gemm_num_tile_cfgs() { return 5; }

template <typename T, typename TA, typename TB, typename TC, int FORM, int BM, int BN>
static void launch_t(const GemmLaunch& g, hipStream_t s) {
  hipLaunchKernelGGL((grouped_gemm_kernel<T, TA, TB, TC, FORM, BM, BN>), dim3(g.ntiles),
                     dim3(NT), 0, s, g.tasks, g.segs, g.tiles, g.ntiles,
                     static_cast<const TA*>(g.a_re), static_cast<const TA*>(g.a_im),
                     static_cast<const TB*>(g.b_re), static_cast<const TB*>(g.b_im),
                     static_cast<TC*>(g.c_re), static_cast<TC*>(g.c_im));
}

// Launch with the tile shape the tile table was built for; a shape the
// kernel does not provide is refused (false), never substituted.
template <typename T, typename TA, typename TB, typename TC, int FORM>
static bool launch_tiles(const GemmLaunch& g, hipStream_t s) {
  switch (g.tile_cfg) {
    case 0: launch_t<T, TA, TB, TC, FORM, 64, 64>(g, s); return true;
    case 1: launch_t<T, TA, TB, TC, FORM, 32, 32>(g, s); return true;
    case 2: launch_t<T, TA, TB, TC, FORM, 128, 64>(g, s); return true;
    case 3: launch_t<T, TA, TB, TC, FORM, 64, 128>(g, s); return true;
    default: return false;
  }
}

// 128 x 128 tiles exist for the packed FP32 kernel only (the FP64 and BF16x3
// kernels would spill registers at that size)
bool gemm_cfg_valid(int cfg, GemmPath path) { return cfg >= 0 && cfg <= (path == PATH_F32 ? 4 : 3); }

bool bf16x3_available() { return true; }

// FP64 grouped GEMM in any operand form (the reduced-precision paths run on
// packed operands, launch_packed_gemm)
bool launch_grouped_gemm(const GemmLaunch& g, hipStream_t s) {
  if (g.ntiles <= 0) return true;
  if (g.path != PATH_F64 || g.a_t != ET_F64 || g.b_t != ET_F64 || g.c_t != ET_F64) return false;
  switch (g.form) {
    case FORM_NN: return launch_tiles<double, double, double, double, FORM_NN>(g, s);
    case FORM_NT: return launch_tiles<double, double, double, double, FORM_NT>(g, s);
    case FORM_CN: return launch_tiles<double, double, double, double, FORM_CN>(g, s);
    case FORM_cNT: return launch_tiles<double, double, double, double, FORM_cNT>(g, s);
  }
  return false;
}

}  // namespace tnt
