// Grouped split-complex GEMM on packed operands: the FP32 and BF16x3 paths
// of H_eff . theta.
//
// C[M x N] = sum over segments A[M x K] B[N x K]^T, with A and B packed
// (kernels.h: k contiguous, rows padded to a multiple of 8 elements, zero
// padding, 16-byte aligned).  Task lists, tile tables and the K-segment walk
// are those of the FP64 kernel: one workgroup per output tile, K summed in a
// fixed order, no atomics.
//
// Loads: a 16-byte group holds G consecutive k of one row and plane (G = 4
// floats or 8 bf16).  Loader item = (row, group), one 16-byte buffer load
// and one 16-byte LDS store per plane; a chunk is 4 groups (BK = 4 G).  The
// chunk's base address is uniform and a lane adds only its row and group
// offset; rows outside the block and groups at or beyond K are given an
// offset past the buffer's range and come back as zeros, so the loop carries
// almost no per-lane address arithmetic.  The LDS row of an operand is 4
// groups plus one padding group (80 bytes), which keeps the 16 rows read by
// one lane slot on distinct banks.
//
// Every fragment of the wave is read from LDS (rows outside the block are
// zero there); MFMAs on fragments wholly outside the block are skipped, and
// tiles whose fragments are all live run a copy of the K walk without those
// tests.
//
// FP32 (16x16x4 MFMA): lane slot s reads group s of its row, i.e. k = 4 s ..
// 4 s + 3; MFMA number kk of the chunk takes element kk of every slot's
// group, so it contracts k in {kk, 4 + kk, 8 + kk, 12 + kk}.  A and B use the
// same assignment, and the four MFMAs of a chunk together cover its 16 k.
// Complex products use Gauss's three real products:
//   P1 += Ar Br,  P2 += Ai Bi,  P3 += (Ar + Ai)(Br + Bi);
//   Cr = P1 - P2,  Ci = P3 - P1 - P2.
//
// BF16x3 (16x16x32 bf16 MFMA): lane slot s reads group s (k = 8 s .. 8 s + 7)
// of each of the four planes (re hi, re lo, im hi, im lo); one MFMA step
// covers the whole 32-k chunk.  A real product is approximated by
// hi*hi + hi*lo + lo*hi (the lo*lo term, of relative size 2^-16, is
// dropped), each with FP32 accumulation, and the complex product uses the
// schoolbook form on the four planes already in LDS:
//   P1 += Ar Br,  P2 += Ai Bi,  P3 += Ar Bi + Ai Br;  Cr = P1 - P2, Ci = P3.
// (Gauss's form would need two more split planes for the sums.)
#include <type_traits>

#include "mfma.h"

namespace tnt {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int FMT> struct Fmt;
template <> struct Fmt<PK_F32> {
  static constexpr int G = 4, BK = 16, PL = 2, EB = 4;
};
template <> struct Fmt<PK_BF16X3> {
  static constexpr int G = 8, BK = 32, PL = 4, EB = 2;
};

constexpr int ROWQ = 5;  // LDS row: 4 groups of data + 1 group of padding

template <int FMT, int BR>
struct PLoader {
  static constexpr int ITEMS = 4 * BR;
  static constexpr int PER = (ITEMS + NT - 1) / NT;
  static constexpr int PL = Fmt<FMT>::PL, G = Fmt<FMT>::G, EB = Fmt<FMT>::EB;
  u32x4 v[PER][PL];
  int rowc[PER];  // the item's row in the segment's operand block, or -1
  int jb[PER];    // element offset of the item's group in the chunk
  __device__ inline void init(int r0, int rows, int tid) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int item = tid + e * NT;
      const int r = item >> 2, j = item & 3;
      rowc[e] = (item < ITEMS && r0 + r < rows) ? r0 + r : -1;
      jb[e] = G * j;
    }
  }
  // Buffer loads: the chunk's base address is uniform (scalar registers); a
  // lane's offset is its row times ld plus its group.  Rows outside the block
  // and groups at or beyond K get an offset past the buffer's range, which
  // the hardware returns as zero without touching memory.
  __device__ inline void load(const char* __restrict__ base, int64_t plane_bytes, int64_t off,
                              int ld, int k0, int K) {
    const char* p = base + (off + k0) * EB;
    const int kv = K - k0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const bool ok = rowc[e] >= 0 && jb[e] < kv;
      const uint32_t o = ok ? (uint32_t)(rowc[e] * ld + jb[e]) * EB : 0x80000000u;
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(p + pl * plane_bytes), (short)0, 0x7fffffff, 0x00020000);
        v[e][pl] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0));
      }
    }
  }
  __device__ inline void store(u32x4 (*S)[BR][ROWQ], int tid) const {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int item = tid + e * NT;
      if (item >= ITEMS) continue;
      const int r = item >> 2, j = item & 3;
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) S[pl][r][j] = v[e][pl];
    }
  }
};

template <int FMT, typename TC, int BM, int BN>
__global__ __launch_bounds__(NT) void packed_gemm_kernel(
    const GemmTask* __restrict__ tasks, const GemmSeg* __restrict__ segs,
    const int2* __restrict__ tiles, int ntiles, const char* __restrict__ A, int64_t a_pb,
    const char* __restrict__ B, int64_t b_pb, TC* __restrict__ Cre, TC* __restrict__ Cim) {
  using F = Fmt<FMT>;
  constexpr int PL = F::PL;
  constexpr int STAGE_BYTES = PL * (BM + BN) * ROWQ * 16;
  // two LDS stages while two workgroups per CU still fit
  constexpr int STAGES = (2 * STAGE_BYTES <= 81920) ? 2 : 1;
  constexpr int FM = BM / 32, FN = BN / 32;  // 16x16 fragments per wave

  __shared__ u32x4 As[STAGES][PL][BM][ROWQ];
  __shared__ u32x4 Bs[STAGES][PL][BN][ROWQ];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int frow = lane & 15, slot = lane >> 4;

  // block b runs on XCD b % 8 and takes slot b / 8 of that XCD's bin of the
  // tile table (the planner balances the bins)
  if ((int)blockIdx.x >= ntiles) return;
  const int2 td = tiles[blockIdx.x];
  if (td.x < 0) return;
  const GemmTask tk = tasks[td.x];
  const int m0 = (td.y & 0xffff) * BM, n0 = (td.y >> 16) * BN;
  const int M = tk.M, N = tk.N;

  f32x4 acc1[FM][FN], acc2[FM][FN], acc3[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) { acc1[i][j][r] = 0; acc2[i][j][r] = 0; acc3[i][j][r] = 0; }

  PLoader<FMT, BM> la;
  PLoader<FMT, BN> lb;
  la.init(m0, M, tid);
  lb.init(n0, N, tid);
  auto load = [&](const GemmSeg& sg, int k0) {
    la.load(A, a_pb, sg.a_off, sg.lda, k0, sg.K);
    lb.load(B, b_pb, sg.b_off, sg.ldb, k0, sg.K);
  };
  auto store = [&](int st) {
    la.store(As[st], tid);
    lb.store(Bs[st], tid);
  };
  // 16x16 fragments wholly outside the block are skipped (uniform per wave)
  const int fm_live = min(FM, max(0, (M - m0 - wm + 15) >> 4));
  const int fn_live = min(FN, max(0, (N - n0 - wn + 15) >> 4));
  // k beyond the segment is zero in LDS: every chunk runs whole
  auto compute_t = [&](int st, auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    if constexpr (FMT == PK_F32) {
      f32x4 ar[FM], ai[FM], as[FM], br[FN], bi[FN], bs[FN];
      // every fragment is read (dead rows hold zeros in LDS): no register
      // needs a defined value on a skipped path
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = __builtin_bit_cast(f32x4, As[st][0][wm + 16 * i + frow][slot]);
        ai[i] = __builtin_bit_cast(f32x4, As[st][1][wm + 16 * i + frow][slot]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = __builtin_bit_cast(f32x4, Bs[st][0][wn + 16 * j + frow][slot]);
        bi[j] = __builtin_bit_cast(f32x4, Bs[st][1][wn + 16 * j + frow][slot]);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i) as[i] = ar[i] + ai[i];
#pragma unroll
      for (int j = 0; j < FN; ++j) bs[j] = br[j] + bi[j];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (FULL || (i < fm_live && j < fn_live)) {
              acc1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i][kk], br[j][kk], acc1[i][j], 0, 0, 0);
              acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i][kk], bi[j][kk], acc2[i][j], 0, 0, 0);
              acc3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[i][kk], bs[j][kk], acc3[i][j], 0, 0, 0);
            }
    } else {
      bf16x8 a[FM][4], b[FN][4];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        if (i < fm_live)
#pragma unroll
          for (int p = 0; p < 4; ++p)
            a[i][p] = __builtin_bit_cast(bf16x8, As[st][p][wm + 16 * i + frow][slot]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        if (j < fn_live)
#pragma unroll
          for (int p = 0; p < 4; ++p)
            b[j][p] = __builtin_bit_cast(bf16x8, Bs[st][p][wn + 16 * j + frow][slot]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          if (FULL || (i < fm_live && j < fn_live)) {
            // planes: 0 re hi, 1 re lo, 2 im hi, 3 im lo
#define X3(acc, pa, pb)                                                                  \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][pa], b[j][pb], acc, 0, 0, 0);     \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][pa], b[j][pb + 1], acc, 0, 0, 0); \
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][pa + 1], b[j][pb], acc, 0, 0, 0);
            X3(acc1[i][j], 0, 0)
            X3(acc2[i][j], 2, 2)
            X3(acc3[i][j], 0, 2)
            X3(acc3[i][j], 2, 0)
#undef X3
          }
    }
  };

  // tiles whose fragments are all live (the common case) run a copy of the
  // walk without the per-fragment tests
  auto compute_full = [&](int st, int) { compute_t(st, std::true_type{}); };
  auto compute_part = [&](int st, int) { compute_t(st, std::false_type{}); };
  if (fm_live == FM && fn_live == FN)
    walk_chunks<F::BK, STAGES>(segs, tk.seg0, tk.nseg, load, store, compute_full);
  else
    walk_chunks<F::BK, STAGES>(segs, tk.seg0, tk.nseg, load, store, compute_part);

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + Mma<float>::row(lane, r);
        const int gn = n0 + wn + j * 16 + frow;
        if (gm < M && gn < N) {
          const int64_t idx = tk.c_off + (int64_t)gm * tk.ldc + gn;
          const float p1 = acc1[i][j][r], p2 = acc2[i][j][r], p3 = acc3[i][j][r];
          Cre[idx] = (TC)(p1 - p2);
          Cim[idx] = (TC)(FMT == PK_F32 ? p3 - p1 - p2 : p3);
        }
      }
}

template <int FMT, typename TC, int BM, int BN>
static void launch_p(const PackedLaunch& g, hipStream_t s) {
  constexpr int EB = Fmt<FMT>::EB;
  hipLaunchKernelGGL((packed_gemm_kernel<FMT, TC, BM, BN>), dim3(g.ntiles), dim3(NT), 0, s,
                     g.tasks, g.segs, g.tiles, g.ntiles, static_cast<const char*>(g.a),
                     g.a_plane * EB, static_cast<const char*>(g.b), g.b_plane * EB,
                     static_cast<TC*>(g.c_re), static_cast<TC*>(g.c_im));
}

template <int FMT, typename TC>
static bool launch_ptiles(const PackedLaunch& g, hipStream_t s) {
  switch (g.tile_cfg) {
    case 0: launch_p<FMT, TC, 64, 64>(g, s); return true;
    case 1: launch_p<FMT, TC, 32, 32>(g, s); return true;
    case 2: launch_p<FMT, TC, 128, 64>(g, s); return true;
    case 3: launch_p<FMT, TC, 64, 128>(g, s); return true;
    case 4:
      if constexpr (FMT == PK_F32) {
        launch_p<FMT, TC, 128, 128>(g, s);
        return true;
      }
      return false;
    default: return false;
  }
}

bool launch_packed_gemm(const PackedLaunch& g, hipStream_t s) {
  if (g.ntiles <= 0) return true;
  if (g.fmt == PK_F32)
    return g.c_t == ET_F32 ? launch_ptiles<PK_F32, float>(g, s)
                           : launch_ptiles<PK_F32, double>(g, s);
  if (g.fmt == PK_BF16X3)
    return g.c_t == ET_F32 ? launch_ptiles<PK_BF16X3, float>(g, s)
                           : launch_ptiles<PK_BF16X3, double>(g, s);
  return false;
}

}  // namespace tnt
