// Device task descriptors and kernel launch entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tnt {

// One K-segment of a grouped complex GEMM: the tile's accumulator gets
// op(A)[M x K] * op(B)[K x N] added, A and B read from the operand planes at
// the given element offsets.  Segments of one task are summed in order.
struct GemmSeg {
  int64_t a_off;
  int64_t b_off;
  int32_t K;
  int32_t lda;
  int32_t ldb;
  int32_t pad;
};

// One output block C[M x N] (row-major, leading dimension ldc) = sum of its
// segments.  A task with no segment writes zeros.
struct GemmTask {
  int64_t c_off;
  int32_t M, N, ldc;
  int32_t seg0, nseg;
  int32_t pad;
};

// Elementwise linear combination dst = sum_t coef_t * src_t over `size`
// elements (used for the sparse MPO contractions).
struct CombTask {
  int64_t dst_off;
  int32_t size;
  int32_t term0;
  int32_t nterm;
  int32_t pad;
};
struct CombTerm {
  int64_t src_off;
  double coef;
};

// Operand-form selectors for the grouped GEMM.
enum GemmForm {
  FORM_NN = 0,   // C = A B           (A: M x K rows, B: K x N rows)
  FORM_NT = 1,   // C = A B^T         (B stored N x K)
  FORM_CN = 2,   // C = A^H B         (A stored K x M, conjugated)
  FORM_cNT = 3,  // C = conj(A) B^T   (A stored M x K, conjugated; B stored N x K)
};

// Element types of operands / result.
enum ElemType { ET_F64 = 0, ET_F32 = 1 };

// Compute path of the grouped GEMM.
enum GemmPath { PATH_F64 = 0, PATH_F32 = 1, PATH_BF16X3 = 2 };

struct GemmLaunch {
  const GemmTask* tasks;
  const GemmSeg* segs;
  const int2* tiles;      // (task, tm | tn << 16) per tile, in dispatch order
  int32_t ntiles;
  int32_t tile_cfg;       // tile-shape id (see gemm_tile_dims)
  const void* a_re; const void* a_im; ElemType a_t;
  const void* b_re; const void* b_im; ElemType b_t;
  void* c_re; void* c_im; ElemType c_t;
  GemmForm form;
  GemmPath path;
};

// ---------------------------------------------------------------------------
// Packed operands of the reduced-precision H_eff paths.  Every block is
// row-major with the contracted index k contiguous, its row stride a
// multiple of 8 elements, its offset a multiple of 8 and its padding columns
// zero, so a loader moves 16 aligned bytes per row and plane in one
// instruction.  A packed buffer holds its planes back to back with a common
// plane stride (elements, a multiple of 8):
//   PK_F32:    float  planes (re, im);
//   PK_BF16X3: bf16   planes (re hi, re lo, im hi, im lo) of the split
//              x = hi + lo, hi = bf16(x), lo = bf16(x - hi).
// ---------------------------------------------------------------------------
enum PackFmt { PK_F32 = 0, PK_BF16X3 = 1 };
inline int pack_planes(PackFmt f) { return f == PK_F32 ? 2 : 4; }
inline int pack_elem_bytes(PackFmt f) { return f == PK_F32 ? 4 : 2; }
inline int64_t pad8(int64_t x) { return (x + 7) & ~int64_t(7); }

// One block copied from FP64 split planes into a packed buffer:
// dst(r, c) = src(c, r) if trans else src(r, c), for r < rows, c < cols of
// the destination; columns cols .. dld-1 are written as zero.
struct PackTask {
  int64_t src_off, dst_off;
  int32_t rows, cols;
  int32_t sld, dld;
  int32_t trans;
  int32_t pad;
};
constexpr int PACK_TILE = 32;  // destination tile edge of the pack kernel
// tiles[i] = (task, tile row | tile col << 16)
void launch_pack(const PackTask* tasks, const int2* tiles, int ntiles, const double* sre,
                 const double* sim, void* dst, int64_t plane, PackFmt f, hipStream_t s);

// One slab of the packed MPO combination: dst(r, c) = sum_t coef_t
// src_t[r * cols + c] (FP32 sources, unpadded) for c < cols, zero for
// cols <= c < dld; chunks of COMB_CHUNK destination elements.
struct CombPTask {
  int64_t dst_off;
  int32_t rows, cols, dld;
  int32_t term0, nterm;
  int32_t pad;
};
void launch_combine_packed(const CombPTask* tasks, const CombTerm* terms, const int2* chunks,
                           int32_t nchunks, const float* src_re, const float* src_im, void* dst,
                           int64_t plane, PackFmt f, hipStream_t s);

// Grouped GEMM on packed operands: C = A B^T, A (M x K) and B (N x K) both
// packed (lda, ldb are the packed row strides); C written as TC planes.
struct PackedLaunch {
  const GemmTask* tasks;
  const GemmSeg* segs;
  const int2* tiles;
  int32_t ntiles;
  int32_t tile_cfg;
  const void* a; int64_t a_plane;
  const void* b; int64_t b_plane;
  void* c_re; void* c_im; ElemType c_t;
  PackFmt fmt;
};
// false when the format / tile shape / output type is not built
bool launch_packed_gemm(const PackedLaunch& g, hipStream_t s);

// Tile shapes available to the planner: returns BM, BN for a config id.
void gemm_tile_dims(int cfg, int* bm, int* bn);
int gemm_num_tile_cfgs();

// false when the (path, operand types, form, tile shape) combination is not
// built; nothing is launched then.
bool launch_grouped_gemm(const GemmLaunch& g, hipStream_t s);
bool gemm_cfg_valid(int cfg, GemmPath path);
bool bf16x3_available();

void launch_combine(const CombTask* tasks, const CombTerm* terms, const int2* chunks,
                    int32_t nchunks, const void* src_re, const void* src_im, void* dst_re,
                    void* dst_im, ElemType t, hipStream_t s);

constexpr int COMB_CHUNK = 1024;  // elements per workgroup of the combine kernel

// elementwise conversions / fills
void launch_convert(const void* src, ElemType st, void* dst, ElemType dt, int64_t n,
                    hipStream_t s);
void launch_fill_zero(void* dst, ElemType t, int64_t n, hipStream_t s);
void launch_scale(double* x, int64_t n, const double* scale_dev, hipStream_t s);
void launch_scale_host(double* x, int64_t n, double scale, hipStream_t s);

// Krylov vector kernels.  A vector of n complex entries is stored as 2n
// doubles: re plane then im plane.  Reductions are two-stage and
// deterministic (fixed per-block order, then one block reduces the partials).
constexpr int RED_BLOCKS = 512;
constexpr int RED_THREADS = 256;
// out[j] = sum over blocks b < nblk of partial[b * k2 + j], j < k2
void launch_reduce_partials(const double* partial, int k2, int nblk, double* out,
                            hipStream_t s);
// partial sums of |x|^2 over 2n doubles
void launch_norm2_partial(const double* x, int64_t n2, double* partial, hipStream_t s);
// finite check: flag[0] set to 1 if any non-finite among n doubles
void launch_check_finite(const double* x, int64_t n, int* flag, hipStream_t s);

// ---------------------------------------------------------------------------
// Segmented Krylov kernels of the batched recurrence (krylov_seg.hip).  A
// batch vector has a re plane of N doubles then an im plane; instance i owns
// complex entries [off_i, off_i + n_i).  Each workgroup owns one SegBlock
// (a range inside one instance); inst_blk[i] = the instance's block range.
// Per-instance scalars are read / written at base + inst * stride.
// ---------------------------------------------------------------------------
struct SegBlock {
  int32_t inst;
  int32_t pad;
  int64_t lo, hi;  // complex entry range
};
void launch_seg_reduce(const double* partial, int k2, const int2* inst_blk, int ninst,
                       double* out, int out_stride, hipStream_t s);
void launch_seg_axpy2(const double* v1, const double* a, int a_stride, const double* v0,
                      const double* b, int b_stride, double* w, int64_t N, const SegBlock* blk,
                      int nblk, hipStream_t s);
void launch_seg_norm2(const double* x, int64_t N, const SegBlock* blk, int nblk, double* part,
                      hipStream_t s);
// mode 0: dst = src * scale_i; mode 1: dst = src / sqrt(scale_i) (0 if <= 0)
void launch_seg_scale_copy(const double* src, double* dst, int64_t N, const SegBlock* blk,
                           int nblk, const double* scale, int stride, int mode, hipStream_t s);
void launch_seg_combine_basis(const double* V, int64_t ld, int k, const double* y, int y_stride,
                              double* out, int64_t N, const SegBlock* blk, int nblk,
                              hipStream_t s);
// Fused recurrence steps over k = 1 .. 32 basis vectors V_0 .. V_{k-1}.
// Each kernel leaves per-workgroup partial sums part[b * W + o] (W = 2k
// values for projections, 1 for norms; nblk * W doubles) and the next
// kernel adds up its instance's partials itself, in a fixed order.
// Partials of c = V^H w, (re, im) pairs:
void launch_seg_cgs_dot(const double* V, int64_t ld, int k, const double* w, int64_t N,
                        const SegBlock* blk, int nblk, double* part, hipStream_t s);
// c = instance sum of part_in; w -= V c; partials of V^H w into part_out;
// the pair of V_{k-1} in c goes to pair_dst + inst * S when pair_dst is set.
void launch_seg_cgs_update_dot(const double* V, int64_t ld, int k, const double* part_in,
                               double* w, int64_t N, const SegBlock* blk, const int2* inst_blk,
                               int nblk, double* part_out, double* pair_dst, int S,
                               hipStream_t s);
// c = instance sum of part_in; w -= V c; partials of |w|^2 into part_out.
void launch_seg_cgs_update_norm(const double* V, int64_t ld, int k, const double* part_in,
                                double* w, int64_t N, const SegBlock* blk, const int2* inst_blk,
                                int nblk, double* part_out, hipStream_t s);
// nrm2 = instance sum of part_in (one value per workgroup); in instance i's
// scalar block sc + i * S: nrm2, beta_j = sqrt(nrm2), scale_j = 1 / beta_j
// unless j >= kmax[i] - 1 or beta_j <= tol * max(1, |alpha_0|) or is not
// finite (then 0); dst = w * scale_j when dst is set.
void launch_seg_cgs_next(const double* part_in, const double* w, double* dst, int64_t N,
                         const SegBlock* blk, const int2* inst_blk, int nblk, double* sc, int S,
                         int nrm2_slot, int alpha0_slot, int beta_slot, int scale_slot, double tol,
                         int j, const int* kmax, hipStream_t s);
// contiguous runs of doubles between device buffers (gathers / scatters)
struct CopyRun {
  const double* src;
  double* dst;
  int64_t count;
};
void launch_copy_runs(const CopyRun* runs, int nruns, int64_t max_count, hipStream_t s);

// Scatter from an interleaved complex matrix into row-major split-plane
// blocks: dst(r, c) = f(src[src_off + r * rs + c * cs]) for r < rows,
// c < cols, where f conjugates when `conj` is set (strides in complex
// elements, possibly negative); with `lower` set, entries with c > r are
// written as zero (the conjugate transpose of an upper-triangular factor).
struct ScatterTask {
  int64_t src_off;
  int64_t rs, cs;
  int64_t dst_off;   // element offset in the destination planes
  int32_t rows, cols;
  int32_t conj;
  int32_t lower;
};
// Gather row-major split-plane blocks into an interleaved complex matrix:
// z[dst_off + r * drs + c * dcs] = f(src(r, c)).
struct GatherTask {
  int64_t src_off;   // element offset of the row-major block in the planes
  int64_t dst_off;   // complex offset
  int64_t drs, dcs;
  int32_t rows, cols;
  int32_t conj;
  int32_t pad;
};
void launch_gather_z(const GatherTask* t, int ntask, int maxrows, int maxcols,
                     const double* re, const double* im, double* z, hipStream_t s);
void launch_scatter_z(const ScatterTask* t, int ntask, int maxrows, int maxcols,
                      const double* src_z, double* re, double* im, hipStream_t s);
// Padded batches of Hermitian matrices (interleaved complex, column-major).
// embed maps an n x n Gram matrix G at src into the npad x npad slot at dst
// as Q diag(G, D) Q / s (D negative, distinct, below G's spectrum; Q a fixed
// Householder reflector that leaves no exact split in the tridiagonal
// reduction; s = trace G, written to *scale: the library eigensolver's
// tolerances are not scale invariant, so every slot is solved at unit
// scale), using vec (2 npad doubles per slot at 2 w_src) as work space;
// extract takes G's eigenpairs back from the slot's ascending eigenpairs (the
// last n values times s, their vectors mapped through Q, first n rows) into an n x n
// eigenvector matrix at z + src_off and n eigenvalues at w + w_dst.  Every task
// names its own z and w, so one batch can serve several thetas.
// One dot product of the observables pass: out[2t], out[2t+1] = re, im of
// coef * sum_{e < n} x[x_off + e] conj(y[y_off + e]).
struct DotTask {
  int64_t x_off, y_off;
  int32_t n;
  int32_t pad;
  double coef;
};
void launch_block_dots(const DotTask* tasks, int ntask, const double* xre, const double* xim,
                       const double* yre, const double* yim, double* out, hipStream_t s);

// Two-site gate on theta (TEBD): destination block t = sum over its terms
// of (cr + i ci) * source block, elementwise over `size` elements; chunks
// are (task, chunk index) pairs of GATE_CHUNK elements.
constexpr int GATE_CHUNK = 1024;
struct GateTask {
  int64_t dst_off;
  int32_t size;
  int32_t term0, nterm;
  int32_t pad;
};
struct GateTerm {
  int64_t src_off;
  double cr, ci;
};
void launch_gate_apply(const GateTask* tasks, const GateTerm* terms, const int2* chunks,
                       int nchunks, const double* sre, const double* sim, double* dre,
                       double* dim, hipStream_t s);

// Automatic blocking: mask[i n + j] = |a_ij|^2 > tol^2 for an m x n matrix
// (row stride ld); and a block copy dst(r, c) = src(r, c) for r < rows,
// c < cols, where a row (column) index of either side is idx[list + r] when
// its list offset is >= 0, else r (source) or base + r (destination);
// entries with |x|^2 <= tol2 are copied as zero (tol2 < 0: none).
// rows[i] = (task, row) pairs, one workgroup each.
struct IndexCopyTask {
  int64_t src_off, src_ld;
  int64_t dst_off, dst_ld;
  int32_t src_ridx, src_cidx;
  int32_t dst_ridx, dst_cidx;
  int32_t dst_rbase, dst_cbase;
  int32_t rows, cols;
  double tol2;
};
void launch_nonzero_mask(const double* re, const double* im, int m, int n, int64_t ld,
                         double tol, unsigned char* mask, hipStream_t s);
void launch_index_copy(const IndexCopyTask* tasks, const int2* rows, int nrows,
                       const int32_t* idx, const double* sre, const double* sim, double* dre,
                       double* dim, hipStream_t s);

struct PadTask {
  double* z;         // the matrix's job buffer: interleaved Gram in, eigenvectors out
  double* w;         // the job's eigenvalue buffer
  int64_t src_off;   // complex offset of the n x n matrix in z
  int64_t dst_off;   // complex offset of the npad x npad slot
  int64_t w_src;     // offset of the slot's npad eigenvalues (and work vector)
  int64_t w_dst;     // offset of the sector's n eigenvalues in w
  int32_t n, npad;
  double* scale;     // padded path: the slot's scale factor (written by embed)
};
// Small sectors (n <= EIG_SMALL_MAX): eigenpairs of the Hermitian matrix at
// z + src_off (interleaved, column-major, upper triangle used), ascending
// values into w + w_dst and their vectors over the matrix, by cyclic Jacobi
// in LDS, one workgroup per task (max_n: the largest n of the tasks, <=
// EIG_SMALL_MAX); info[i] = 0 when task i converged, else 1.  Only z, w,
// src_off, w_dst and n of a task are read.
constexpr int EIG_SMALL_MAX = 32;
void launch_eig_small(const PadTask* t, int ntask, int max_n, int* info, hipStream_t s);
void launch_pad_embed(const PadTask* t, int ntask, int max_n, int max_npad, double* vec,
                      double* dst_z, hipStream_t s);
void launch_pad_extract(const PadTask* t, int ntask, int max_n, const double* slot_z,
                        const double* slot_w, hipStream_t s);

// Grouped complex GEMM (zgemm_grouped.hip): one 64 x 64 tile of
// C = op(A) B (sub = 0) or C -= op(A) B (sub = 1) per task, op(A) = A (opa = 0)
// or A^H (opa = 1); A, B, C interleaved complex FP64, column-major with the
// given leading dimensions; m x n is the whole product, (i0, j0) the tile's
// origin.  K is summed in increasing order within each tile.
struct ZTask {
  const double* A;
  const double* B;
  double* C;
  int32_t m, n, k, lda, ldb, ldc;
  int32_t i0, j0, opa, sub;
};
void launch_zgemm_grouped(const ZTask* tasks, int ntask, hipStream_t s);

// Householder reduction of a batch of Hermitian matrices of one order np to
// real symmetric tridiagonal form (LAPACK's lower convention: reflector k in
// A(k+2:, k) with A(k+1, k) = 1, scalars tau, diagonal d, off-diagonal e), in
// panels of TRD_NB columns; matrix b of the batch starts at A + b sA, and so
// on for every array.  Per column k of a panel starting at j0 (in-panel
// index i = k - j0, nbp columns): launch_trd_column, then launch_trd_gemv if
// k < np - 1; after the panel, if columns remain, launch_trd_column with
// do_col = 0 (finishes the panel's last W column) and the trailing update
// A(t0:, t0:) -= X(t0:, 0:2 nbp) X(t0:, nbp:3 nbp)^H (t0 = j0 + nbp), a
// complex GEMM left to the caller.  np <= TRD_MAX_N.
constexpr int TRD_NB = 32;
constexpr int TRD_MAX_N = 2048;
struct TrdBatch {
  double2* A;     // matrices, np x np, full storage, column-major (ld np)
  int64_t sA;
  double2* X;     // panel columns [V | W | V], np x 3 nbp (ld np)
  int64_t sX;
  double2* yp;    // partial products, ceil(np / 64) x np
  int64_t sY;
  double2* tp;    // partial dot products, ceil(np / 64) x 2 TRD_NB
  int64_t sT;
  double* d;      // np diagonal entries
  int64_t sd;
  double* e;      // np - 1 off-diagonal entries
  int64_t se;
  double2* tau;   // np - 1 reflector scalars
  int64_t stau;
  int np;
};
void launch_trd_column(const TrdBatch& b, int cnt, int j0, int nbp, int i, int do_col,
                       hipStream_t s);
void launch_trd_gemv(const TrdBatch& b, int cnt, int k, int i, int nbp, hipStream_t s);

// Column staging of the deflated SVD (interleaved complex, column-major):
// dst = scale * src over n complex values (one task per column), and the
// squared 2-norm of n complex values at src into *out (one workgroup per
// task, fixed summation order).
struct ZCopyTask {
  const double* src;
  double* dst;
  int64_t n;
  double scale;
};
struct ZNormTask {
  const double* src;
  double* out;
  int64_t n;
};
void launch_zcopy(const ZCopyTask* t, int ntask, int64_t max_n, hipStream_t s);
void launch_znorm2(const ZNormTask* t, int ntask, hipStream_t s);
// flags[t.slot] = 1 when any of t.x[0 .. t.n) is not finite (flags cleared
// by the caller)
struct FiniteTask {
  const double* x;
  int64_t n;
  int slot;
};
void launch_check_finite_batch(const FiniteTask* t, int ntask, int64_t max_n, int* flags,
                               hipStream_t s);

// z[2k] = re[k], z[2k+1] = (conj ? -im[k] : im[k]) for k < n
void launch_interleave(const double* re, const double* im, double* z, int64_t n, int conj,
                       hipStream_t s);

}  // namespace tnt
