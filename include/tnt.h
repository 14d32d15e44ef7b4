/*
 * libtnt_mi355x -- two-site DMRG hot path for 1D U(1)-symmetric MPS on one
 * AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows "The Tensor Network Theory Library"
 * (Al-Assam, Clark, Jaksch):
 *   - block tensors with U(1) charges: appendix A.1.1 (symmetric nodes: each
 *     leg is incoming or outgoing, only elements whose incoming charges sum
 *     to the outgoing charge are stored, one dense block per charge label);
 *   - the H_eff contractor handed to an eigensolver: Sec. 4.2;
 *   - the iterative lowest-eigenpair search driven by that contractor:
 *     Sec. 4.2 (network minimisation);
 *   - the truncated SVD, its four truncation rules and its error: appendix
 *     B.1.2 (Eq. trunc_err);
 *   - the variational sweep over an MPS with an MPO Hamiltonian: Sec. 4.3.
 *
 * Conventions shared by every call
 *   - Complex data are split into two real planes (re, im) of the same dtype.
 *     A block is stored row-major with the leg order given below; `offset`
 *     is the element offset of the block inside each plane.
 *   - Host metadata arrays are borrowed for the duration of the call only.
 *     Device planes are borrowed; the library never frees caller memory.
 *   - Every call is enqueued on the context's stream.  Calls that must
 *     inspect device results on the host (eigensolver, SVD, sweep) block
 *     until those results are available; tnt_heff2_apply does not block.
 *   - Status codes: 0 = OK, > 0 = warning (result valid), < 0 = error (no
 *     output written, or outputs unspecified).  tnt_last_error() gives a
 *     human-readable reason.  The library never prints and never aborts.
 *     A kernel fault surfaces as TNT_E_HIP at the next blocking call or
 *     tnt_sync().
 *   - Not thread safe per context: calls on one context must not overlap.
 */
#ifndef TNT_MI355X_H
#define TNT_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tnt_status;

enum {
  TNT_OK = 0,
  TNT_W_NOCONV = 1,      /* eigensolver residual above tolerance after kmax steps */
  TNT_E_ARG = -1,        /* invalid argument (null pointer, bad enum, bad size)    */
  TNT_E_SHAPE = -2,      /* block extents inconsistent between tensors           */
  TNT_E_CHARGE = -3,     /* a block violates the U(1) rule sum(in) = sum(out)     */
  TNT_E_CAPACITY = -4,   /* caller buffer too small                               */
  TNT_E_ALLOC = -5,      /* device allocation failed                              */
  TNT_E_NONFINITE = -6,  /* NaN or Inf found in an input or produced               */
  TNT_E_HIP = -7,        /* HIP runtime or library error                          */
  TNT_E_STATE = -8       /* object used in a wrong state                          */
};

/* arithmetic of the H_eff contraction */
enum { TNT_FP64 = 0, TNT_FP32 = 1, TNT_BF16X3 = 2 };
/* element type of a plane */
enum { TNT_DT_F64 = 0, TNT_DT_F32 = 1 };
/* where the singular values go after the SVD */
enum { TNT_ABSORB_RIGHT = 0, TNT_ABSORB_LEFT = 1 };
/* truncation error function (appendix B.1.2) */
enum { TNT_ERR_2NORM = 0, TNT_ERR_SUMSQ = 1, TNT_ERR_1NORM = 2 };

typedef struct tnt_ctx_s* tnt_ctx;

/* ------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------ */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  The context owns a caching
 * device-memory pool (workspaces, plans, MPS storage); it is released by
 * tnt_ctx_destroy.  Errors: TNT_E_ARG (out is NULL), TNT_E_HIP. */
tnt_status tnt_ctx_create(int32_t device, void* hip_stream, tnt_ctx* out);
void tnt_ctx_destroy(tnt_ctx ctx);
/* Reason for the last non-OK status on this context (never NULL). */
const char* tnt_last_error(tnt_ctx ctx);
/* Wait for all work enqueued by the context; TNT_E_HIP on a device fault. */
tnt_status tnt_sync(tnt_ctx ctx);
/* Bytes currently held by the context's device pool (in use + cached). */
int64_t tnt_pool_bytes(tnt_ctx ctx);
/* Device memory of the context in bytes (host query, no device work):
 * out[0] held by the pool (in use + cached), out[1] in use, out[2] the
 * most in use at once since the context was created, out[3] the device
 * workspace held by the library's rocBLAS / rocSOLVER handles.  The pool
 * keeps released blocks for reuse; before it allocates more it returns
 * its cached blocks to the runtime (a device synchronisation) when they
 * exceed both 4 GiB and the bytes in use, so out[0] stays below about
 * twice out[2] plus 4 GiB.  out is caller-owned host memory of 4 values.
 * Errors: TNT_E_ARG (null out). */
tnt_status tnt_ctx_memory(tnt_ctx ctx, int64_t* out);
/* Tile-shape autotuning of the H_eff grouped GEMMs (on by default): the
 * first application of a new block structure times every candidate tile
 * shape of each GEMM step of at least 1e9 flops and caches the choice per
 * shape bucket (smaller steps are launch-latency bound and take the
 * planner's default shape).  Results do not depend on the shape (the
 * summation order over K is the same).  on = 0 disables tuning (the
 * planner's default shape is used) and clears the cache. */
tnt_status tnt_ctx_set_autotune(tnt_ctx ctx, int32_t on);

/* HIP-graph execution of the Lanczos recurrence (off by default).  With
 * on = 1, tnt_lanczos_ground and the sweeps record the k matvec +
 * re-orthogonalisation steps of a bond once into a HIP graph (kept with the
 * cached operator, re-recorded when a workspace it uses was reallocated)
 * and replay it with one launch; results are identical to the eager path.
 * The sweeps then report no per-matvec device times (seconds_matvec,
 * seconds_gemm and gemm_launches stay 0).  Errors: TNT_E_ARG. */
tnt_status tnt_ctx_set_graphs(tnt_ctx ctx, int32_t on);

/* Tridiagonal reduction of the SVD's sector eigenproblems (Appendix B.1.2,
 * the node SVD; Gram matrices of the sectors, see tnt_theta_svd_truncate).
 * Problems whose padded order is >= min_order (and <= 2048) are reduced to
 * tridiagonal form by the library's own panel Householder kernels (two
 * launches per column) and finished by rocSOLVER's divide and conquer and
 * back-transformation; the others, and all of them with min_order = 0, go
 * through rocSOLVER's batched Hermitian eigensolver.  Both give the
 * eigenpairs to the backward error of a stable FP64 eigensolver, so kept
 * dimensions and truncation errors agree wherever the cut is decisive.
 * The default is 0: the library offers its divide and conquer and
 * back-transformation only one matrix per call, which costs more than the
 * reduction saves (a chi = 1024 sweep takes about twice as long with the
 * option from order 256 up).  A negative min_order restores the default.
 * Errors: none beyond a bad context. */
tnt_status tnt_ctx_set_eig_reduction(tnt_ctx ctx, int32_t min_order);

/* ------------------------------------------------------------------------
 * Block tensors (appendix A.1.1)
 *
 * Each block carries one integer label and one extent per leg.  Roles:
 *   theta  rank 4, legs (a, s1, s2, b), dir (+1, +1, +1, -1):
 *          labels (q_a, s1, s2, q_b), extents (dim_a, 1, 1, dim_b),
 *          rule q_b = q_a + s1 + s2.  Stored as a dim_a x dim_b matrix.
 *   L env  rank 3, legs (a', w, a), dir (-1, +1, +1): labels (q_a', w, q_a)
 *          where w is the MPO bond index (its charge is the MPO's
 *          bond_charge[w]), extents (dim_a', 1, dim_a), rule
 *          q_a' = q_a + bond_charge[w].  a' is the bra index.
 *   R env  same as L env with legs (b', u, b), rule q_b' = q_b + charge[u].
 * A block whose labels violate its rule is rejected with TNT_E_CHARGE.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t rank;
  int32_t nblocks;
  const int32_t* qn;      /* [nblocks * rank] host: labels                      */
  const int32_t* extent;  /* [nblocks * rank] host: extents                     */
  const int64_t* offset;  /* [nblocks] host: element offset of each block        */
  void* re;               /* device plane, dtype elements                        */
  void* im;               /* device plane                                        */
  int32_t dtype;          /* TNT_DT_F64 | TNT_DT_F32                             */
  int64_t capacity;       /* elements available in each plane                    */
} tnt_btensor;

/* One MPO site W[w, w', s', s] (Sec. 4.3: the Hamiltonian as a chain).
 * Host arrays, borrowed.  Every nonzero element must obey
 * s' - s = bond_charge[w'] - bond_charge[w]  (else TNT_E_CHARGE). */
typedef struct {
  int32_t d;                  /* physical dimension (labels s = 0..d-1 are the charges) */
  int32_t D;                  /* MPO bond dimension                                     */
  const int32_t* bond_charge; /* [D]                                                    */
  const double* W;            /* [D*D*d*d], index ((w*D + w')*d + s')*d + s              */
} tnt_mpo_site;

/* Bose-Hubbard MPO site (Sec. 5, Eq. 2 with V = 0; occupancy 0..nmax):
 * H = -J sum (b_j^+ b_{j+1} + h.c.) + sum (U/2 n_j (n_j - 1) - mu n_j).
 * Fills W (host, 16 d^2 doubles, d = nmax + 1, layout of tnt_mpo_site with
 * D = 4) and bond_charge[4] = (0, +1, -1, 0).  The chain operator uses the
 * left boundary index 3 and the right boundary index 0.  Host only.
 * Errors: TNT_E_ARG (nmax outside 0..63, NULL), TNT_E_NONFINITE. */
tnt_status tnt_mpo_bose_hubbard(int32_t nmax, double J, double U, double mu, double* W,
                                int32_t* bond_charge);

/* Spin-1 isotropic Heisenberg MPO site (the DMRG timing workload of Sec. 3,
 * Table tab:dmrgtimes): H = J sum S_j . S_{j+1}.  Local states s = m + 1 in
 * {0, 1, 2} (m = S^z), so the U(1) charge of a site is s and total S^z = 0
 * is total charge L.  Fills W (host, 225 doubles, layout of tnt_mpo_site
 * with d = 3, D = 5) and bond_charge[5] = (0, +1, -1, 0, 0).  The chain
 * operator uses the left boundary index 4 and the right boundary index 0.
 * Host only.  Errors: TNT_E_ARG (NULL), TNT_E_NONFINITE. */
tnt_status tnt_mpo_spin1_heisenberg(double J, double* W, int32_t* bond_charge);

/* Bond Hamiltonians for tnt_tebd_step: h (host, (L-1) d^4 doubles) gets
 * h_j, j = 1..L-1, as d^2 x d^2 row-major matrices with row s1' d + s2' and
 * column s1 d + s2, so that sum_j h_j = H.  Bose-Hubbard (Sec. 5, Eq. 2,
 * V = 0, d = nmax + 1): the bond's hopping plus the on-site terms of its
 * two sites, each shared equally with the site's other bond (an end site
 * puts its whole term on its only bond).  Spin-1 Heisenberg (d = 3):
 * h_j = J S_j . S_{j+1}.  Host only.  Errors: TNT_E_ARG, TNT_E_NONFINITE. */
tnt_status tnt_bond_hamiltonians_bose_hubbard(int32_t L, int32_t nmax, double J, double U,
                                              double mu, double* h);
tnt_status tnt_bond_hamiltonians_spin1(int32_t L, double J, double* h);

/* One-site H_eff . A (Sec. 4.2, the contractor, in its one-site form, as
 * used by single-site updates):
 *   out[a', s', b'] = sum L[a', w, a] W[w, u, s', s] R[b', u, b] A[a, s, b].
 * A and out are rank-3 site tensors: labels (q_a, s, q_b), extents
 * (dim_a, 1, dim_b), rule q_b = q_a + s, TNT_DT_F64, the same block set and
 * extents (offsets may differ).  L, R: environments as for tnt_heff2_apply.
 * FP64 arithmetic.  Output blocks no term reaches are written as zeros.
 * Synchronises the context's stream.  Errors: TNT_E_ARG, TNT_E_SHAPE,
 * TNT_E_CHARGE, TNT_E_CAPACITY. */
tnt_status tnt_heff1_apply(tnt_ctx ctx, const tnt_btensor* L, const tnt_mpo_site* W,
                           const tnt_btensor* R, const tnt_btensor* A, const tnt_btensor* out);

/* ------------------------------------------------------------------------
 * H_eff . theta (Sec. 4.2, the contractor, in two-site form)
 *
 *   out[a', s1', s2', b'] = sum L[a', w, a] W1[w, v, s1', s1] W2[v, u, s2', s2]
 *                               R[b', u, b] theta[a, s1, s2, b]
 *
 * theta and out: same block set and extents (offsets may differ), dtype
 * TNT_DT_F64.  L, R: TNT_DT_F64.  precision selects the arithmetic of the
 * contraction (TNT_FP64; TNT_FP32 = FP32 MFMA with FP32 accumulation;
 * TNT_BF16X3 = three-term bf16 split products with FP32 accumulation); the
 * result is always written as FP64.  Output blocks no term reaches are
 * written as zeros.  Asynchronous (no host wait).
 * Errors: TNT_E_ARG, TNT_E_SHAPE (extents disagree), TNT_E_CHARGE,
 * TNT_E_CAPACITY (a block runs past a plane's capacity), TNT_E_ALLOC.
 * ------------------------------------------------------------------------ */
tnt_status tnt_heff2_apply(tnt_ctx ctx, const tnt_btensor* L, const tnt_mpo_site* W1,
                           const tnt_mpo_site* W2, const tnt_btensor* R,
                           const tnt_btensor* theta, tnt_btensor* out, int32_t precision);

/* tnt_heff2_apply for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation).
 * Same operands, result and errors as tnt_heff2_apply; the operator's task
 * tables, intermediate slabs and packed operand copies are placed in one
 * device array of 64 MiB that the library holds on each GPU it runs on until
 * the process ends, so the call makes no device allocation (no hipMalloc,
 * hipFree or allocating library routine).  Operators whose tables and
 * workspaces exceed 64 MiB are refused with TNT_E_CAPACITY before anything
 * is launched (an FP64 two-site operator of a chi = 256 chain needs about
 * 25 MB).  Every call on one GPU reuses that GPU's array: calls that overlap
 * on one GPU (from two contexts or threads) race and give undefined results.
 * The plan is built on the host at every call, with default tile shapes (no
 * timing launches).  Synchronises the context's stream before returning. */
tnt_status tnt_heff2_apply_noalloc(tnt_ctx ctx, const tnt_btensor* L, const tnt_mpo_site* W1,
                                   const tnt_mpo_site* W2, const tnt_btensor* R,
                                   const tnt_btensor* theta, tnt_btensor* out,
                                   int32_t precision);

/* n independent applications (arrays of n operands, each with the meaning
 * of tnt_heff2_apply: different chains, bonds and block structures) packed
 * into one grouped launch per contraction step.  Inputs are gathered into a
 * batch vector and results scattered back; out[i] gets exactly what
 * tnt_heff2_apply would write.  Blocks until the copies are done.
 * Errors as for tnt_heff2_apply (the first failing instance decides). */
tnt_status tnt_heff2_apply_batched(tnt_ctx ctx, int32_t n, const tnt_btensor* const* L,
                                   const tnt_mpo_site* const* W1, const tnt_mpo_site* const* W2,
                                   const tnt_btensor* const* R, const tnt_btensor* const* theta,
                                   tnt_btensor* const* out, int32_t precision);

/* Algorithmic FLOP count of one tnt_heff2_apply on these block structures
 * (host only, no device access).  Counting rule: a complex multiply-add is
 * 8 flops, a real-times-complex term 4 flops per element; step 1 (L.theta
 * slabs that feed a nonzero MPO term), the MPO terms, and step 4 (. R).
 * Writes {step1, mpo, step4} to `parts` when non-NULL.  Returns the total,
 * or -1 on invalid input. */
int64_t tnt_heff2_flops(const tnt_btensor* L, const tnt_mpo_site* W1, const tnt_mpo_site* W2,
                        const tnt_btensor* R, const tnt_btensor* theta, int64_t* parts);

/* ------------------------------------------------------------------------
 * Lowest eigenpair of H_eff (Sec. 4.2, network minimisation; the initial
 * guess is the current theta).  Plain Lanczos in FP64: alpha/beta
 * recurrence with classical Gram-Schmidt against all previous Krylov
 * vectors, applied twice (the first pass also removes the three-term
 * part alpha_j v_j + beta_{j-1} v_{j-1}), stop at kmax steps
 * or when beta_j <= beta_tol * max(1, |alpha_0|); lowest Ritz pair of the
 * tridiagonal matrix; then one FP64 matvec for the Rayleigh quotient
 * E_refined and the residual |H psi - E psi|.  The matvecs inside the
 * iteration use `precision`; the refinement is always FP64.
 * theta (FP64) is the start vector on entry and the normalised ground
 * vector on exit.  Blocks until the result is on the host.
 * Returns TNT_W_NOCONV when residual > resid_tol (> 0) after kmax steps.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t kmax;        /* Krylov steps (1 .. 32)                */
  int32_t precision;   /* TNT_FP64 | TNT_FP32 | TNT_BF16X3      */
  double beta_tol;     /* breakdown tolerance (e.g. 1e-12)      */
  double resid_tol;    /* <= 0: never warn                      */
} tnt_lanczos_params;

typedef struct {
  double E_ritz;
  double E_refined;
  double residual;
  int32_t steps;
} tnt_lanczos_result;

tnt_status tnt_lanczos_ground(tnt_ctx ctx, const tnt_btensor* L, const tnt_mpo_site* W1,
                              const tnt_mpo_site* W2, const tnt_btensor* R,
                              tnt_btensor* theta, const tnt_lanczos_params* p,
                              tnt_lanczos_result* r);

/* The same for n independent problems at once (different chains, bonds,
 * block structures; arrays of n operands with the meaning above, one
 * parameter set for all, r[n] results).  Every recurrence step applies all n
 * operators with one grouped launch per contraction step, and the vector
 * work (dots, re-orthogonalisation, normalisation) runs segmented per
 * instance; each instance follows the single-problem recurrence (its own
 * step count min(kmax, dim), breakdown, Ritz vector and FP64 refinement).
 * Returns TNT_W_NOCONV when any instance misses resid_tol.  Errors as for
 * tnt_lanczos_ground (the first failing instance decides). */
tnt_status tnt_lanczos_ground_batched(tnt_ctx ctx, int32_t n, const tnt_btensor* const* L,
                                      const tnt_mpo_site* const* W1,
                                      const tnt_mpo_site* const* W2, const tnt_btensor* const* R,
                                      tnt_btensor* const* theta, const tnt_lanczos_params* p,
                                      tnt_lanczos_result* r);

/* ------------------------------------------------------------------------
 * Truncated SVD of theta (appendix B.1.2).
 *
 * For every middle charge m = q_a + s1, the matrix with rows (s1, a) and
 * columns (s2, b) (s ascending, then the sector's index) is decomposed in
 * FP64.  Singular values of all sectors are pooled and sorted descending
 * (ties: smaller m, then smaller index); the kept number chi is the
 * smallest allowed by the active rules: chi <= chi_max; lambda >= abs_tol
 * (if > 0); lambda/lambda_0 >= rel_tol (if > 0); the largest discard whose
 * error stays strictly below err_tol (if > 0); at least 1.
 * eps = error of the discarded values (err_type).  With renormalise != 0 the
 * kept values are scaled to unit 2-norm.
 *
 * Outputs (FP64 planes, written by the call):
 *   A[a, s1, c]: blocks (q_a, s1) in ascending (q_a, s1), extent
 *                (dim_a, kept(m)), rank-3 labels (q_a, s1, m);
 *   B[c, s2, b]: blocks (m, s2) in ascending (m, s2), labels (m, s2, q_b);
 *   absorb RIGHT: A = U, B = S V^+;  absorb LEFT: A = U S, B = V^+.
 *   Blocks are packed contiguously from offset 0 in the order above; the
 *   call writes nblocks, qn, extent and offset of A and B into the
 *   caller's arrays (capacity max_blocks each) and the kept (renormalised)
 *   singular values, sector by sector in ascending m, into S (capacity
 *   s_capacity); bond_q/bond_dim (capacity max_blocks) get the new bond.
 * Errors: TNT_E_CAPACITY when planes, metadata or S are too small
 * (nothing is written to the planes then), TNT_E_NONFINITE.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t chi_max;
  int32_t err_type;    /* TNT_ERR_*                     */
  double abs_tol;      /* <= 0: off                     */
  double rel_tol;      /* <= 0: off                     */
  double err_tol;      /* <= 0: off                     */
  int32_t renormalise; /* non-zero: unit 2-norm          */
} tnt_trunc_params;

typedef struct {
  int32_t max_blocks;  /* capacity of qn/extent (x3) and offset arrays  */
  int32_t nblocks;     /* written                                       */
  int32_t* qn;         /* [max_blocks*3] written                        */
  int32_t* extent;     /* [max_blocks*3] written                        */
  int64_t* offset;     /* [max_blocks] written                          */
  double* re;          /* device plane                                  */
  double* im;          /* device plane                                  */
  int64_t capacity;    /* elements per plane                            */
} tnt_site_out;

typedef struct {
  int32_t chi;         /* kept bond dimension           */
  int32_t nsectors;    /* sectors of the new bond       */
  double eps;          /* truncation error              */
  double lambda0;      /* largest singular value        */
  double norm_kept;    /* 2-norm of the kept values before renormalising */
} tnt_trunc_result;

tnt_status tnt_theta_svd_truncate(tnt_ctx ctx, const tnt_btensor* theta,
                                  const tnt_trunc_params* p, int32_t absorb,
                                  tnt_site_out* A, tnt_site_out* B,
                                  double* S, int32_t s_capacity,
                                  int32_t* bond_q, int32_t* bond_dim,
                                  tnt_trunc_result* r);

/* Host-only helper: the kept count the rules above give for a descending
 * spectrum `lam` of length n (no device access).  Returns chi >= 1, or -1
 * on invalid input; writes the truncation error to *eps when non-NULL. */
int32_t tnt_trunc_select(const double* lam, int32_t n, const tnt_trunc_params* p, double* eps);

/* ------------------------------------------------------------------------
 * MPS, environments and the sweep (Sec. 4.3, two-site form)
 *
 * An MPS handle owns device storage for L site tensors A_j[a, s, b]
 * (blocks (q_left, s), extents (dim(q_left), dim(q_left + s))) and their
 * bond sector tables; bond 0 holds one charge and bond L holds one charge.
 * ------------------------------------------------------------------------ */
typedef struct tnt_mps_s* tnt_mps;
typedef struct tnt_env_s* tnt_env;

/* Create an empty MPS of L sites with physical dimension d. */
tnt_status tnt_mps_create(tnt_ctx ctx, int32_t L, int32_t d, tnt_mps* out);
void tnt_mps_destroy(tnt_mps mps);
/* Set bond `ell` (0..L) to sectors q[i] of dimension dim[i] (ascending q). */
tnt_status tnt_mps_set_bond(tnt_mps mps, int32_t ell, int32_t nsec, const int32_t* q,
                            const int32_t* dim);
/* Upload site j (1..L) from host planes: blocks listed by (q_left[i], s[i]),
 * each dim(q_left) x dim(q_left + s) row-major, concatenated in list order.
 * Bonds j-1 and j must be set first.  Blocks not listed are zero. */
tnt_status tnt_mps_set_site(tnt_mps mps, int32_t j, int32_t nblocks, const int32_t* q_left,
                            const int32_t* s, const double* re, const double* im);
/* Number of sectors of bond ell, and its table (arrays of capacity cap). */
int32_t tnt_mps_bond_size(tnt_mps mps, int32_t ell);
tnt_status tnt_mps_get_bond(tnt_mps mps, int32_t ell, int32_t cap, int32_t* q, int32_t* dim);
/* Download site j: writes its blocks in ascending (q_left, s) into the
 * host arrays (block count capacity cap, element capacity ecap). */
tnt_status tnt_mps_get_site(tnt_mps mps, int32_t j, int32_t cap, int32_t* nblocks,
                            int32_t* q_left, int32_t* s, int64_t ecap, double* re, double* im);
/* Bring the MPS to right-canonical form (sites L..2 right isometries,
 * norm carried by site 1, then site 1 scaled to unit norm), by Householder
 * QR of each left sector's (a) x (s, b) matrix on the device (no truncation;
 * a sector shrinks to its rank bound min(rows, cols)); every absorbed factor
 * is rescaled to unit norm on the way, so long chains cannot overflow. */
tnt_status tnt_mps_right_canonicalize(tnt_ctx ctx, tnt_mps mps);

/* One TEBD time step (time evolution by two-site Trotter gates, Sec. 1 and
 * the example of Sec. 5, Fig. fig:time_evolve_results): with the bond
 * Hamiltonians h (host, layout of tnt_bond_hamiltonians_*; each real
 * symmetric and charge-conserving), applies exp(-i h_j dt/2) to
 * theta = A_j B_{j+1} and splits it by the truncated SVD (`trunc`,
 * appendix B.1.2) for j = 1..L-1 (centre moving right), then for
 * j = L-1..1 (centre moving back): a second-order Trotter step.  The MPS
 * must be right-canonical with its centre on site 1 (tnt_mps_right_
 * canonicalize, a product state, or the state a sweep or a previous step
 * leaves) and is left the same way.  bond_eps / bond_chi (host, may be
 * NULL, capacity record_cap >= 2(L-1)) receive the truncation error and
 * kept dimension of each gate in order; stats (host, may be NULL, 6
 * doubles): seconds total, seconds theta + gate, seconds SVD, sum of the
 * truncation errors, largest truncation error, largest kept chi.
 * Synchronises the context's stream.  Errors: TNT_E_ARG (NULL, chi_max < 1,
 * h not symmetric), TNT_E_CHARGE (h mixes charges), TNT_E_CAPACITY,
 * TNT_E_STATE (a site not set), TNT_E_NONFINITE. */
tnt_status tnt_tebd_step(tnt_ctx ctx, tnt_mps mps, const double* h, double dt,
                         const tnt_trunc_params* trunc, int32_t record_cap, double* bond_eps,
                         int32_t* bond_chi, double* stats);

/* Truncated SVD of a matrix with no known symmetry through automatic
 * blocking (the library's auto-blocking mode, Fig. fig:autoblocking, Table
 * tab:tebdtimes): entries with |a_ij| <= tol are dropped; rows and columns
 * are grouped into the connected components of the bipartite graph of the
 * remaining entries (the block-diagonal form after permutations); every
 * block gets the block SVD of the U(1) sectors, and all blocks' singular
 * values are cut together by `trunc` (appendix B.1.2).
 * a_re / a_im: device planes, m x n, row stride lda >= n (borrowed).
 * Outputs (device planes, overwritten): U (m rows, stride ldu >= chi_max)
 * with orthonormal columns, B = S V^+ (chi_max rows, stride ldb >= n), so
 * that U B is the truncated matrix (renormalised if trunc->renormalise);
 * columns of U / rows of B beyond chi are zero.  Host outputs: S (chi_max
 * doubles: the kept singular values, grouped by block in the order of each
 * block's smallest row index, descending within a block, column c of U
 * belonging to S[c]), chi, nblocks (may be NULL), eps (may be NULL:
 * truncation error of the trunc->err_type kind).  Singular values below
 * about 1e-7 of the largest are not resolved (they count as zero).
 * Synchronises the context's stream.  Errors: TNT_E_ARG (NULL, shapes,
 * strides, chi_max < 1, tol < 0), TNT_E_NONFINITE. */
tnt_status tnt_auto_block_svd(tnt_ctx ctx, const double* a_re, const double* a_im, int32_t m,
                              int32_t n, int64_t lda, double tol, const tnt_trunc_params* trunc,
                              double* u_re, double* u_im, int64_t ldu, double* b_re,
                              double* b_im, int64_t ldb, double* S, int32_t* chi,
                              int32_t* nblocks, double* eps);

/* Two-point correlations of the state for every pair of sites (the outputs
 * of the ground-state example of Sec. 5, Fig. fig:ground_state_results):
 *   out[(i-1) L + (j-1)] = <psi| O^dagger_i O_j |psi> / <psi|psi>,
 * i, j = 1..L, with i = j giving <(O^dagger O)_i>.  With O = b this is the
 * single-particle density matrix rho_ij = <b^dagger_i b_j>, whose diagonal
 * is the density <n_j>.  `op` (host, d*d doubles, op[s' d + s] = <s'|O|s>,
 * real) may be nonzero only where s' - s = dq.  out_re / out_im: host,
 * L*L doubles each (the matrix is Hermitian; both triangles are filled).
 * flops (host, may be NULL) receives the pass's algorithmic flops.  Any
 * gauge of the MPS is accepted and it is left unchanged.  Runs one
 * left-to-right pass of FP64 grouped GEMMs over all open strings at once
 * and synchronises the context's stream.  Errors: TNT_E_ARG (NULL),
 * TNT_E_STATE (a site not set, zero norm), TNT_E_CHARGE (an entry of op
 * breaks dq), TNT_E_NONFINITE. */
tnt_status tnt_mps_correlation(tnt_ctx ctx, tnt_mps mps, const double* op, int32_t dq,
                               double* out_re, double* out_im, double* flops);

/* Environments of a right-canonical MPS for the chain MPO `mpo` (L sites,
 * borrowed only during this call: the handle keeps its own copy).  Left
 * boundary selects MPO index `left_index`, right boundary `right_index`. */
tnt_status tnt_env_create(tnt_ctx ctx, tnt_mps mps, const tnt_mpo_site* mpo,
                          int32_t left_index, int32_t right_index, tnt_env* out);
void tnt_env_destroy(tnt_env env);

typedef struct {
  tnt_lanczos_params lanczos;
  tnt_trunc_params trunc;
  int32_t record_cap;  /* capacity of the per-bond arrays below (>= 2(L-1)) */
  double* bond_E;      /* [record_cap] FP64 Rayleigh energy per bond update, may be NULL */
  double* bond_eps;    /* [record_cap] truncation error, may be NULL        */
  int32_t* bond_chi;   /* [record_cap] kept chi, may be NULL                */
  int32_t* bond_steps; /* [record_cap] Lanczos steps, may be NULL           */
} tnt_sweep_params;

typedef struct {
  double energy;          /* E of the last bond update                      */
  double max_residual;
  double max_eps;
  int32_t updates;        /* bond updates done = 2(L-1)                     */
  int32_t max_chi;
  int64_t matvecs;        /* H_eff applications in the iteration            */
  double matvec_flops;    /* algorithmic flops of those matvecs              */
  double seconds_total;   /* host wall time of the sweep                     */
  double seconds_matvec;  /* device time of the iteration matvecs            */
  double seconds_lanczos; /* device time of the Krylov vector work           */
  double seconds_svd;     /* wall time of the SVD-truncate steps             */
  double seconds_env;     /* wall time of environment updates                */
  double gemm_flops;      /* algorithmic flops of the iteration matvecs' grouped-GEMM launches */
  double seconds_gemm;    /* device time of those launches (HIP events)      */
  int64_t gemm_launches;  /* number of those launches                        */
  double seconds_theta;   /* wall time of theta formation                   */
  double seconds_setup;   /* wall time of H_eff plan lookup or build,
                             environment packing and Krylov reservation     */
  int64_t eig_retries;    /* sector eigenproblems of the SVD steps redone with
                             the Jacobi eigensolver after divide and conquer
                             failed or returned non-finite vectors          */
} tnt_sweep_result;

/* One sweep: right pass over bonds 1..L-1 then left pass L-1..1 (each:
 * theta formation, Lanczos, SVD-truncate, environment update), in place on
 * `mps` and `env`.  Blocks until done. */
tnt_status tnt_dmrg_sweep(tnt_ctx ctx, tnt_mps mps, tnt_env env, const tnt_sweep_params* p,
                          tnt_sweep_result* r);

/* One sweep of each of n independent chains (different L, chi, couplings):
 * the chains advance in lockstep, one bond update per chain per step, and
 * the Lanczos problems of all chains active at a step run as one batch
 * (tnt_lanczos_ground_batched); theta formation, SVD-truncate and the
 * environment update stay per chain.  p[i] and r[i] per chain (truncation
 * and record arrays may differ; the Lanczos parameters must agree, else
 * TNT_E_ARG).  Each chain ends exactly as tnt_dmrg_sweep would leave it,
 * up to rounding.  The timing fields of every r[i] are totals of the whole
 * batch.  Blocks until done. */
tnt_status tnt_dmrg_sweep_batched(tnt_ctx ctx, int32_t n, const tnt_mps* mps, const tnt_env* env,
                                  const tnt_sweep_params* p, tnt_sweep_result* r);

#ifdef __cplusplus
}
#endif
#endif /* TNT_MI355X_H */
