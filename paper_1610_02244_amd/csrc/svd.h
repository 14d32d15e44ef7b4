// Truncated SVD of a two-site vector with U(1) sectors.
#pragma once

#include <functional>
#include <memory>
#include <vector>

#include "layout.h"

namespace tnt {

// Site-tensor layout A[x, s, y]: key (q_x, s) -> block dim(q_x) x dim(q_x + s).
struct SiteH {
  std::map<std::pair<int, int>, BlockRef> blocks;
  int64_t elems = 0;
};
// Canonical packed site layout: ascending (q, s) over every allowed block.
SiteH make_site(const Bond& left, const Bond& right, int d);

struct SvdOut {
  Bond bond;                 // new middle bond (kept dims per sector)
  SiteH A, B;                // packed layouts of the two factors
  std::vector<double> lam;   // kept singular values, sectors ascending (renormalised)
  int chi = 0;
  double eps = 0, lambda0 = 0, norm_kept = 0;
  int levels = 1;            // deflation levels used to resolve the spectrum
};

// Output planes for the factors, provided once the kept bond is known.
struct FactorPlanes {
  double *a_re = nullptr, *a_im = nullptr, *b_re = nullptr, *b_im = nullptr;
};
using FactorAlloc = std::function<FactorPlanes(const SvdOut&)>;

// The context's rocBLAS handle (created on first use) bound to its stream.
void* blas_handle(Ctx& c);
// Device workspace bytes held by the context's rocBLAS / rocSOLVER handles.
int64_t blas_workspace_bytes(const Ctx& c);

// Selection of the kept count (host); see tnt_trunc_select.
int trunc_select(const double* lam, int n, const tnt_trunc_params& p, double* eps);
double trunc_error(const double* lam, int n, int kind);

// theta (FP64 planes in layout th) -> factors A[a, s1, c], B[c, s2, b]
// written packed into the planes `alloc` returns (it may throw to abort
// before anything is written).  Rows of sector m are the (s1, q_a) pairs and
// columns the (s2, q_b) pairs present among theta's blocks with q_a + s1 = m.
SvdOut svd_truncate_dev(Ctx& c, const ThetaH& th, const double* re, const double* im,
                        const tnt_trunc_params& p, int absorb, const FactorAlloc& alloc);

// The same in phases, so that the eigendecompositions of several thetas
// share batched calls: svd_begin launches the sector Gram matrices of one
// theta (its planes must stay valid until svd_finish), svd_eig decomposes
// every sector of every job, svd_refine resolves the small singular values
// by deflation (levels of smaller eigenproblems, batched across the jobs;
// job i is cut with p[i]), svd_finish selects the kept values and writes
// the factors.
struct SvdJob;
std::shared_ptr<SvdJob> svd_begin(Ctx& c, const ThetaH& th, const double* re, const double* im,
                                  int absorb);
void svd_eig(Ctx& c, const std::vector<SvdJob*>& jobs);
void svd_refine(Ctx& c, const std::vector<SvdJob*>& jobs,
                const std::vector<tnt_trunc_params>& p);
SvdOut svd_finish(Ctx& c, SvdJob& job, const tnt_trunc_params& p, const FactorAlloc& alloc);

// Deflation levels the last svd_refine used for a job (1 = no refinement).
int svd_levels(const SvdJob& job);

}  // namespace tnt
