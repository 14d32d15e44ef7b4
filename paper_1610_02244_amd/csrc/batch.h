// Batches of independent two-site problems (different chains, bonds, block
// structures) driven through one merged H_eff operator: one grouped launch
// per contraction step for all instances, and a Lanczos recurrence whose
// vector operations are segmented per instance.
#pragma once

#include <memory>
#include <vector>

#include "lanczos.h"

namespace tnt {

// Device copy of a run list, re-uploaded only when the list changes (the
// host list stays alive with the table, so no wait is needed after an
// upload; an event guards against rewriting it while a copy is pending).
struct RunTable {
  std::vector<CopyRun> host;
  DevBuf dev;
  int64_t max_count = 0;
  hipEvent_t done = nullptr;
  ~RunTable();
  // enqueue the copies of `runs` on the context stream
  void run(Ctx& c, const std::vector<CopyRun>& runs);
};

struct BatchHeff {
  std::shared_ptr<HeffOp> op;       // merged operator over the batch vector
  std::vector<BatchPart> parts;     // per instance
  std::vector<int64_t> n;           // complex entries per instance
  std::vector<int64_t> L_ext, R_ext;
  int64_t N = 0, L_tot = 0, R_tot = 0;
  DevBuf envs;                      // [L re | L im | R re | R im] of all instances
  RunTable env_runs;
  SegLayout seg;
  int precision = TNT_FP64;
  int ninst() const { return (int)n.size(); }
};

// Merge the per-instance operators (each built for its own theta layout,
// n[i] complex entries) into one batch operator; instance i's vector goes to
// complex offset sum_{j<i} n[j].
void build_batch(Ctx& c, BatchHeff& b, const std::vector<std::shared_ptr<HeffOp>>& ops,
                 const std::vector<int64_t>& n, int prec);
// The same from the instances' host plans (no per-instance device tables);
// L_ext / R_ext: each instance's environment extents; tunable: as for
// HeffOp::build_plan (off for an operator used once).
void build_batch_plans(Ctx& c, BatchHeff& b, const std::vector<const HeffPlan*>& plans,
                       const std::vector<int64_t>& L_ext, const std::vector<int64_t>& R_ext,
                       const std::vector<int64_t>& n, int prec, bool tunable);
// Gather every instance's FP64 environments into the batch planes and bind
// them (refreshes the packed copies).
void bind_batch_envs(Ctx& c, BatchHeff& b, const std::vector<const double*>& Lre,
                     const std::vector<const double*>& Lim, const std::vector<const double*>& Rre,
                     const std::vector<const double*>& Rim);

// Batched lowest eigenpairs: x (re plane of N doubles, then im plane) holds
// the start vectors on entry and the normalised ground vectors on exit;
// out[i] per instance (steps, Ritz and refined energies, residual).
void lanczos_run_batched(Ctx& c, BatchHeff& b, BatchKrylov& K, double* x,
                         const tnt_lanczos_params& p, std::vector<LanczosOut>& out,
                         Timers* tm);

}  // namespace tnt
