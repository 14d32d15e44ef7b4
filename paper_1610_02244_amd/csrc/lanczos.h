// Lanczos eigensolver state and driver.
#pragma once

#include <vector>

#include "plan.h"

namespace tnt {

// Block table of the segmented Krylov kernels over a batch vector.
struct SegLayout {
  std::vector<SegBlock> blk;
  std::vector<int2> inst_blk;  // per instance: [first, last) block
  DevBuf dev;                  // blk then inst_blk
  int nblk = 0;
  const SegBlock* d_blk() const { return dev.as<SegBlock>(); }
  const int2* d_inst() const {
    return reinterpret_cast<const int2*>(dev.as<char>() + blk.size() * sizeof(SegBlock));
  }
  void build(Ctx& c, const std::vector<int64_t>& off, const std::vector<int64_t>& n);
};

// Krylov space of a batch of instances (per-instance scalars at stride S).
struct BatchKrylov {
  int kmax = 0, ninst = 0, S = 0;  // S: per-instance scalar stride
  int64_t N = 0;
  DevBuf basis, w, part, part2, scal, kdev;  // part, part2: alternating reduction partials
  HostStage stage;
  void reserve(Ctx& c, int kmax, int64_t N, int ninst, int nblk);
};

// Krylov space of one problem: the batch machinery with a single instance.
struct Krylov {
  SegLayout seg;
  int64_t n = -1;  // complex entries the block table was built for
  BatchKrylov bk;
  void reserve(Ctx& c, int kmax, int64_t n);
};

struct Timers {
  double matvec_s = 0;  // device time of iteration matvecs
  double gemm_s = 0;    // device time of their grouped-GEMM launches
  int64_t gemm_launches = 0;
};

struct LanczosOut {
  double E_ritz = 0, E = 0, residual = 0;
  int steps = 0;
  int64_t matvecs = 0;
};

// Lowest eigenpairs of m independent problems sharing one operator over a
// batch vector (instance i: n[i] complex entries at the block table's
// offsets); x (re plane of N = sum n[i] doubles, then im plane) holds the
// start vectors on entry and the normalised ground vectors on exit.
void lanczos_core(Ctx& c, HeffOp& op, const SegLayout& seg, const std::vector<int64_t>& n,
                  BatchKrylov& K, double* x, const tnt_lanczos_params& p,
                  std::vector<LanczosOut>& out, Timers* tm);

// x: 2n doubles (re | im) in the operator's theta layout; start vector on
// entry, normalised ground vector on exit.
LanczosOut lanczos_run(Ctx& c, HeffOp& op, Krylov& K, double* x, const tnt_lanczos_params& p,
                       Timers* tm);

void jacobi_eigh(std::vector<double>& a, std::vector<double>& v, int n);
void tridiag_lowest(const std::vector<double>& alpha, const std::vector<double>& beta,
                    double* eval, std::vector<double>& evec);

}  // namespace tnt
