// Lanczos eigensolver state and driver.
#pragma once

#include <vector>

#include "plan.h"

namespace tnt {

struct Krylov {
  int kmax = 0;
  int64_t n = 0;      // complex entries per vector
  DevBuf basis;       // kmax vectors of 2n doubles (re | im)
  DevBuf w;           // work vector
  DevBuf part;        // reduction partials
  DevBuf scal;        // device scalar slots
  HostStage stage;    // pinned host slots
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

// x: 2n doubles (re | im) in the operator's theta layout; start vector on
// entry, normalised ground vector on exit.
LanczosOut lanczos_run(Ctx& c, HeffOp& op, Krylov& K, double* x, const tnt_lanczos_params& p,
                       Timers* tm);

void jacobi_eigh(std::vector<double>& a, std::vector<double>& v, int n);
void tridiag_lowest(const std::vector<double>& alpha, const std::vector<double>& beta,
                    double* eval, std::vector<double>& evec);

}  // namespace tnt
