// MPS and environment storage, and the two-site sweep (Sec. 4.3).
#pragma once

#include <complex>

#include <vector>

#include "lanczos.h"
#include "svd.h"

namespace tnt {

struct MpsH {
  Ctx* ctx = nullptr;
  int L = 0, d = 0;
  std::vector<Bond> bonds;    // 0..L
  std::vector<SiteH> lay;     // site j at index j-1
  std::vector<DevBuf> dat;    // [re (elems) | im (elems)] per site
  double* re(int j) { return dat[j - 1].as<double>(); }
  double* im(int j) { return dat[j - 1].as<double>() + lay[j - 1].elems; }
};

struct EnvS {
  MpsH* mps = nullptr;
  std::vector<MpoH> W;        // site j at index j-1
  int left_index = 0, right_index = 0;
  std::vector<int> qw;
  std::vector<EnvH> Llay;     // L_j, j = 0..L
  std::vector<EnvH> Rlay;     // R_j, j = 1..L+1
  std::vector<DevBuf> Ldat, Rdat;
  double* Lre(int j) { return Ldat[j].as<double>(); }
  double* Lim(int j) { return Ldat[j].as<double>() + Llay[j].elems; }
  double* Rre(int j) { return Rdat[j].as<double>(); }
  double* Rim(int j) { return Rdat[j].as<double>() + Rlay[j].elems; }
};

// theta_j = A_j A_{j+1} into a packed FP64 buffer (re | im); returns its layout.
ThetaH form_theta(Ctx& c, MpsH& m, int j, DevBuf& out);
// L_j from L_{j-1}, A_j, W_j ; R_j from R_{j+1}, A_j, W_j.
void update_left_env(Ctx& c, EnvS& e, int j);
void update_right_env(Ctx& c, EnvS& e, int j);
void build_boundaries(Ctx& c, EnvS& e);
void right_canonicalize(Ctx& c, MpsH& m);
// C[(i-1) L + (j-1)] = <O^dagger_i O_j> / <psi|psi> for a real d x d
// operator op[s' d + s] whose nonzero entries all have s' - s = dq
// (validated by the caller); *flops = the pass's algorithmic flops.
// theta of sites (j, j+1) into `out` (grown as needed), canonical layout
ThetaH form_theta(Ctx& c, MpsH& m, int j, DevBuf& out);

struct TebdStats {
  double t_total = 0, t_gate = 0, t_svd = 0;
  double sum_eps = 0, max_eps = 0;
  int max_chi = 0;
};
// One second-order TEBD step (bond Hamiltonians h: (L-1) blocks of d^2 x d^2
// real symmetric, charge-conserving, validated by the caller).
void tebd_step(Ctx& c, MpsH& m, const double* h, double dt, const tnt_trunc_params& tp,
               TebdStats& st, double* bond_eps, int32_t* bond_chi);

void correlation_matrix(Ctx& c, MpsH& m, const std::vector<double>& op, int dq,
                        std::vector<std::complex<double>>& C, double* flops);

struct SweepStats {
  double energy = 0, max_residual = 0, max_eps = 0;
  int updates = 0, max_chi = 0;
  int64_t matvecs = 0;
  double matvec_flops = 0;
  double gemm_flops = 0, t_gemm = 0;
  int64_t gemm_launches = 0;
  double t_total = 0, t_matvec = 0, t_lanczos = 0, t_svd = 0, t_env = 0, t_theta = 0, t_setup = 0;
  int64_t eig_retries = 0;
};

void dmrg_sweep(Ctx& c, MpsH& m, EnvS& e, const tnt_sweep_params& p, SweepStats& st);
// One sweep of each of several chains, bond updates in lockstep with one
// batched Lanczos per step (ps[i]: the chain's parameters; the Lanczos
// parameters of ps[0] apply to all).  Timings in st are batch totals.
void dmrg_sweep_batched(Ctx& c, const std::vector<MpsH*>& ms, const std::vector<EnvS*>& es,
                        const tnt_sweep_params* ps, std::vector<SweepStats>& st);

}  // namespace tnt
