// Model MPOs (host only).  The Bose-Hubbard chain of Sec. 5, Eq. (2) with
// V = 0, written as a D = 4 lower-triangular MPO: rows w index the left
// MPO bond, columns w' the right one, and the chain operator is
// e_3^T W_1 ... W_L e_0.  Operators on the truncated local space
// |n>, n = 0..nmax:  b|n> = sqrt(n)|n-1>,  h = U/2 n(n-1) - mu n.
#include <cmath>

#include "../../include/tnt.h"

extern "C" tnt_status tnt_mpo_bose_hubbard(int32_t nmax, double J, double U, double mu,
                                           double* W, int32_t* bond_charge) {
  if (nmax < 0 || nmax > 63 || !W || !bond_charge) return TNT_E_ARG;
  if (!std::isfinite(J) || !std::isfinite(U) || !std::isfinite(mu)) return TNT_E_NONFINITE;
  const int d = nmax + 1, D = 4;
  auto at = [&](int w, int wp, int sp, int s) -> double& {
    return W[((w * D + wp) * d + sp) * d + s];
  };
  for (int i = 0; i < D * D * d * d; ++i) W[i] = 0.0;
  for (int n = 0; n < d; ++n) {
    at(0, 0, n, n) = 1.0;                                  // identity (right part done)
    at(3, 3, n, n) = 1.0;                                  // identity (left part pending)
    at(3, 0, n, n) = 0.5 * U * n * (n - 1.0) - mu * n;     // on-site term
  }
  for (int n = 1; n < d; ++n) {
    const double a = std::sqrt((double)n);
    at(1, 0, n - 1, n) = a;       // b   closing a hop
    at(2, 0, n, n - 1) = a;       // b^+ closing a hop
    at(3, 1, n, n - 1) = -J * a;  // -J b^+ opening a hop
    at(3, 2, n - 1, n) = -J * a;  // -J b   opening a hop
  }
  // U(1) charge of each MPO bond index (net bosons created to its left)
  bond_charge[0] = 0;
  bond_charge[1] = 1;
  bond_charge[2] = -1;
  bond_charge[3] = 0;
  return TNT_OK;
}
