// Model MPOs (host only), lower triangular: rows w index the left MPO bond,
// columns w' the right one.
//  - The Bose-Hubbard chain of Sec. 5, Eq. (2) with V = 0, D = 4, chain
//    operator e_3^T W_1 ... W_L e_0.  Operators on the truncated local space
//    |n>, n = 0..nmax:  b|n> = sqrt(n)|n-1>,  h = U/2 n(n-1) - mu n.
//  - The spin-1 isotropic Heisenberg chain of the DMRG timing table (Sec. 3,
//    Table tab:dmrgtimes), D = 5, chain operator e_4^T W_1 ... W_L e_0, on
//    s = m + 1 = 0, 1, 2 (m = S^z), so the U(1) charge of a site is s.
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

// H = J sum S_j . S_{j+1} = J sum [Sz Sz + (S+ S- + S- S+) / 2]; the raising
// element of spin 1 is sqrt(2) for both m = -1 and m = 0.
extern "C" tnt_status tnt_mpo_spin1_heisenberg(double J, double* W, int32_t* bond_charge) {
  if (!W || !bond_charge) return TNT_E_ARG;
  if (!std::isfinite(J)) return TNT_E_NONFINITE;
  const int d = 3, D = 5;
  auto at = [&](int w, int wp, int sp, int s) -> double& {
    return W[((w * D + wp) * d + sp) * d + s];
  };
  for (int i = 0; i < D * D * d * d; ++i) W[i] = 0.0;
  const double r2 = std::sqrt(2.0);
  for (int s = 0; s < d; ++s) {
    at(0, 0, s, s) = 1.0;            // identity (right part done)
    at(4, 4, s, s) = 1.0;            // identity (left part pending)
    at(3, 0, s, s) = s - 1.0;        // Sz closing a bond
    at(4, 3, s, s) = J * (s - 1.0);  // J Sz opening a bond
  }
  for (int s = 0; s + 1 < d; ++s) {
    at(1, 0, s, s + 1) = r2;            // S-   closing
    at(2, 0, s + 1, s) = r2;            // S+   closing
    at(4, 1, s + 1, s) = 0.5 * J * r2;  // J/2 S+ opening
    at(4, 2, s, s + 1) = 0.5 * J * r2;  // J/2 S- opening
  }
  // U(1) charge of each MPO bond index (net charge raised to its left)
  bond_charge[0] = 0;
  bond_charge[1] = 1;
  bond_charge[2] = -1;
  bond_charge[3] = 0;
  bond_charge[4] = 0;
  return TNT_OK;
}
