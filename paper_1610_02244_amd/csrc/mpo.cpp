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

// Bond Hamiltonians for a TEBD step, h_j on sites (j, j+1) as d^2 x d^2
// matrices, row (s1' d + s2'), column (s1 d + s2); sum_j h_j = H.
// Bose-Hubbard (Sec. 5, Eq. 2 with V = 0): the hopping of the bond plus the
// on-site terms of its two sites, each shared equally with the site's other
// bond (an end site puts its whole term on its only bond).
extern "C" tnt_status tnt_bond_hamiltonians_bose_hubbard(int32_t L, int32_t nmax, double J,
                                                         double U, double mu, double* h) {
  if (!h || L < 2 || nmax < 1) return TNT_E_ARG;
  if (!std::isfinite(J) || !std::isfinite(U) || !std::isfinite(mu)) return TNT_E_NONFINITE;
  const int d = nmax + 1, n = d * d;
  auto onsite = [&](int k) { return 0.5 * U * k * (k - 1.0) - mu * k; };
  for (int b = 1; b < L; ++b) {
    double* hb = h + (size_t)(b - 1) * n * n;
    for (int i = 0; i < n * n; ++i) hb[i] = 0.0;
    const double wl = b == 1 ? 1.0 : 0.5, wr = b + 1 == L ? 1.0 : 0.5;
    for (int s1 = 0; s1 < d; ++s1)
      for (int s2 = 0; s2 < d; ++s2) {
        const int col = s1 * d + s2;
        hb[(size_t)col * n + col] = wl * onsite(s1) + wr * onsite(s2);
        // -J b^dagger_1 b_2: (s1 + 1, s2 - 1), amplitude sqrt((s1 + 1) s2)
        if (s1 + 1 < d && s2 >= 1)
          hb[(size_t)((s1 + 1) * d + (s2 - 1)) * n + col] = -J * std::sqrt((s1 + 1.0) * s2);
        // -J b_1 b^dagger_2
        if (s1 >= 1 && s2 + 1 < d)
          hb[(size_t)((s1 - 1) * d + (s2 + 1)) * n + col] = -J * std::sqrt(s1 * (s2 + 1.0));
      }
  }
  return TNT_OK;
}

// Spin-1 isotropic Heisenberg (Table tab:tebdtimes): h_j = J S_j . S_{j+1}
// on s = S^z + 1, the same on every bond.
extern "C" tnt_status tnt_bond_hamiltonians_spin1(int32_t L, double J, double* h) {
  if (!h || L < 2) return TNT_E_ARG;
  if (!std::isfinite(J)) return TNT_E_NONFINITE;
  const int d = 3, n = 9;
  for (int b = 1; b < L; ++b) {
    double* hb = h + (size_t)(b - 1) * n * n;
    for (int i = 0; i < n * n; ++i) hb[i] = 0.0;
    for (int s1 = 0; s1 < d; ++s1)
      for (int s2 = 0; s2 < d; ++s2) {
        const int col = s1 * d + s2;
        hb[(size_t)col * n + col] = J * (s1 - 1.0) * (s2 - 1.0);
        // J/2 S+_1 S-_2 and J/2 S-_1 S+_2; every spin-1 ladder element is sqrt(2)
        if (s1 + 1 < d && s2 >= 1) hb[(size_t)((s1 + 1) * d + (s2 - 1)) * n + col] = J;
        if (s1 >= 1 && s2 + 1 < d) hb[(size_t)((s1 - 1) * d + (s2 + 1)) * n + col] = J;
      }
  }
  return TNT_OK;
}
