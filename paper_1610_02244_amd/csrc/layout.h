// Host-side views of the U(1) block tensors handed over the C-ABI, with the
// validation the ABI promises (charge rule, consistent extents, capacity).
#pragma once

#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "common.h"

namespace tnt {

using Bond = std::map<int, int>;  // charge -> sector dimension

struct BlockRef {
  int64_t off;
  int rows, cols;
};

struct MpoH {
  int d = 0, D = 0;
  std::vector<int> qw;
  std::vector<double> W;  // [((w*D + w')*d + s')*d + s]
  double at(int w, int wp, int sp, int s) const { return W[((w * D + wp) * d + sp) * d + s]; }
};

// theta[a, s1, s2, b]: key (q_a, s1, s2)
struct ThetaH {
  int d = 0;
  std::map<std::array<int, 3>, BlockRef> blocks;
  Bond left, right;
  int64_t elems = 0;   // sum of block sizes
  int64_t extent = 0;  // max(offset + size)
};

// environment [x', w, x]: key (w, q_x) -> block (dim(q_x + qw[w]) x dim(q_x))
struct EnvH {
  std::map<std::pair<int, int>, BlockRef> blocks;
  Bond bond;
  int64_t elems = 0;
  int64_t extent = 0;
};

MpoH parse_mpo(const tnt_mpo_site* m, const char* what);
ThetaH parse_theta(const tnt_btensor* t, int d, const char* what);
EnvH parse_env(const tnt_btensor* t, const MpoH& mpo, const char* what);
// extents of sectors present in both must agree
void check_bond_match(const Bond& a, const Bond& b, const char* what);
void check_same_structure(const ThetaH& a, const ThetaH& b);

// Theta layout from bonds in canonical order: ascending (q_a, s1, s2), packed.
ThetaH make_theta(const Bond& left, const Bond& right, int d);
// Environment layout in canonical order: ascending (q, w), packed.
EnvH make_env(const Bond& bond, const std::vector<int>& qw);

std::string bond_str(const Bond& b);

}  // namespace tnt
