// Parsing and validation of block-tensor descriptors (U(1) rule of the
// symmetric nodes: sum of incoming labels = sum of outgoing labels).
#include "layout.h"

#include <cmath>
#include <sstream>

namespace tnt {

static void need(bool ok, tnt_status code, const std::string& msg) {
  if (!ok) fail(code, msg);
}

MpoH parse_mpo(const tnt_mpo_site* m, const char* what) {
  need(m != nullptr, TNT_E_ARG, std::string(what) + ": null MPO site");
  need(m->d >= 1 && m->d <= 64 && m->D >= 1 && m->D <= 64, TNT_E_ARG,
       std::string(what) + ": MPO d/D out of range");
  need(m->bond_charge != nullptr && m->W != nullptr, TNT_E_ARG,
       std::string(what) + ": null MPO arrays");
  MpoH h;
  h.d = m->d;
  h.D = m->D;
  h.qw.assign(m->bond_charge, m->bond_charge + m->D);
  h.W.assign(m->W, m->W + (size_t)m->D * m->D * m->d * m->d);
  for (int w = 0; w < h.D; ++w)
    for (int wp = 0; wp < h.D; ++wp)
      for (int sp = 0; sp < h.d; ++sp)
        for (int s = 0; s < h.d; ++s) {
          const double v = h.at(w, wp, sp, s);
          need(std::isfinite(v), TNT_E_NONFINITE, std::string(what) + ": non-finite MPO entry");
          if (v != 0.0 && sp - s != h.qw[wp] - h.qw[w])
            fail(TNT_E_CHARGE, std::string(what) + ": MPO element violates s'-s = q(w')-q(w)");
        }
  return h;
}

static void check_common(const tnt_btensor* t, int rank, const char* what) {
  need(t != nullptr, TNT_E_ARG, std::string(what) + ": null tensor");
  need(t->rank == rank, TNT_E_ARG, std::string(what) + ": wrong rank");
  need(t->nblocks >= 0, TNT_E_ARG, std::string(what) + ": negative block count");
  if (t->nblocks > 0)
    need(t->qn && t->extent && t->offset, TNT_E_ARG, std::string(what) + ": null metadata");
  need(t->dtype == TNT_DT_F64 || t->dtype == TNT_DT_F32, TNT_E_ARG,
       std::string(what) + ": bad dtype");
  need(t->capacity >= 0, TNT_E_ARG, std::string(what) + ": negative capacity");

}

static void set_dim(Bond& b, int q, int dim, const char* what) {
  auto it = b.find(q);
  if (it == b.end()) b[q] = dim;
  else if (it->second != dim)
    fail(TNT_E_SHAPE, std::string(what) + ": sector " + std::to_string(q) +
                          " has inconsistent extents");
}

ThetaH parse_theta(const tnt_btensor* t, int d, const char* what) {
  check_common(t, 4, what);
  ThetaH h;
  h.d = d;
  for (int i = 0; i < t->nblocks; ++i) {
    const int* q = t->qn + 4 * i;
    const int* e = t->extent + 4 * i;
    need(e[1] == 1 && e[2] == 1, TNT_E_SHAPE, std::string(what) + ": physical extents must be 1");
    need(e[0] >= 1 && e[3] >= 1, TNT_E_SHAPE, std::string(what) + ": empty block");
    need(q[1] >= 0 && q[1] < d && q[2] >= 0 && q[2] < d, TNT_E_ARG,
         std::string(what) + ": physical label out of range");
    if (q[3] != q[0] + q[1] + q[2])
      fail(TNT_E_CHARGE, std::string(what) + ": block violates q_b = q_a + s1 + s2");
    const int64_t off = t->offset[i];
    const int64_t sz = (int64_t)e[0] * e[3];
    need(off >= 0, TNT_E_ARG, std::string(what) + ": negative offset");
    if (off + sz > t->capacity) fail(TNT_E_CAPACITY, std::string(what) + ": block past capacity");
    std::array<int, 3> key{q[0], q[1], q[2]};
    need(!h.blocks.count(key), TNT_E_ARG, std::string(what) + ": duplicate block");
    h.blocks[key] = BlockRef{off, e[0], e[3]};
    set_dim(h.left, q[0], e[0], what);
    set_dim(h.right, q[3], e[3], what);
    h.elems += sz;
    h.extent = std::max(h.extent, off + sz);
  }
  return h;
}

EnvH parse_env(const tnt_btensor* t, const MpoH& mpo, const char* what) {
  check_common(t, 3, what);
  EnvH h;
  for (int i = 0; i < t->nblocks; ++i) {
    const int* q = t->qn + 3 * i;
    const int* e = t->extent + 3 * i;
    need(q[1] >= 0 && q[1] < mpo.D, TNT_E_ARG, std::string(what) + ": MPO index out of range");
    need(e[1] == 1, TNT_E_SHAPE, std::string(what) + ": MPO-leg extent must be 1");
    need(e[0] >= 1 && e[2] >= 1, TNT_E_SHAPE, std::string(what) + ": empty block");
    if (q[0] != q[2] + mpo.qw[q[1]])
      fail(TNT_E_CHARGE, std::string(what) + ": block violates q' = q + q(w)");
    const int64_t off = t->offset[i];
    const int64_t sz = (int64_t)e[0] * e[2];
    need(off >= 0, TNT_E_ARG, std::string(what) + ": negative offset");
    if (off + sz > t->capacity) fail(TNT_E_CAPACITY, std::string(what) + ": block past capacity");
    std::pair<int, int> key{q[1], q[2]};
    need(!h.blocks.count(key), TNT_E_ARG, std::string(what) + ": duplicate block");
    h.blocks[key] = BlockRef{off, e[0], e[2]};
    set_dim(h.bond, q[0], e[0], what);
    set_dim(h.bond, q[2], e[2], what);
    h.elems += sz;
    h.extent = std::max(h.extent, off + sz);
  }
  return h;
}

void check_bond_match(const Bond& a, const Bond& b, const char* what) {
  for (auto& kv : a) {
    auto it = b.find(kv.first);
    if (it != b.end() && it->second != kv.second)
      fail(TNT_E_SHAPE, std::string(what) + ": sector " + std::to_string(kv.first) +
                            " extent " + std::to_string(kv.second) + " vs " +
                            std::to_string(it->second));
  }
}

void check_same_structure(const ThetaH& a, const ThetaH& b) {
  if (a.blocks.size() != b.blocks.size())
    fail(TNT_E_SHAPE, "output block set differs from theta");
  for (auto& kv : a.blocks) {
    auto it = b.blocks.find(kv.first);
    if (it == b.blocks.end() || it->second.rows != kv.second.rows ||
        it->second.cols != kv.second.cols)
      fail(TNT_E_SHAPE, "output block set differs from theta");
  }
}

ThetaH make_theta(const Bond& left, const Bond& right, int d) {
  ThetaH h;
  h.d = d;
  int64_t off = 0;
  for (auto& l : left)
    for (int s1 = 0; s1 < d; ++s1)
      for (int s2 = 0; s2 < d; ++s2) {
        auto it = right.find(l.first + s1 + s2);
        if (it == right.end()) continue;
        h.blocks[{l.first, s1, s2}] = BlockRef{off, l.second, it->second};
        h.left[l.first] = l.second;
        h.right[it->first] = it->second;
        off += (int64_t)l.second * it->second;
      }
  h.elems = h.extent = off;
  return h;
}

EnvH make_env(const Bond& bond, const std::vector<int>& qw) {
  EnvH h;
  h.bond = bond;
  int64_t off = 0;
  for (auto& b : bond)
    for (int w = 0; w < (int)qw.size(); ++w) {
      auto it = bond.find(b.first + qw[w]);
      if (it == bond.end()) continue;
      h.blocks[{w, b.first}] = BlockRef{off, it->second, b.second};
      off += (int64_t)it->second * b.second;
    }
  h.elems = h.extent = off;
  return h;
}

std::string bond_str(const Bond& b) {
  std::ostringstream os;
  os << "{";
  for (auto& kv : b) os << kv.first << ":" << kv.second << " ";
  os << "}";
  return os.str();
}

}  // namespace tnt
