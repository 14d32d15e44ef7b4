// Two-site TEBD time step on a U(1) block MPS (time evolution by
// Trotterised two-site gates, Sec. 1; the time-evolution example of Sec. 5
// and the timing workload of Table tab:tebdtimes).
//
// H = sum_j h_j over the bonds (j, j+1).  One step of dt applies
// G_j = exp(-i h_j dt/2) to theta = A_j B_{j+1} for j = 1..L-1 and then for
// j = L-1..1, each followed by the truncated SVD of appendix B.1.2 that moves
// the orthogonality centre along with the gate; the symmetric product of the
// two passes is a second-order Trotter step.  The gates are formed on the
// host from the eigen-decomposition of the real symmetric h_j; on the device
// a step per bond is: theta formation (grouped GEMM), the gate (one
// elementwise launch), the block SVD.
#include <chrono>
#include <cmath>
#include <cstring>

#include "dmrg.h"
#include "kernels.h"

namespace tnt {

namespace {
double clock_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

// G = V diag(exp(-i tau lambda)) V^T for real symmetric h (n x n, row-major)
static void make_gate(const double* h, int n, double tau, std::vector<double>& gre,
                      std::vector<double>& gim) {
  std::vector<double> a(h, h + (size_t)n * n), v;
  jacobi_eigh(a, v, n);
  gre.assign((size_t)n * n, 0.0);
  gim.assign((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    const double lam = a[(size_t)k * n + k];
    const double cr = std::cos(tau * lam), ci = -std::sin(tau * lam);
    for (int r = 0; r < n; ++r) {
      const double vr = v[(size_t)r * n + k];
      if (vr == 0.0) continue;
      for (int col = 0; col < n; ++col) {
        const double vv = vr * v[(size_t)col * n + k];
        gre[(size_t)r * n + col] += cr * vv;
        gim[(size_t)r * n + col] += ci * vv;
      }
    }
  }
}

void tebd_step(Ctx& c, MpsH& m, const double* h, double dt, const tnt_trunc_params& tp,
               TebdStats& st, double* bond_eps, int32_t* bond_chi) {
  const int L = m.L, d = m.d, n = d * d;
  if (L < 2) fail(TNT_E_STATE, "need at least two sites");
  std::vector<std::vector<double>> gr(L - 1), gi(L - 1);
  for (int b = 0; b < L - 1; ++b) make_gate(h + (size_t)b * n * n, n, 0.5 * dt, gr[b], gi[b]);
  DevBuf theta, gated;
  int rec = 0;
  const double t0 = clock_s();
  for (int pass = 0; pass < 2; ++pass) {
    for (int step = 0; step < L - 1; ++step) {
      const int j = pass == 0 ? 1 + step : L - 1 - step;
      const double ta = clock_s();
      ThetaH th = form_theta(c, m, j, theta);
      // gate terms: destination (qa, s1', s2') from sources (qa, s1, s2),
      // s1 + s2 = s1' + s2'
      std::vector<GateTask> tasks;
      std::vector<GateTerm> terms;
      std::vector<int2> chunks;
      const std::vector<double>& Gr = gr[j - 1];
      const std::vector<double>& Gi = gi[j - 1];
      for (auto& kv : th.blocks) {
        const int qa = kv.first[0], s1p = kv.first[1], s2p = kv.first[2];
        const int size = kv.second.rows * kv.second.cols;
        GateTask t{kv.second.off, size, (int)terms.size(), 0, 0};
        for (int s1 = 0; s1 < d; ++s1) {
          const int s2 = s1p + s2p - s1;
          if (s2 < 0 || s2 >= d) continue;
          const size_t gidx = (size_t)(s1p * d + s2p) * n + (s1 * d + s2);
          if (Gr[gidx] == 0.0 && Gi[gidx] == 0.0) continue;
          auto src = th.blocks.find({qa, s1, s2});
          if (src == th.blocks.end()) continue;
          terms.push_back(GateTerm{src->second.off, Gr[gidx], Gi[gidx]});
          t.nterm++;
        }
        const int tix = (int)tasks.size();
        tasks.push_back(t);
        for (int ck = 0; ck * GATE_CHUNK < size; ++ck) chunks.push_back(make_int2(tix, ck));
      }
      const size_t tb = tasks.size() * sizeof(GateTask), mb = terms.size() * sizeof(GateTerm);
      const size_t cb = chunks.size() * sizeof(int2);
      const size_t o1 = (tb + 255) / 256 * 256, o2 = o1 + (mb + 255) / 256 * 256;
      std::vector<char> host(o2 + cb + 8, 0);
      if (tb) std::memcpy(host.data(), tasks.data(), tb);
      if (mb) std::memcpy(host.data() + o1, terms.data(), mb);
      if (cb) std::memcpy(host.data() + o2, chunks.data(), cb);
      DevBuf tab(&c.pool, host.size());
      TNT_HIP(hipMemcpyAsync(tab.ptr, host.data(), host.size(), hipMemcpyHostToDevice, c.stream));
      gated.ensure(&c.pool, std::max<int64_t>(1, 2 * th.elems) * sizeof(double));
      const double* sre = theta.as<double>();
      double* dre = gated.as<double>();
      launch_gate_apply(reinterpret_cast<const GateTask*>(tab.as<char>()),
                        reinterpret_cast<const GateTerm*>(tab.as<char>() + o1),
                        reinterpret_cast<const int2*>(tab.as<char>() + o2), (int)chunks.size(),
                        sre, sre + th.elems, dre, dre + th.elems, c.stream);
      TNT_HIP(hipStreamSynchronize(c.stream));  // host tables released below
      const double tb2 = clock_s();
      st.t_gate += tb2 - ta;
      const int absorb = pass == 0 ? TNT_ABSORB_RIGHT : TNT_ABSORB_LEFT;
      DevBuf na, nb;
      SvdOut r = svd_truncate_dev(c, th, dre, dre + th.elems, tp, absorb, [&](const SvdOut& o) {
        na = DevBuf(&c.pool, std::max<int64_t>(1, 2 * o.A.elems) * 8);
        nb = DevBuf(&c.pool, std::max<int64_t>(1, 2 * o.B.elems) * 8);
        FactorPlanes fp;
        fp.a_re = na.as<double>();
        fp.a_im = na.as<double>() + o.A.elems;
        fp.b_re = nb.as<double>();
        fp.b_im = nb.as<double>() + o.B.elems;
        return fp;
      });
      st.t_svd += clock_s() - tb2;
      m.bonds[j] = r.bond;
      m.lay[j - 1] = r.A;
      m.dat[j - 1] = std::move(na);
      m.lay[j] = r.B;
      m.dat[j] = std::move(nb);
      st.sum_eps += r.eps;
      st.max_eps = std::max(st.max_eps, r.eps);
      st.max_chi = std::max(st.max_chi, r.chi);
      if (bond_eps) bond_eps[rec] = r.eps;
      if (bond_chi) bond_chi[rec] = r.chi;
      ++rec;
    }
  }
  st.t_total = clock_s() - t0;
}

}  // namespace tnt
