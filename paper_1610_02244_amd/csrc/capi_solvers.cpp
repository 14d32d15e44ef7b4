// C-ABI: eigensolver, truncated SVD, MPS/environment handles and the sweep.
#include <climits>
#include <cmath>
#include <cstring>

#include "batch.h"
#include "capi_util.h"
#include "dmrg.h"

namespace tnt {

// Block-by-block copy between two layouts of the same block set (FP64).
static void copy_blocks(Ctx& c, const ThetaH& src, const double* sre, const double* sim,
                        const ThetaH& dst, double* dre, double* dim) {
  HostComb h;
  for (auto& kv : dst.blocks) {
    const BlockRef& s = src.blocks.at(kv.first);
    h.add_task(kv.second.off, kv.second.rows * kv.second.cols);
    h.add_term(s.off, 1.0);
  }
  h.finalize();
  DevTables t;
  t.upload(c, {}, {&h});
  run_comb(c, t.c[0], sre, sim, dre, dim, ET_F64);
  TNT_HIP(hipStreamSynchronize(c.stream));
}

static ThetaH packed(const ThetaH& t) {
  ThetaH p = t;
  int64_t off = 0;
  for (auto& kv : p.blocks) {
    kv.second.off = off;
    off += (int64_t)kv.second.rows * kv.second.cols;
  }
  p.elems = p.extent = off;
  return p;
}

static void check_trunc(const tnt_trunc_params* p) {
  if (!p) fail(TNT_E_ARG, "null truncation parameters");
  if (p->chi_max < 1) fail(TNT_E_ARG, "chi_max must be >= 1");
  if (p->err_type < TNT_ERR_2NORM || p->err_type > TNT_ERR_1NORM) fail(TNT_E_ARG, "bad err_type");
  if (std::isnan(p->abs_tol) || std::isnan(p->rel_tol) || std::isnan(p->err_tol))
    fail(TNT_E_ARG, "NaN tolerance");
}

static void check_lanczos(const tnt_lanczos_params* p) {
  if (!p) fail(TNT_E_ARG, "null Lanczos parameters");
  check_precision(p->precision);
  if (p->kmax < 1 || p->kmax > 32) fail(TNT_E_ARG, "kmax must be in [1, 32]");
  if (!(p->beta_tol >= 0)) fail(TNT_E_ARG, "beta_tol must be >= 0");
}

struct MpsObj {
  Ctx* ctx;
  MpsH m;
};
struct EnvObj {
  Ctx* ctx;
  MpsObj* mps;
  EnvS e;
};

}  // namespace tnt

using namespace tnt;

extern "C" {

tnt_status tnt_lanczos_ground(tnt_ctx ctx, const tnt_btensor* L, const tnt_mpo_site* W1,
                              const tnt_mpo_site* W2, const tnt_btensor* R, tnt_btensor* theta,
                              const tnt_lanczos_params* p, tnt_lanczos_result* r) {
  tnt_status ret = TNT_OK;
  TNT_API_BEGIN(ctx)
  if (!r) fail(TNT_E_ARG, "null result");
  check_lanczos(p);
  HeffArgs a = parse_heff_args(L, W1, W2, R, theta, nullptr);
  if (L->dtype != TNT_DT_F64 || R->dtype != TNT_DT_F64 || theta->dtype != TNT_DT_F64)
    fail(TNT_E_ARG, "L, R and theta must be FP64 planes");
  if (a.th.blocks.empty()) fail(TNT_E_SHAPE, "theta has no block");
  HeffArgs ap = a;
  ap.th = packed(a.th);
  ap.out = ap.th;
  const int64_t n = ap.th.elems;
  auto op = cached_heff(c, ap, p->precision);
  op->bind_envs(L->re, L->im, R->re, R->im);
  Krylov K;
  K.reserve(c, p->kmax, n);
  DevBuf x(&c.pool, 2 * n * sizeof(double));
  double* xp = x.as<double>();
  copy_blocks(c, a.th, static_cast<const double*>(theta->re),
              static_cast<const double*>(theta->im), ap.th, xp, xp + n);
  LanczosOut o = lanczos_run(c, *op, K, xp, *p, nullptr);
  copy_blocks(c, ap.th, xp, xp + n, a.th, static_cast<double*>(theta->re),
              static_cast<double*>(theta->im));
  r->E_ritz = o.E_ritz;
  r->E_refined = o.E;
  r->residual = o.residual;
  r->steps = o.steps;
  if (p->resid_tol > 0 && o.residual > p->resid_tol) ret = TNT_W_NOCONV;
  return ret;
  TNT_API_END
}

tnt_status tnt_lanczos_ground_batched(tnt_ctx ctx, int32_t n, const tnt_btensor* const* L,
                                      const tnt_mpo_site* const* W1,
                                      const tnt_mpo_site* const* W2, const tnt_btensor* const* R,
                                      tnt_btensor* const* theta, const tnt_lanczos_params* p,
                                      tnt_lanczos_result* r) {
  tnt_status ret = TNT_OK;
  TNT_API_BEGIN(ctx)
  if (n < 1 || !L || !W1 || !W2 || !R || !theta || !r) fail(TNT_E_ARG, "null or empty batch");
  check_lanczos(p);
  const uint64_t rh = raw_hash_batch(n, L, W1, W2, R, theta, nullptr, p->precision,
                                     0xa4093822299f31d0ULL);
  std::shared_ptr<BatchCall> bc = find_batch_call(c, rh);
  if (bc) {
    // the same descriptors were parsed and validated before
    for (int i = 0; i < n; ++i)
      for (const tnt_btensor* t : {L[i], R[i], (const tnt_btensor*)theta[i]})
        if (!t->re || !t->im) fail(TNT_E_ARG, "null plane");
  } else {
    bc = std::make_shared<BatchCall>();
    std::vector<int64_t> nn;
    for (int i = 0; i < n; ++i) {
      HeffArgs a = parse_heff_args(L[i], W1[i], W2[i], R[i], theta[i], nullptr);
      if (L[i]->dtype != TNT_DT_F64 || R[i]->dtype != TNT_DT_F64 || theta[i]->dtype != TNT_DT_F64)
        fail(TNT_E_ARG, "L, R and theta must be FP64 planes");
      if (a.th.blocks.empty()) fail(TNT_E_SHAPE, "theta has no block");
      bc->tlay.push_back(a.th);
      a.th = packed(a.th);
      a.out = a.th;
      nn.push_back(a.th.elems);
      bc->olay.push_back(a.th);
      bc->ops.push_back(cached_heff(c, a, p->precision));
    }
    bc->b = cached_batch(c, bc->ops, nn, p->precision);
    store_batch_call(c, rh, bc);
  }
  BatchHeff& B = *bc->b;
  std::vector<const double *> Lr, Li, Rr, Ri;
  for (int i = 0; i < n; ++i) {
    Lr.push_back(static_cast<const double*>(L[i]->re));
    Li.push_back(static_cast<const double*>(L[i]->im));
    Rr.push_back(static_cast<const double*>(R[i]->re));
    Ri.push_back(static_cast<const double*>(R[i]->im));
  }
  bind_batch_envs(c, B, Lr, Li, Rr, Ri);
  bc->xy.ensure(&c.pool, std::max<int64_t>(1, 2 * B.N) * sizeof(double));
  double* x = bc->xy.as<double>();
  // every block of every instance into the batch vector, and back afterwards
  std::vector<CopyRun> in, back;
  for (int i = 0; i < n; ++i) {
    const int64_t off = B.parts[i].x_off;
    double* tre = static_cast<double*>(theta[i]->re);
    double* tim = static_cast<double*>(theta[i]->im);
    for (auto& kv : bc->olay[i].blocks) {
      const BlockRef& src = bc->tlay[i].blocks.at(kv.first);
      const int64_t cnt = (int64_t)src.rows * src.cols;
      in.push_back(CopyRun{tre + src.off, x + off + kv.second.off, cnt});
      in.push_back(CopyRun{tim + src.off, x + B.N + off + kv.second.off, cnt});
      back.push_back(CopyRun{x + off + kv.second.off, tre + src.off, cnt});
      back.push_back(CopyRun{x + B.N + off + kv.second.off, tim + src.off, cnt});
    }
  }
  bc->in.run(c, in);
  std::vector<LanczosOut> o;
  lanczos_run_batched(c, B, bc->K, x, *p, o, nullptr);
  bc->back.run(c, back);
  TNT_HIP(hipStreamSynchronize(c.stream));
  for (int i = 0; i < n; ++i) {
    r[i].E_ritz = o[i].E_ritz;
    r[i].E_refined = o[i].E;
    r[i].residual = o[i].residual;
    r[i].steps = o[i].steps;
    if (p->resid_tol > 0 && o[i].residual > p->resid_tol) ret = TNT_W_NOCONV;
  }
  return ret;
  TNT_API_END
}

tnt_status tnt_theta_svd_truncate(tnt_ctx ctx, const tnt_btensor* theta,
                                  const tnt_trunc_params* p, int32_t absorb, tnt_site_out* A,
                                  tnt_site_out* B, double* S, int32_t s_capacity,
                                  int32_t* bond_q, int32_t* bond_dim, tnt_trunc_result* r) {
  TNT_API_BEGIN(ctx)
  check_trunc(p);
  if (!A || !B || !S || !bond_q || !bond_dim || !r) fail(TNT_E_ARG, "null output");
  if (!A->qn || !A->extent || !A->offset || !A->re || !A->im || !B->qn || !B->extent ||
      !B->offset || !B->re || !B->im)
    fail(TNT_E_ARG, "null output arrays");
  ThetaH th = parse_theta(theta, 64, "theta");
  if (theta->dtype != TNT_DT_F64) fail(TNT_E_ARG, "theta must be FP64");
  if (th.blocks.empty()) fail(TNT_E_SHAPE, "theta has no block");
  SvdOut o = svd_truncate_dev(
      c, th, static_cast<const double*>(theta->re), static_cast<const double*>(theta->im), *p,
      absorb, [&](const SvdOut& s) {
        if ((int64_t)s.A.blocks.size() > A->max_blocks || (int64_t)s.B.blocks.size() > B->max_blocks)
          fail(TNT_E_CAPACITY, "factor metadata arrays too small");
        if (s.A.elems > A->capacity || s.B.elems > B->capacity)
          fail(TNT_E_CAPACITY, "factor planes too small for the kept bond");
        if ((int64_t)s.lam.size() > s_capacity) fail(TNT_E_CAPACITY, "S too small");
        if ((int64_t)s.bond.size() > A->max_blocks) fail(TNT_E_CAPACITY, "bond arrays too small");
        FactorPlanes fp;
        fp.a_re = A->re; fp.a_im = A->im; fp.b_re = B->re; fp.b_im = B->im;
        return fp;
      });
  int i = 0;
  for (auto& kv : o.A.blocks) {
    const int qa = kv.first.first, s1 = kv.first.second;
    A->qn[3 * i] = qa; A->qn[3 * i + 1] = s1; A->qn[3 * i + 2] = qa + s1;
    A->extent[3 * i] = kv.second.rows; A->extent[3 * i + 1] = 1; A->extent[3 * i + 2] = kv.second.cols;
    A->offset[i] = kv.second.off;
    ++i;
  }
  A->nblocks = i;
  i = 0;
  for (auto& kv : o.B.blocks) {
    const int m = kv.first.first, s2 = kv.first.second;
    B->qn[3 * i] = m; B->qn[3 * i + 1] = s2; B->qn[3 * i + 2] = m + s2;
    B->extent[3 * i] = kv.second.rows; B->extent[3 * i + 1] = 1; B->extent[3 * i + 2] = kv.second.cols;
    B->offset[i] = kv.second.off;
    ++i;
  }
  B->nblocks = i;
  std::memcpy(S, o.lam.data(), o.lam.size() * sizeof(double));
  i = 0;
  for (auto& kv : o.bond) {
    bond_q[i] = kv.first;
    bond_dim[i] = kv.second;
    ++i;
  }
  r->chi = o.chi;
  r->nsectors = (int32_t)o.bond.size();
  r->eps = o.eps;
  r->lambda0 = o.lambda0;
  r->norm_kept = o.norm_kept;
  TNT_API_END
}

int32_t tnt_trunc_select(const double* lam, int32_t n, const tnt_trunc_params* p, double* eps) {
  try {
    if (!lam || n < 0) return -1;
    check_trunc(p);
    for (int i = 0; i < n; ++i)
      if (!std::isfinite(lam[i]) || lam[i] < 0 || (i > 0 && lam[i] > lam[i - 1])) return -1;
    return trunc_select(lam, n, *p, eps);
  } catch (...) {
    return -1;
  }
}

// ---------------------------------------------------------------------------
// MPS
// ---------------------------------------------------------------------------
tnt_status tnt_mps_create(tnt_ctx ctx, int32_t L, int32_t d, tnt_mps* out) {
  TNT_API_BEGIN(ctx)
  if (!out) fail(TNT_E_ARG, "null out");
  if (L < 2 || d < 1 || d > 64) fail(TNT_E_ARG, "need L >= 2 and 1 <= d <= 64");
  auto* o = new MpsObj{&c, MpsH()};
  o->m.ctx = &c;
  o->m.L = L;
  o->m.d = d;
  o->m.bonds.assign(L + 1, Bond());
  o->m.lay.assign(L, SiteH());
  o->m.dat.resize(L);
  *out = reinterpret_cast<tnt_mps>(o);
  TNT_API_END
}

void tnt_mps_destroy(tnt_mps mps) { delete reinterpret_cast<MpsObj*>(mps); }

tnt_status tnt_mps_set_bond(tnt_mps mps, int32_t ell, int32_t nsec, const int32_t* q,
                            const int32_t* dim) {
  if (!mps) return TNT_E_ARG;
  MpsObj* o = reinterpret_cast<MpsObj*>(mps);
  TNT_API_BEGIN(o->ctx)
  if (ell < 0 || ell > o->m.L || nsec < 1 || !q || !dim) fail(TNT_E_ARG, "bad bond arguments");
  Bond b;
  for (int i = 0; i < nsec; ++i) {
    if (dim[i] < 1) fail(TNT_E_SHAPE, "sector dimension must be >= 1");
    if (i > 0 && q[i] <= q[i - 1]) fail(TNT_E_ARG, "charges must be strictly ascending");
    b[q[i]] = dim[i];
  }
  o->m.bonds[ell] = b;
  TNT_API_END
}

tnt_status tnt_mps_set_site(tnt_mps mps, int32_t j, int32_t nblocks, const int32_t* q_left,
                            const int32_t* s, const double* re, const double* im) {
  if (!mps) return TNT_E_ARG;
  MpsObj* o = reinterpret_cast<MpsObj*>(mps);
  TNT_API_BEGIN(o->ctx)
  MpsH& m = o->m;
  if (j < 1 || j > m.L) fail(TNT_E_ARG, "site index out of range");
  if (m.bonds[j - 1].empty() || m.bonds[j].empty()) fail(TNT_E_STATE, "set bonds j-1 and j first");
  if (nblocks < 0 || (nblocks > 0 && (!q_left || !s || !re || !im))) fail(TNT_E_ARG, "null input");
  SiteH lay = make_site(m.bonds[j - 1], m.bonds[j], m.d);
  std::vector<double> h(std::max<int64_t>(1, 2 * lay.elems), 0.0);
  int64_t pos = 0;
  for (int i = 0; i < nblocks; ++i) {
    if (s[i] < 0 || s[i] >= m.d) fail(TNT_E_ARG, "physical label out of range");
    auto it = lay.blocks.find({q_left[i], s[i]});
    if (it == lay.blocks.end())
      fail(TNT_E_CHARGE, "block (" + std::to_string(q_left[i]) + "," + std::to_string(s[i]) +
                             ") has no sector on both bonds");
    const int64_t n = (int64_t)it->second.rows * it->second.cols;
    for (int64_t k = 0; k < n; ++k) {
      if (!std::isfinite(re[pos + k]) || !std::isfinite(im[pos + k]))
        fail(TNT_E_NONFINITE, "non-finite site entry");
      h[it->second.off + k] = re[pos + k];
      h[lay.elems + it->second.off + k] = im[pos + k];
    }
    pos += n;
  }
  DevBuf buf(&c.pool, h.size() * sizeof(double));
  TNT_HIP(hipMemcpyAsync(buf.ptr, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice,
                         c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  m.lay[j - 1] = lay;
  m.dat[j - 1] = std::move(buf);
  TNT_API_END
}

int32_t tnt_mps_bond_size(tnt_mps mps, int32_t ell) {
  if (!mps) return -1;
  MpsObj* o = reinterpret_cast<MpsObj*>(mps);
  if (ell < 0 || ell > o->m.L) return -1;
  return (int32_t)o->m.bonds[ell].size();
}

tnt_status tnt_mps_get_bond(tnt_mps mps, int32_t ell, int32_t cap, int32_t* q, int32_t* dim) {
  if (!mps) return TNT_E_ARG;
  MpsObj* o = reinterpret_cast<MpsObj*>(mps);
  TNT_API_BEGIN(o->ctx)
  if (ell < 0 || ell > o->m.L || !q || !dim) fail(TNT_E_ARG, "bad arguments");
  const Bond& b = o->m.bonds[ell];
  if ((int)b.size() > cap) fail(TNT_E_CAPACITY, "bond arrays too small");
  int i = 0;
  for (auto& kv : b) {
    q[i] = kv.first;
    dim[i] = kv.second;
    ++i;
  }
  TNT_API_END
}

tnt_status tnt_mps_get_site(tnt_mps mps, int32_t j, int32_t cap, int32_t* nblocks,
                            int32_t* q_left, int32_t* s, int64_t ecap, double* re, double* im) {
  if (!mps) return TNT_E_ARG;
  MpsObj* o = reinterpret_cast<MpsObj*>(mps);
  TNT_API_BEGIN(o->ctx)
  MpsH& m = o->m;
  if (j < 1 || j > m.L || !nblocks || !q_left || !s || !re || !im) fail(TNT_E_ARG, "bad arguments");
  const SiteH& lay = m.lay[j - 1];
  if (!m.dat[j - 1].ptr) fail(TNT_E_STATE, "site not set");
  if ((int)lay.blocks.size() > cap || lay.elems > ecap) fail(TNT_E_CAPACITY, "output too small");
  std::vector<double> h(std::max<int64_t>(1, 2 * lay.elems));
  TNT_HIP(hipMemcpyAsync(h.data(), m.dat[j - 1].ptr, 2 * lay.elems * sizeof(double),
                         hipMemcpyDeviceToHost, c.stream));
  TNT_HIP(hipStreamSynchronize(c.stream));
  int i = 0;
  int64_t pos = 0;
  for (auto& kv : lay.blocks) {  // ascending (q_left, s)
    q_left[i] = kv.first.first;
    s[i] = kv.first.second;
    const int64_t n = (int64_t)kv.second.rows * kv.second.cols;
    std::memcpy(re + pos, h.data() + kv.second.off, n * sizeof(double));
    std::memcpy(im + pos, h.data() + lay.elems + kv.second.off, n * sizeof(double));
    pos += n;
    ++i;
  }
  *nblocks = i;
  TNT_API_END
}

tnt_status tnt_mps_right_canonicalize(tnt_ctx ctx, tnt_mps mps) {
  TNT_API_BEGIN(ctx)
  if (!mps) fail(TNT_E_ARG, "null mps");
  MpsObj* o = reinterpret_cast<MpsObj*>(mps);
  for (int j = 1; j <= o->m.L; ++j)
    if (!o->m.dat[j - 1].ptr) fail(TNT_E_STATE, "site " + std::to_string(j) + " not set");
  right_canonicalize(c, o->m);
  TNT_HIP(hipStreamSynchronize(c.stream));
  TNT_API_END
}

tnt_status tnt_mps_correlation(tnt_ctx ctx, tnt_mps mps, const double* op, int32_t dq,
                               double* out_re, double* out_im, double* flops) {
  TNT_API_BEGIN(ctx)
  if (!mps || !op || !out_re || !out_im) fail(TNT_E_ARG, "null argument");
  MpsObj* o = reinterpret_cast<MpsObj*>(mps);
  MpsH& m = o->m;
  for (int j = 1; j <= m.L; ++j)
    if (!m.dat[j - 1].ptr) fail(TNT_E_STATE, "site " + std::to_string(j) + " not set");
  const int d = m.d;
  std::vector<double> w(op, op + (size_t)d * d);
  for (int sp = 0; sp < d; ++sp)
    for (int s = 0; s < d; ++s) {
      const double v = w[(size_t)sp * d + s];
      if (!std::isfinite(v)) fail(TNT_E_NONFINITE, "operator entry not finite");
      if (v != 0.0 && sp - s != dq)
        fail(TNT_E_CHARGE, "operator entry (" + std::to_string(sp) + ", " + std::to_string(s) +
                               ") breaks the charge change dq");
    }
  std::vector<std::complex<double>> C;
  double fl = 0.0;
  correlation_matrix(c, m, w, dq, C, &fl);
  for (size_t i = 0; i < C.size(); ++i) {
    out_re[i] = C[i].real();
    out_im[i] = C[i].imag();
  }
  if (flops) *flops = fl;
  TNT_API_END
}

tnt_status tnt_tebd_step(tnt_ctx ctx, tnt_mps mps, const double* h, double dt,
                         const tnt_trunc_params* trunc, int32_t record_cap, double* bond_eps,
                         int32_t* bond_chi, double* stats) {
  TNT_API_BEGIN(ctx)
  if (!mps || !h || !trunc) fail(TNT_E_ARG, "null argument");
  MpsObj* o = reinterpret_cast<MpsObj*>(mps);
  MpsH& m = o->m;
  for (int j = 1; j <= m.L; ++j)
    if (!m.dat[j - 1].ptr) fail(TNT_E_STATE, "site " + std::to_string(j) + " not set");
  if (!std::isfinite(dt)) fail(TNT_E_NONFINITE, "dt not finite");
  if (trunc->chi_max < 1) fail(TNT_E_ARG, "chi_max < 1");
  if ((bond_eps || bond_chi) && record_cap < 2 * (m.L - 1))
    fail(TNT_E_CAPACITY, "record arrays shorter than 2(L-1)");
  const int d = m.d, n = d * d;
  for (int b = 0; b < m.L - 1; ++b) {
    const double* hb = h + (size_t)b * n * n;
    double scale = 0.0;
    for (int i = 0; i < n * n; ++i) {
      if (!std::isfinite(hb[i])) fail(TNT_E_NONFINITE, "bond Hamiltonian entry not finite");
      scale = std::max(scale, std::fabs(hb[i]));
    }
    for (int r = 0; r < n; ++r)
      for (int col = 0; col < n; ++col) {
        const double v = hb[(size_t)r * n + col];
        if (std::fabs(v - hb[(size_t)col * n + r]) > 1e-12 * scale)
          fail(TNT_E_ARG, "bond Hamiltonian " + std::to_string(b + 1) + " not symmetric");
        if (v != 0.0 && r / d + r % d != col / d + col % d)
          fail(TNT_E_CHARGE, "bond Hamiltonian " + std::to_string(b + 1) +
                                 " does not conserve the charge");
      }
  }
  TebdStats st;
  tebd_step(c, m, h, dt, *trunc, st, bond_eps, bond_chi);
  if (stats) {
    stats[0] = st.t_total;
    stats[1] = st.t_gate;
    stats[2] = st.t_svd;
    stats[3] = st.sum_eps;
    stats[4] = st.max_eps;
    stats[5] = st.max_chi;
  }
  TNT_API_END
}

// ---------------------------------------------------------------------------
// environments and sweep
// ---------------------------------------------------------------------------
tnt_status tnt_env_create(tnt_ctx ctx, tnt_mps mps, const tnt_mpo_site* mpo, int32_t left_index,
                          int32_t right_index, tnt_env* out) {
  TNT_API_BEGIN(ctx)
  if (!mps || !mpo || !out) fail(TNT_E_ARG, "null argument");
  MpsObj* mo = reinterpret_cast<MpsObj*>(mps);
  MpsH& m = mo->m;
  auto* eo = new EnvObj{&c, mo, EnvS()};
  try {
    EnvS& e = eo->e;
    e.mps = &m;
    for (int j = 0; j < m.L; ++j) {
      e.W.push_back(parse_mpo(&mpo[j], "mpo"));
      if (e.W.back().d != m.d) fail(TNT_E_SHAPE, "MPO physical dimension differs from the MPS");
      if (j > 0 && (e.W.back().D != e.W[0].D || e.W.back().qw != e.W[0].qw))
        fail(TNT_E_SHAPE, "MPO sites disagree in bond dimension or charges");
    }
    e.qw = e.W[0].qw;
    if (left_index < 0 || left_index >= e.W[0].D || right_index < 0 || right_index >= e.W[0].D)
      fail(TNT_E_ARG, "boundary index out of range");
    e.left_index = left_index;
    e.right_index = right_index;
    for (int j = 1; j <= m.L; ++j)
      if (!m.dat[j - 1].ptr) fail(TNT_E_STATE, "site " + std::to_string(j) + " not set");
    build_boundaries(c, e);
    for (int j = m.L; j >= 3; --j) update_right_env(c, e, j);
  } catch (...) {
    delete eo;
    throw;
  }
  *out = reinterpret_cast<tnt_env>(eo);
  TNT_API_END
}

void tnt_env_destroy(tnt_env env) { delete reinterpret_cast<EnvObj*>(env); }

static void fill_result(const SweepStats& st, tnt_sweep_result* r) {
  r->energy = st.energy;
  r->max_residual = st.max_residual;
  r->max_eps = st.max_eps;
  r->updates = st.updates;
  r->max_chi = st.max_chi;
  r->matvecs = st.matvecs;
  r->matvec_flops = st.matvec_flops;
  r->seconds_total = st.t_total;
  r->seconds_matvec = st.t_matvec;
  r->seconds_lanczos = st.t_lanczos;
  r->seconds_svd = st.t_svd;
  r->seconds_env = st.t_env;
  r->seconds_theta = st.t_theta;
  r->seconds_setup = st.t_setup;
  r->gemm_flops = st.gemm_flops;
  r->seconds_gemm = st.t_gemm;
  r->gemm_launches = st.gemm_launches;
  r->eig_retries = st.eig_retries;
}

tnt_status tnt_dmrg_sweep_batched(tnt_ctx ctx, int32_t n, const tnt_mps* mps, const tnt_env* env,
                                  const tnt_sweep_params* p, tnt_sweep_result* r) {
  TNT_API_BEGIN(ctx)
  if (n < 1 || !mps || !env || !p || !r) fail(TNT_E_ARG, "null or empty batch");
  std::vector<MpsH*> ms;
  std::vector<EnvS*> es;
  for (int i = 0; i < n; ++i) {
    if (!mps[i] || !env[i]) fail(TNT_E_ARG, "null MPS or environment handle");
    MpsObj* mo = reinterpret_cast<MpsObj*>(mps[i]);
    EnvObj* eo = reinterpret_cast<EnvObj*>(env[i]);
    if (eo->mps != mo) fail(TNT_E_STATE, "environment belongs to another MPS");
    if (mo->ctx != &c) fail(TNT_E_STATE, "MPS belongs to another context");
    for (int k = 0; k < i; ++k)
      if (ms[k] == &mo->m) fail(TNT_E_ARG, "an MPS appears twice in the batch");
    check_lanczos(&p[i].lanczos);
    check_trunc(&p[i].trunc);
    if (p[i].lanczos.kmax != p[0].lanczos.kmax ||
        p[i].lanczos.precision != p[0].lanczos.precision ||
        p[i].lanczos.beta_tol != p[0].lanczos.beta_tol)
      fail(TNT_E_ARG, "Lanczos parameters differ within the batch");
    ms.push_back(&mo->m);
    es.push_back(&eo->e);
  }
  std::vector<SweepStats> st;
  dmrg_sweep_batched(c, ms, es, p, st);
  for (int i = 0; i < n; ++i) fill_result(st[i], &r[i]);
  TNT_API_END
}

tnt_status tnt_dmrg_sweep(tnt_ctx ctx, tnt_mps mps, tnt_env env, const tnt_sweep_params* p,
                          tnt_sweep_result* r) {
  TNT_API_BEGIN(ctx)
  if (!mps || !env || !p || !r) fail(TNT_E_ARG, "null argument");
  MpsObj* mo = reinterpret_cast<MpsObj*>(mps);
  EnvObj* eo = reinterpret_cast<EnvObj*>(env);
  if (eo->mps != mo) fail(TNT_E_STATE, "environment belongs to another MPS");
  check_lanczos(&p->lanczos);
  check_trunc(&p->trunc);
  SweepStats st;
  dmrg_sweep(c, mo->m, eo->e, *p, st);
  fill_result(st, r);
  TNT_API_END
}

}  // extern "C"
