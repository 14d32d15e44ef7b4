// Task-list plans for the grouped kernels and their device copies.
#pragma once

#include <memory>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "layout.h"

namespace tnt {

// Host task list of one grouped-GEMM launch.
struct HostGemm {
  std::vector<GemmTask> tasks;
  std::vector<GemmSeg> segs;
  std::vector<int2> tiles;  // built by finalize (the default tile shape)
  int tile_cfg = 0;
  // tile tables of further candidate shapes (autotuning), built by add_variant
  std::vector<int> var_cfg;
  std::vector<std::vector<int2>> var_tiles;
  double flops = 0;         // 8 * sum M N K (complex MACs)

  int add_task(int64_t c_off, int M, int N, int ldc) {
    tasks.push_back(GemmTask{c_off, M, N, ldc, (int)segs.size(), 0, 0});
    return (int)tasks.size() - 1;
  }
  void add_seg(int64_t a_off, int lda, int64_t b_off, int ldb, int K) {
    segs.push_back(GemmSeg{a_off, b_off, K, lda, ldb, 0});
    GemmTask& t = tasks.back();
    t.nseg++;
    flops += 8.0 * t.M * (double)t.N * K;
  }
  // Build the tile table for a tile shape: tasks are spread over the 8 XCD
  // bins by greedy cost balancing (largest first); block b of the launch
  // runs on XCD b % 8 and takes slot b / 8 of that bin (empty slots exit).
  void finalize(int cfg);
  // Tile table of another candidate shape (kept beside the default one).
  void add_variant(int cfg);
  std::vector<int2> build_tiles(int cfg) const;
};

// Host task list of one combine launch.
struct HostComb {
  std::vector<CombTask> tasks;
  std::vector<CombTerm> terms;
  std::vector<int2> chunks;
  double flops = 0;  // 4 per term per element

  void add_task(int64_t dst_off, int size) {
    tasks.push_back(CombTask{dst_off, size, (int)terms.size(), 0, 0});
  }
  void add_term(int64_t src_off, double coef) {
    terms.push_back(CombTerm{src_off, coef});
    tasks.back().nterm++;
    flops += 4.0 * tasks.back().size;
  }
  void finalize();
};

// Host task list of one packed MPO combination (kernels.h CombPTask).
struct HostCombP {
  std::vector<CombPTask> tasks;
  std::vector<CombTerm> terms;
  std::vector<int2> chunks;
  void add_task(int64_t dst_off, int rows, int cols, int dld) {
    tasks.push_back(CombPTask{dst_off, rows, cols, dld, (int)terms.size(), 0, 0});
  }
  void add_term(int64_t src_off, double coef) {
    terms.push_back(CombTerm{src_off, coef});
    tasks.back().nterm++;
  }
  void finalize();
};

// Pack tasks of one packed operand (kernels.h PackTask) and their tiles.
struct HostPack {
  std::vector<PackTask> tasks;
  std::vector<int2> tiles;
  int64_t elems = 0;  // plane stride in elements (a multiple of 8)
  // destination block rows x cols (row stride pad8(cols)) from a source
  // block at src_off with leading dimension sld, read transposed if `trans`;
  // returns the destination offset
  int64_t add(int64_t src_off, int rows, int cols, int sld, bool trans);
};

// Device copy of several host task lists in one allocation.
struct DevTables {
  DevBuf buf;
  std::vector<char> host;  // kept alive until the tables are dropped
  // one grouped GEMM: its tasks and one tile table per candidate shape;
  // `sel` picks the table a launch uses
  struct G {
    const GemmTask* tasks;
    const GemmSeg* segs;
    const int2* tiles[8];
    int ntiles[8];
    int cfg[8];
    int nvar = 0;
    int sel = 0;
  };
  struct C { const CombTask* tasks; const CombTerm* terms; const int2* chunks; int nchunks; };
  struct CP { const CombPTask* tasks; const CombTerm* terms; const int2* chunks; int nchunks; };
  struct P { const PackTask* tasks; const int2* tiles; int ntiles; int64_t elems; };
  std::vector<G> g;
  std::vector<C> c;
  std::vector<CP> cp;
  std::vector<P> p;
  // Copy the lists to the device: into pool memory, or to `dst` (at least
  // image_bytes of the same lists) when given.
  void upload(Ctx& ctx, const std::vector<const HostGemm*>& gs,
              const std::vector<const HostComb*>& cs,
              const std::vector<const HostCombP*>& cps = {},
              const std::vector<const HostPack*>& pks = {}, void* dst = nullptr);
  // Device bytes the lists occupy (256-byte aligned pieces).
  static size_t image_bytes(const std::vector<const HostGemm*>& gs,
                            const std::vector<const HostComb*>& cs,
                            const std::vector<const HostCombP*>& cps = {},
                            const std::vector<const HostPack*>& pks = {});
};

void run_gemm(Ctx& ctx, const DevTables::G& g, GemmForm form, GemmPath path,
              const void* are, const void* aim, ElemType at, const void* bre, const void* bim,
              ElemType bt, void* cre, void* cim, ElemType ct);
void run_gemm_variant(Ctx& ctx, const DevTables::G& g, int v, GemmForm form, GemmPath path,
                      const void* are, const void* aim, ElemType at, const void* bre,
                      const void* bim, ElemType bt, void* cre, void* cim, ElemType ct);
void run_comb(Ctx& ctx, const DevTables::C& c, const void* sre, const void* sim, void* dre,
              void* dim, ElemType t);

// Default tile shape for a task list (used when no tuned choice exists).
int default_tile_cfg(const HostGemm& h, GemmPath path);
// Candidate tile shapes of a path.
std::vector<int> tile_candidates(GemmPath path);
// GEMM path of a TNT_FP64 / TNT_FP32 / TNT_BF16X3 operator
GemmPath gemm_path(int precision);
// Shape bucket of a task list for the tuning cache (path, flop-weighted
// typical block dimension, log2 of the flop count).
uint64_t tune_bucket(const HostGemm& h, GemmPath path, int which);

// ---------------------------------------------------------------------------
// The two-site H_eff plan: step 1 (L . theta), MPO combination, step 4 (. R)
// ---------------------------------------------------------------------------
struct HeffPlan {
  HostGemm step1, step4;
  HostComb mpo;
  int64_t t1_elems = 0, t3_elems = 0;
  // reduced-precision path on packed operands (built when `packed`):
  // step 1 = Lp . Xp^T (Xp: theta packed transposed) into FP32 T1 slabs,
  // the combination writes packed T3 slabs, step 4 = T3p . Rp^T
  bool packed = false;
  HostGemm step1p, step4p;
  HostCombP mpop;
  HostPack Lp, Rp, Xp;
  int64_t t3p_elems = 0;
  int64_t flops_step1 = 0, flops_mpo = 0, flops_step4 = 0;
  int64_t flops() const { return flops_step1 + flops_mpo + flops_step4; }
  std::vector<std::array<int, 3>> out_keys;
};

HeffPlan build_heff_plan(const EnvH& L, const MpoH& W1, const MpoH& W2, const EnvH& R,
                         const ThetaH& th, const ThetaH& out, bool packed);

// Where one instance's operands sit inside a batch: its theta / out blocks
// at complex offset x_off of the batch vector planes, its L and R planes at
// element offsets L_off, R_off of the batch environment planes.
struct BatchPart {
  int64_t x_off, L_off, R_off;
};
// One plan over all instances: task lists concatenated with every operand
// offset moved to the batch buffers (slab, packed-copy and table offsets
// stacked instance after instance).  All plans must agree in `packed`.
HeffPlan merge_heff_plans(const std::vector<const HeffPlan*>& plans,
                          const std::vector<BatchPart>& where);

// A ready-to-apply H_eff operator on one bond: the plan and its device
// tables.  Intermediate slabs and packed operand copies live in the
// context's shared workspaces (Ctx::ws), sized on use: ws[0] T1 slabs,
// ws[1] T3 slabs, ws[2] / ws[3] packed L / R, ws[4] packed theta.
struct HeffOp {
  Ctx* ctx = nullptr;
  HeffPlan plan;
  DevTables tab;
  int precision = TNT_FP64;
  const double* L_re = nullptr; const double* L_im = nullptr;
  const double* R_re = nullptr; const double* R_im = nullptr;
  int64_t L_ext = 0, R_ext = 0;

  // plan + device tables + workspaces for these block structures
  void build(Ctx& c, const EnvH& L, const MpoH& W1, const MpoH& W2, const EnvH& R,
             const ThetaH& th, const ThetaH& out, int prec);
  // the same for a ready plan (a merged batch plan)
  // tunable: time the tile-shape candidates at the first application when
  // the shape bucket has no cached decision (off for one-off operators)
  void build_plan(Ctx& c, HeffPlan&& p, int prec, bool tunable = true);
  // build_plan in two parts: the tile tables on the host, then their copy
  // to the device (pool memory, or `dst` with table_bytes() bytes)
  void plan_tables(Ctx& c, HeffPlan&& p, int prec, bool tunable);
  size_t table_bytes() const;
  void upload_tables(void* dst);
  // Caller-provided workspaces (ws[0..4] roles, see above), used instead of
  // the context's when set; ws_bytes() gives the sizes an application needs.
  void* ext_ws[5] = {};
  void ws_bytes(int prec, int64_t out[5]) const;
  void* wsp(int i) const;
  void ensure_ws(int i, int64_t bytes);
  // point at the environments' FP64 planes (and refresh the packed copies)
  void bind_envs(const void* lre, const void* lim, const void* rre, const void* rim);
  PackFmt fmt() const { return precision == TNT_BF16X3 ? PK_BF16X3 : PK_F32; }
  // y = H_eff x with x, y in the theta / out layouts given at build (FP64 planes).
  // With `tev` (4 events), tev[0]/tev[1] bracket the step-1 GEMM launch and
  // tev[2]/tev[3] the step-4 launch.
  void apply(const double* xre, const double* xim, double* yre, double* yim, int prec,
             const hipEvent_t* tev = nullptr);
  // Everything apply may need before it can run without host interaction
  // (workspaces sized, tile shapes tuned), so that a sequence of applies can
  // be captured into a HIP graph.
  void prepare(const double* xre, const double* xim, double* yre, double* yim, int prec);
  // Captured Lanczos recurrence of this operator (lanczos.cpp), valid while
  // every buffer it references keeps its address.
  struct Graph {
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> key;
  } graph;
  ~HeffOp();
  // Pick the tile shape of each grouped GEMM by timing every candidate on
  // (x -> y) (results do not depend on the shape: every shape sums K in the
  // same order); decisions are cached per shape bucket in the context.
  void autotune(const double* xre, const double* xim, double* yre, double* yim, int prec);
  bool tuned = false;
  // one grouped-GEMM launch of step 1 or 4 with tile table v
  void launch_step(int step, int v, bool fp64, const double* xre, const double* xim,
                   double* yre, double* yim);
};

}  // namespace tnt
