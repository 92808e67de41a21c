// C ABI of librgp: argument validation, workspace layout and the launch sequences of the hot path.
#include <hip/hip_runtime.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rgp.h"
#include "rgp_internal.hpp"
#include "rgp_launch.hpp"
#include "batch.hpp"

namespace rgp {
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_stats_header(double* stats, const State* st, const unsigned long long* guarded,
                               hipStream_t s);
}  // namespace rgp

using namespace rgp;

Recorder*& rgp::active_recorder() {
  thread_local Recorder* r = nullptr;
  return r;
}
bool& rgp::batch_plans() {
  thread_local bool b = false;
  return b;
}
int& rgp::batch_march_min() {
  thread_local int m = 0;
  return m;
}

namespace {

thread_local int g_last_hip = 0;

// Named host ranges (ROCTx) around the phases of a correction while they are enqueued (or
// recorded): a tracer (rocprofv3 --marker-trace) shows them beside the launches they issue.  The
// calls return at once when no tracer is attached.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  Range(const char* fmt, int v) {
    char buf[48];
    std::snprintf(buf, sizeof buf, fmt, v);
    roctxRangePushA(buf);
  }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// ---- kernel timing registry -------------------------------------------------------------
struct TimingRec {
  int kind, tag;
  unsigned grid;
  int64_t cells, nodes;
  hipEvent_t e0, e1;
};
std::mutex g_timing_mu;
std::atomic<bool> g_timing_on{false};
std::vector<TimingRec> g_timing;
size_t g_timing_used = 0;

constexpr size_t kAlign = 256;
constexpr double kGuardSlope = 0.99;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool dtype_of(rgp_dtype t, DType* out) {
  switch (t) {
    case RGP_F64: *out = DType::F64; return true;
    case RGP_F32: *out = DType::F32; return true;
    case RGP_BF16: *out = DType::BF16; return true;
  }
  return false;
}

size_t dsize(DType t) { return t == DType::F64 ? 8 : (t == DType::F32 ? 4 : 2); }

rgp_status check_types(rgp_dtype img, rgp_dtype real, DType* di, DType* dr) {
  if (!dtype_of(img, di) || !dtype_of(real, dr)) return RGP_EINVAL;
  if (*dr == DType::BF16) return RGP_EDTYPE;
  if (*dr == DType::F32 && *di == DType::F64) return RGP_EDTYPE;
  return RGP_OK;
}

rgp_status check_grid(const rgp_grid* g) {
  if (!g) return RGP_EINVAL;
  if (g->pe < 0 || g->pe > 2) return RGP_EINVAL;
  int64_t cells = 1, nodes = 1;
  for (int d = 0; d < 3; ++d) {
    if (g->m[d] < 1 || g->m[d] > (int64_t(1) << 24)) return RGP_ESHAPE;
    if (!(g->h[d] > 0.0) || !std::isfinite(g->h[d])) return RGP_EINVAL;
    cells *= g->m[d];
    nodes *= g->m[d] + (d == g->pe ? 1 : 0);
    if (nodes > (int64_t(1) << 28)) return RGP_ESHAPE;
  }
  if (g->m[g->pe] < 2) return RGP_ESHAPE;
  // the contiguous axis of the field (its two halo rows are held by at most 1024 lanes)
  if (g->m[2] + (g->pe == 2 ? 1 : 0) > 512) return RGP_ESHAPE;
  (void)cells;
  return RGP_OK;
}

Geom make_geom(const int64_t m[3], int pe, const double h[3]) {
  Geom g{};
  int ax[2], k = 0;
  for (int d = 0; d < 3; ++d)
    if (d != pe) ax[k++] = d;
  int64_t n[3];
  for (int d = 0; d < 3; ++d) n[d] = m[d] + (d == pe ? 1 : 0);
  const int64_t cst[3] = {m[1] * m[2], m[2], 1};
  const int64_t nst[3] = {n[1] * n[2], n[2], 1};
  g.mp = (int32_t)m[pe];
  g.nx = (int32_t)m[ax[0]];
  g.ny = (int32_t)m[ax[1]];
  g.pe = pe;
  g.ncol = (int64_t)g.nx * g.ny;
  g.cxs = cst[ax[0]];
  g.cys = cst[ax[1]];
  g.cps = cst[pe];
  g.nxs = nst[ax[0]];
  g.nys = nst[ax[1]];
  g.nps = nst[pe];
  g.ncell = m[0] * m[1] * m[2];
  g.nnode = n[0] * n[1] * n[2];
  g.hx = h[ax[0]];
  g.hy = h[ax[1]];
  g.hp = h[pe];
  g.vol = h[0] * h[1] * h[2];
  g.by_ny = make_fastdiv((uint32_t)g.ny);
  g.by_nct = make_fastdiv((uint32_t)((g.ncol + kWave - 1) / kWave));
  return g;
}

Geom geom_of(const rgp_grid* gr) { return make_geom(gr->m, gr->pe, gr->h); }

// Bump allocator over the caller's workspace (sizes computed with a null base).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t bytes) {
    off = align_up(off);
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

// Slots of block sums (kMaxGrid blocks x kPartStride doubles each).
enum PartSlot { kPartLoss = 0, kPartPcg0, kPartPcg1, kPartTrial0, kPartTrial1, kPartTrial2,
                kPartHvp, kPartShift, kPartSlots };

struct Control {
  State* st;
  PcgSlot* slots;
  unsigned long long* guarded;
  double* part;
  double* slot(int k) const { return part + (size_t)k * kMaxGrid * kPartStride; }
};

Control carve_control(Carver& c) {
  Control k;
  k.st = static_cast<State*>(c.take(sizeof(State)));
  k.slots = static_cast<PcgSlot*>(c.take(2 * sizeof(PcgSlot)));
  k.guarded = static_cast<unsigned long long*>(c.take(sizeof(unsigned long long)));
  k.part = static_cast<double*>(c.take((size_t)kPartSlots * kMaxGrid * kPartStride * sizeof(double)));
  return k;
}

// Level geometry of the pyramid: level 0 is the caller's grid.
struct Level {
  int64_t m[3];
  double h[3];
  Geom g;
};

int make_levels(const rgp_grid* gr, int levels, Level* out) {
  for (int l = 0; l < levels; ++l) {
    for (int d = 0; d < 3; ++d) {
      out[l].m[d] = l == 0 ? gr->m[d] : (out[l - 1].m[d] + 1) / 2;
      out[l].h[d] = l == 0 ? gr->h[d] : 2.0 * out[l - 1].h[d];
    }
    if (out[l].m[gr->pe] < 2) return -1;
    out[l].g = make_geom(out[l].m, gr->pe, out[l].h);
  }
  return 0;
}

constexpr int kMaxLevels = 12;

struct CorrectWs {
  Control ctl;
  void* img[kMaxLevels][2];  // levels >= 1 (real type)
  void* B[2];
  void* G;
  void* Dg;
  void* Of;
  void* X;
  void* R[2];
  void* P[2];
  void* W[2];
  // L-BFGS only: the gradient of the previous step, the pair rings (mem + 1 slots each), the
  // metadata of two consecutive steps and the block sums of a step's inner products
  void* G2 = nullptr;
  void* S = nullptr;
  void* Y = nullptr;
  LbfgsMeta* meta = nullptr;
  double* lb_part = nullptr;
};

// Lays the correction's buffers out from ws (a null ws only counts); *bytes: the total size.
CorrectWs carve_correct(void* ws, const Level* lv, int levels, DType real,
                        const rgp_solver_opts* o, size_t* bytes = nullptr) {
  Carver c(ws);
  CorrectWs w;
  w.ctl = carve_control(c);
  const size_t rs = dsize(real);
  for (int l = 0; l < kMaxLevels; ++l) w.img[l][0] = w.img[l][1] = nullptr;
  for (int l = 1; l < levels; ++l) {
    w.img[l][0] = c.take(lv[l].g.ncell * rs);
    w.img[l][1] = c.take(lv[l].g.ncell * rs);
  }
  const size_t nb = lv[0].g.nnode * rs;
  w.B[0] = c.take(nb);
  w.B[1] = c.take(nb);
  w.G = c.take(nb);
  w.Dg = c.take(nb);
  w.Of = c.take(nb);
  w.X = c.take(nb);
  for (int i = 0; i < 2; ++i) {
    w.R[i] = c.take(nb);
    w.P[i] = c.take(nb);
    w.W[i] = c.take(nb);
  }
  if (o->solver == RGP_SOLVER_LBFGS) {
    w.G2 = c.take(nb);
    w.S = c.take(nb * (size_t)(o->lbfgs_memory + 1));
    w.Y = c.take(nb * (size_t)(o->lbfgs_memory + 1));
    w.meta = static_cast<LbfgsMeta*>(c.take(2 * sizeof(LbfgsMeta)));
    w.lb_part = static_cast<double*>(
        c.take((size_t)kLbfgsSums(o->lbfgs_memory) * kMaxGrid * sizeof(double)));
  }
  if (bytes) *bytes = align_up(c.off);
  return w;
}

size_t correct_bytes(const Level* lv, int levels, DType real, const rgp_solver_opts* o) {
  size_t bytes = 0;
  carve_correct(nullptr, lv, levels, real, o, &bytes);
  return bytes;
}

#define RGP_HIP(call)                          \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) {                    \
      g_last_hip = (int)e_;                    \
      return RGP_EHIP;                         \
    }                                          \
  } while (0)

rgp_status check_opts(const rgp_solver_opts* o) {
  if (!o) return RGP_EINVAL;
  if (!(o->alpha >= 0.0) || !(o->beta >= 0.0) || !std::isfinite(o->alpha) ||
      !std::isfinite(o->beta))
    return RGP_EINVAL;
  if (o->levels < 1 || o->levels > kMaxLevels) return RGP_EINVAL;
  if (o->gn_iters < 0 || o->gn_iters > 10000) return RGP_EINVAL;
  if (o->pcg_iters < 1 || o->pcg_iters > 1000) return RGP_EINVAL;
  if (o->ls_max_trials < 1 || o->ls_max_trials > 10) return RGP_EINVAL;
  if (!(o->pcg_rtol >= 0.0) || !(o->armijo_c >= 0.0) || !(o->ot_eps >= 0.0)) return RGP_EINVAL;
  if (o->ot_blur != 0 && o->ot_blur != 1) return RGP_EINVAL;
  if (o->solver != RGP_SOLVER_GN && o->solver != RGP_SOLVER_LBFGS &&
      o->solver != RGP_SOLVER_ADMM)
    return RGP_EINVAL;
  if (o->solver == RGP_SOLVER_ADMM && (!(o->alpha > 0.0) || !std::isfinite(o->admm_rho0)))
    return RGP_EINVAL;
  if (o->solver == RGP_SOLVER_LBFGS && (o->lbfgs_memory < 1 || o->lbfgs_memory > kLbfgsMaxMem))
    return RGP_EINVAL;
  if (o->batch_march < 0 || o->batch_march > kMarchMax) return RGP_EINVAL;
  return RGP_OK;
}

// The Armijo passes of one step on the direction in w.X: gamma = 1 alone (it is accepted in most
// steps), then the remaining candidates 2^-1 .. 2^-9 in one pass; a pass after an accepted step
// exits at once.
hipError_t armijo_passes(const CorrectWs& w, const Geom& g, const void* Ip, const void* Im,
                         DType img, DType real, const rgp_solver_opts* o, const void* b,
                         const void* grad, double* rec, hipStream_t s,
                         const void* prox_c = nullptr) {
  hipError_t e;
  const Control& k = w.ctl;
  int first = 0;
  const int passes[2] = {1, kMaxTrialCand};
  for (int p = 0; p < 2 && first < o->ls_max_trials; ++p) {
    const int nc = std::min(passes[p], o->ls_max_trials - first);
    TrialArgs ta{};
    ta.g = g;
    ta.Ip = Ip;
    ta.Im = Im;
    ta.b = b;
    ta.q = w.X;
    ta.grad = grad;
    ta.alpha = o->alpha;
    ta.beta = o->beta;
    ta.armijo_c = o->armijo_c;
    ta.st = k.st;
    ta.part = k.slot(kPartTrial0 + p);
    ta.first = first;
    ta.nc = nc;
    ta.prox_c = prox_c;
    if ((e = launch_trial(ta, img, real, s)) != hipSuccess) return e;
    DecideArgs da{};
    da.part_prev = ta.part;
    da.nprod_prev = plan_trial(g, real, nc).grid;
    da.prev_first = first;
    da.prev_nc = nc;
    da.total = o->ls_max_trials;
    da.vol = g.vol;
    da.alpha = o->alpha;
    da.beta = o->beta;
    da.armijo_c = o->armijo_c;
    da.st = k.st;
    da.record = rec;
    if ((e = launch_decide(da, s)) != hipSuccess) return e;
    first += nc;
  }
  return hipSuccess;
}

// `gn_iters` L-BFGS steps on one level (Sec. 2.3.3).  Each step: the objective and gradient at
// the current iterate (applying the previous accepted step), the new curvature pair, the two-loop
// recursion into w.X, and the Armijo passes of the Gauss-Newton solve.  The gradients of
// consecutive steps alternate between w.G and w.G2.  b enters and leaves in B[cur].
hipError_t run_level_lbfgs(const CorrectWs& w, const Geom& g, const void* Ip, const void* Im,
                           DType img, DType real, const rgp_solver_opts* o, int& cur,
                           double* records, hipStream_t s) {
  hipError_t e;
  const Control& k = w.ctl;
  const Launch Llg = plan_loss_grad(g, real);
  const unsigned nblk_dots = lbfgs_dots_grid(g.nnode);
  const int mem = o->lbfgs_memory;
  void* grads[2] = {w.G, w.G2};
  for (int it = 0; it < o->gn_iters; ++it) {
    double* rec = records ? records + (size_t)it * kStatFields : nullptr;
    void* gcur = grads[it & 1];
    LossGradArgs la{};
    la.g = g;
    la.Ip = Ip;
    la.Im = Im;
    la.b_in = w.B[cur];
    la.q = w.X;
    la.step = it > 0;
    la.level_start = it == 0;
    la.b_out = it > 0 ? w.B[1 - cur] : nullptr;
    la.grad = gcur;
    la.alpha = o->alpha;
    la.beta = o->beta;
    la.st = k.st;
    la.part = k.slot(kPartLoss);
    if ((e = launch_loss_grad(la, img, real, s)) != hipSuccess) return e;
    if (it > 0) cur = 1 - cur;

    LbfgsArgs a{};
    a.n = g.nnode;
    a.g = gcur;
    a.g_old = grads[(it + 1) & 1];
    a.x = w.X;
    a.S = w.S;
    a.Y = w.Y;
    a.meta_prev = w.meta + ((it + 1) & 1);
    a.meta = w.meta + (it & 1);
    a.part = w.lb_part;
    a.part_max = k.slot(kPartHvp);
    a.nprod = nblk_dots;
    a.st = k.st;
    a.mem = mem;
    a.pair = it > 0 ? 1 : 0;
    // the new pair needs gamma of the previous step: before the state is reset below
    a.phase = kLbDots;
    if ((e = launch_lbfgs(a, real, s)) != hipSuccess) return e;
    if ((e = launch_loss_final(LossFinalArgs{k.slot(kPartLoss), Llg.grid, g.vol, o->alpha,
                                             o->beta, k.st, nullptr, rec, 1},
                               s)) != hipSuccess)
      return e;
    a.phase = kLbScalar;
    if ((e = launch_lbfgs(a, real, s)) != hipSuccess) return e;
    a.phase = kLbCombine;
    if ((e = launch_lbfgs(a, real, s)) != hipSuccess) return e;
    if ((e = armijo_passes(w, g, Ip, Im, img, real, o, w.B[cur], gcur, rec, s)) != hipSuccess)
      return e;
  }
  if (o->gn_iters > 0) {
    ApplyArgs aa{};
    aa.b = w.B[cur];
    aa.q = w.X;
    aa.st = k.st;
    aa.n = g.nnode;
    if ((e = launch_apply_step(aa, real, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// `gn_iters` ADMM iterations on one level (Sec. 2.3.2).  Per iteration: the b-update (the
// objective, gradient and tridiagonal Gauss-Newton blocks of F_rho at b, block PCG per column,
// the Armijo passes on F_rho, b += gamma q), the z-update (four transform passes, the last also
// updating u and c = z - u), the adaptation of rho and the rescaling of u it asks for.  z, u and
// c live in the PCG vectors of the workspace (unused by ADMM), the transform passes' scratch in
// two more of them.  b enters and leaves in B[cur].
hipError_t run_level_admm(const CorrectWs& w, const Geom& g, const int64_t m[3], int pe,
                          const double h[3], const void* Ip, const void* Im, DType img,
                          DType real, const rgp_solver_opts* o, int cur, double* records,
                          hipStream_t s) {
  hipError_t e;
  const Control& k = w.ctl;
  const Launch Llg = plan_loss_grad(g, real);
  void* z = w.R[0];
  void* u = w.R[1];
  void* c = w.P[0];
  void* t1 = w.P[1];
  void* t2 = w.W[0];
  int ax[2], na = 0;
  for (int d = 0; d < 3; ++d)
    if (d != pe) ax[na++] = d;
  const int A = ax[0], B = ax[1];   // B: the faster cross axis
  int32_t n[3];
  for (int d = 0; d < 3; ++d) n[d] = (int32_t)(m[d] + (d == pe ? 1 : 0));
  AdmmVecArgs va{};
  va.n = g.nnode;
  va.b = w.B[cur];
  va.z = z;
  va.u = u;
  va.c = c;
  va.rho0 = o->admm_rho0 > 0.0 ? o->admm_rho0 : o->alpha;
  va.st = k.st;
  if ((e = launch_admm_vec(va, true, real, s)) != hipSuccess) return e;
  for (int it = 0; it < o->gn_iters; ++it) {
    double* rec = records ? records + (size_t)it * kStatFields : nullptr;
    LossGradArgs la{};
    la.g = g;
    la.Ip = Ip;
    la.Im = Im;
    la.b_in = w.B[cur];
    la.step = 0;
    la.level_start = it == 0;
    la.grad = w.G;
    la.diag = w.Dg;
    la.off = w.Of;
    la.alpha = o->alpha;
    la.beta = o->beta;
    la.st = k.st;
    la.part = k.slot(kPartLoss);
    la.prox_c = c;
    if ((e = launch_loss_grad(la, img, real, s)) != hipSuccess) return e;
    if ((e = launch_loss_final(LossFinalArgs{k.slot(kPartLoss), Llg.grid, g.vol, o->alpha,
                                             o->beta, k.st, nullptr, rec, 1},
                               s)) != hipSuccess)
      return e;
    BlockPcgArgs bp{};
    bp.g = g;
    bp.diag = w.Dg;
    bp.off = w.Of;
    bp.grad = w.G;
    bp.x = w.X;
    bp.maxit = o->pcg_iters;
    bp.rtol = o->pcg_rtol;
    bp.st = k.st;
    bp.part = k.slot(kPartPcg0);
    if ((e = launch_block_pcg(bp, real, s)) != hipSuccess) return e;
    if ((e = armijo_passes(w, g, Ip, Im, img, real, o, w.B[cur], w.G, rec, s, c)) != hipSuccess)
      return e;
    ApplyArgs aa{};
    aa.b = w.B[cur];
    aa.q = w.X;
    aa.st = k.st;
    aa.n = g.nnode;
    if ((e = launch_apply_step(aa, real, s)) != hipSuccess) return e;
    // z-update: B from rho (b + u), A with the scaling, A, B with the multiplier update
    DhtArgs da{};
    for (int d = 0; d < 3; ++d) da.n[d] = n[d];
    da.b = w.B[cur];
    da.u = u;
    da.c = c;
    da.alpha = o->alpha;
    da.st = k.st;
    da.part = k.slot(kPartPcg1);
    const int modes[4] = {kDhtFirst, kDhtScale, kDhtPlain, kDhtLast};
    const int axes[4] = {B, A, A, B};
    const void* srcs[4] = {nullptr, t1, t2, t1};
    void* dsts[4] = {t1, t2, t1, z};
    for (int p = 0; p < 4; ++p) {
      da.mode = modes[p];
      da.axis = axes[p];
      da.other_axis = axes[p] == A ? B : A;
      da.inv_h2[0] = 1.0 / (h[da.axis] * h[da.axis]);
      da.inv_h2[1] = 1.0 / (h[da.other_axis] * h[da.other_axis]);
      da.src = srcs[p];
      da.dst = dsts[p];
      if ((e = launch_dht(da, real, s)) != hipSuccess) return e;
    }
    int lpb = 0;
    const unsigned nprod = dht_grid(n, B, &lpb);
    if ((e = launch_admm_rho(AdmmRhoArgs{k.st, k.slot(kPartPcg1), nprod, rec}, s)) != hipSuccess)
      return e;
    if ((e = launch_admm_vec(va, false, real, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// `gn_iters` Gauss-Newton steps on one level.  b enters in B[cur]; on return the final field is
// in B[cur].
hipError_t run_level(const CorrectWs& w, const Geom& g, const void* Ip, const void* Im, DType img,
                     DType real, const rgp_solver_opts* o, int& cur, double* records,
                     hipStream_t s) {
  hipError_t e;
  const Control& k = w.ctl;
  const Launch Llg = plan_loss_grad(g, real);
  const PcgPlan Lpcg = plan_pcg(g, real);
  for (int it = 0; it < o->gn_iters; ++it) {
    const Range range("rgp: Gauss-Newton step %d", it);
    double* rec = records ? records + (size_t)it * kStatFields : nullptr;
    LossGradArgs la{};
    la.g = g;
    la.Ip = Ip;
    la.Im = Im;
    la.b_in = w.B[cur];
    la.q = w.X;
    la.step = it > 0;
    la.level_start = it == 0;
    la.b_out = it > 0 ? w.B[1 - cur] : nullptr;
    la.grad = w.G;
    la.diag = w.Dg;
    la.off = w.Of;
    la.alpha = o->alpha;
    la.beta = o->beta;
    la.st = k.st;
    la.part = k.slot(kPartLoss);
    if ((e = launch_loss_grad(la, img, real, s)) != hipSuccess) return e;
    if (it > 0) cur = 1 - cur;

    for (int i = 0; i <= o->pcg_iters; ++i) {
      const int in = (i + 1) & 1, out = i & 1;
      PcgScalarArgs sa{};
      sa.st = k.st;
      sa.slots = k.slots;
      sa.part_prev = k.slot(kPartPcg0 + in);
      sa.nprod = Lpcg.grid;
      sa.iter = i;
      sa.maxit = o->pcg_iters;
      sa.rtol = o->pcg_rtol;
      sa.gn_mode = 1;
      sa.fused = Lpcg.fused;
      sa.lf = LossFinalArgs{k.slot(kPartLoss), Llg.grid, g.vol, o->alpha, o->beta, k.st,
                            nullptr, rec, 1};
      if (!sa.fused && (e = launch_pcg_scalars(sa, s)) != hipSuccess) return e;
      PcgArgs pa{};
      pa.g = g;
      pa.diag = w.Dg;
      pa.off = w.Of;
      pa.rhs = w.G;
      pa.rhs_sign = -1.0;
      pa.x = w.X;
      pa.r_in = w.R[in];
      pa.p_in = w.P[in];
      pa.w_in = w.W[in];
      pa.r_out = w.R[out];
      pa.p_out = w.P[out];
      pa.w_out = w.W[out];
      pa.alpha = o->alpha;
      pa.part = k.slot(kPartPcg0 + out);
      pa.sc = sa;
      if ((e = launch_pcg_step(pa, real, s)) != hipSuccess) return e;
    }

    if ((e = armijo_passes(w, g, Ip, Im, img, real, o, w.B[cur], w.G, rec, s)) != hipSuccess)
      return e;
  }
  if (o->gn_iters > 0) {
    ApplyArgs aa{};
    aa.b = w.B[cur];
    aa.q = w.X;
    aa.st = k.st;
    aa.n = g.nnode;
    if ((e = launch_apply_step(aa, real, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* rgp_status_string(rgp_status s) {
  switch (s) {
    case RGP_OK: return "ok";
    case RGP_EINVAL: return "invalid argument";
    case RGP_ESHAPE: return "grid extents out of range";
    case RGP_EDTYPE: return "unsupported dtype combination";
    case RGP_ENONFINITE: return "an input image holds a non-finite value";
    case RGP_EBARRIER: return "a level started outside the barrier (|d b / d v| >= 1)";
    case RGP_ELINESEARCH: return "no Armijo trial step was accepted";
    case RGP_EHIP: return "HIP runtime error";
    case RGP_EWORKSPACE: return "workspace missing or too small";
  }
  return "unknown status";
}

int rgp_last_hip_error(void) { return g_last_hip; }

void rgp_default_opts(rgp_solver_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->alpha = 300.0;
  o->beta = 1e-4;
  o->levels = 1;
  o->gn_iters = 5;
  o->pcg_iters = 10;
  o->ls_max_trials = 10;
  o->pcg_rtol = 0.1;
  o->armijo_c = 1e-4;
  o->ot_eps = 1e-3;
  o->ot_guard = 1;
  o->use_b_init = 0;
  o->ot_blur = 0;
  o->solver = RGP_SOLVER_GN;
  o->lbfgs_memory = 10;
  o->admm_rho0 = 0.0;
}

rgp_status rgp_workspace_size(rgp_op op, const rgp_grid* grid, rgp_dtype real_t,
                              const rgp_solver_opts* opts, size_t* bytes) {
  if (!bytes) return RGP_EINVAL;
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  DType dr;
  if (!dtype_of(real_t, &dr) || dr == DType::BF16) return RGP_EDTYPE;
  const Geom g = geom_of(grid);
  Carver c(nullptr);
  switch (op) {
    case RGP_OP_OT_INIT:
    case RGP_OP_LOSS_GRAD:
    case RGP_OP_GN_HVP:
    case RGP_OP_APPLY_CORRECTION:
      carve_control(c);
      break;
    case RGP_OP_PCG_SOLVE:
      carve_control(c);
      for (int i = 0; i < 6; ++i) c.take(g.nnode * dsize(dr));
      break;
    case RGP_OP_CORRECT: {
      if ((st = check_opts(opts)) != RGP_OK) return st;
      Level lv[kMaxLevels];
      if (make_levels(grid, opts->levels, lv) != 0) return RGP_ESHAPE;
      *bytes = correct_bytes(lv, opts->levels, dr, opts);
      return RGP_OK;
    }
    default:
      return RGP_EINVAL;
  }
  *bytes = align_up(c.off);
  return RGP_OK;
}

static rgp_status need_ws(rgp_op op, const rgp_grid* grid, rgp_dtype real_t,
                          const rgp_solver_opts* opts, void* ws, size_t ws_bytes) {
  size_t need = 0;
  rgp_status st = rgp_workspace_size(op, grid, real_t, opts, &need);
  if (st != RGP_OK) return st;
  if (!ws || ws_bytes < need) return RGP_EWORKSPACE;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return RGP_EWORKSPACE;
  return RGP_OK;
}

rgp_status rgp_ot_init(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                       const void* I_minus, rgp_dtype real_t, void* b0, double ot_eps,
                       int32_t guard, uint64_t* n_guarded_dev, void* ws, size_t ws_bytes,
                       void* stream) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  if (!ot_column_supported((int)grid->m[grid->pe])) return RGP_ESHAPE;
  DType di, dr;
  if ((st = check_types(img_t, real_t, &di, &dr)) != RGP_OK) return st;
  if (!I_plus || !I_minus || !b0 || !(ot_eps >= 0.0)) return RGP_EINVAL;
  if ((st = need_ws(RGP_OP_OT_INIT, grid, real_t, nullptr, ws, ws_bytes)) != RGP_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const Geom g = geom_of(grid);
  Carver c(ws);
  Control k = carve_control(c);
  unsigned long long* gd = n_guarded_dev ? reinterpret_cast<unsigned long long*>(n_guarded_dev)
                                         : k.guarded;
  RGP_HIP(launch_shift(ShiftArgs{I_plus, I_minus, g.ncell, k.slot(kPartShift), gd}, di, s));
  OtArgs oa{};
  oa.g = g;
  oa.Ip = I_plus;
  oa.Im = I_minus;
  oa.b0 = b0;
  oa.st = k.st;
  oa.shift_part = k.slot(kPartShift);
  oa.shift_nprod = shift_grid(g.ncell);
  oa.eps = ot_eps;
  oa.guard = guard ? 1 : 0;
  oa.guard_slope = kGuardSlope;
  oa.guarded = gd;
  RGP_HIP(launch_ot(oa, di, dr, s));
  return RGP_OK;
}

// Shape checks of the image-only pyramid transfers: only m is read.
static rgp_status check_image_grid(const rgp_grid* g, RestrictArgs* ra) {
  if (!g) return RGP_EINVAL;
  int64_t cells = 1;
  for (int d = 0; d < 3; ++d) {
    if (g->m[d] < 1 || g->m[d] > (int64_t(1) << 24)) return RGP_ESHAPE;
    cells *= g->m[d];
    if (cells > (int64_t(1) << 28)) return RGP_ESHAPE;
    ra->mf[d] = g->m[d];
    ra->mc[d] = (g->m[d] + 1) / 2;
  }
  return RGP_OK;
}

rgp_status rgp_restrict_image(const rgp_grid* grid, rgp_dtype img_t, const void* src,
                              rgp_dtype real_t, void* dst, void* stream) {
  RestrictArgs ra{};
  rgp_status st = check_image_grid(grid, &ra);
  if (st != RGP_OK) return st;
  DType di, dr;
  if ((st = check_types(img_t, real_t, &di, &dr)) != RGP_OK) return st;
  if (!src || !dst || src == dst) return RGP_EINVAL;
  ra.src = src;
  ra.dst = dst;
  RGP_HIP(launch_restrict(ra, di, dr, static_cast<hipStream_t>(stream)));
  return RGP_OK;
}

rgp_status rgp_restrict_image_adjoint(const rgp_grid* grid, rgp_dtype real_t,
                                      const void* g_coarse, void* g_fine, int32_t accumulate,
                                      void* stream) {
  RestrictArgs ra{};
  rgp_status st = check_image_grid(grid, &ra);
  if (st != RGP_OK) return st;
  DType dr;
  if (!dtype_of(real_t, &dr)) return RGP_EINVAL;
  if (dr == DType::BF16) return RGP_EDTYPE;
  if (!g_coarse || !g_fine || g_coarse == g_fine) return RGP_EINVAL;
  RestrictAdjArgs aa{};
  aa.src = g_coarse;
  aa.dst = g_fine;
  for (int d = 0; d < 3; ++d) {
    aa.mf[d] = ra.mf[d];
    aa.mc[d] = ra.mc[d];
  }
  aa.accumulate = accumulate != 0;
  RGP_HIP(launch_restrict_adjoint(aa, dr, static_cast<hipStream_t>(stream)));
  return RGP_OK;
}

rgp_status rgp_blur_field(const rgp_grid* grid, rgp_dtype real_t, const void* b_in, void* b_out,
                          void* stream) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  DType dr;
  if (!dtype_of(real_t, &dr) || dr == DType::BF16) return RGP_EDTYPE;
  if (!b_in || !b_out || b_in == b_out) return RGP_EINVAL;
  BlurArgs ba{};
  ba.src = b_in;
  ba.dst = b_out;
  for (int d = 0; d < 3; ++d) ba.n[d] = (uint32_t)(grid->m[d] + (d == grid->pe ? 1 : 0));
  ba.cells = grid->m[0] * grid->m[1] * grid->m[2];
  RGP_HIP(launch_blur(ba, dr, static_cast<hipStream_t>(stream)));
  return RGP_OK;
}

}  // extern "C"

namespace {

// Argument checks of rgp_loss_grad and rgp_loss_grad_noalloc (everything but the workspace).
rgp_status check_loss_grad(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                           const void* I_minus, rgp_dtype real_t, const void* b, double alpha,
                           double beta, const void* hdiag, const void* hoff, DType* di,
                           DType* dr) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  if ((st = check_types(img_t, real_t, di, dr)) != RGP_OK) return st;
  if (!I_plus || !I_minus || !b) return RGP_EINVAL;
  if ((hdiag == nullptr) != (hoff == nullptr)) return RGP_EINVAL;
  if (!(alpha >= 0.0) || !(beta >= 0.0) || !std::isfinite(alpha) || !std::isfinite(beta))
    return RGP_EINVAL;
  return RGP_OK;
}

// The launches of one objective/gradient evaluation: loss_grad writes its FP64 block sums to
// `part` (kMaxGrid * kPartStride doubles), and the final reduction turns them into J, D, S, P,
// using `st` as its state block.  Every block sum the reduction reads is written by the same
// launch, so neither buffer has to hold anything on entry.
rgp_status enqueue_loss_grad(const rgp_grid* grid, DType di, DType dr, const void* I_plus,
                             const void* I_minus, const void* b, double alpha, double beta,
                             double* jdsp_dev, void* grad, void* hdiag, void* hoff, State* st,
                             double* part, hipStream_t s) {
  const Geom g = geom_of(grid);
  LossGradArgs la{};
  la.g = g;
  la.Ip = I_plus;
  la.Im = I_minus;
  la.b_in = b;
  la.grad = grad;
  la.diag = hdiag;
  la.off = hoff;
  la.alpha = alpha;
  la.beta = beta;
  la.st = st;
  la.part = part;
  RGP_HIP(launch_loss_grad(la, di, dr, s));
  if (jdsp_dev) {
    const Launch L = plan_loss_grad(g, dr);
    RGP_HIP(launch_loss_final(
        LossFinalArgs{part, L.grid, g.vol, alpha, beta, st, jdsp_dev, nullptr, 0}, s));
  }
  return RGP_OK;
}

// ---- allocation-free objective/gradient ----------------------------------------------------
// rgp_loss_grad_noalloc keeps its state block and loss_grad's block sums in this file-scope
// device array instead of a caller workspace.  Each GPU holds its own copy (at its own address)
// for the life of the process.  In host code `scratch` only names the symbol: its device address
// comes from hipGetSymbolAddress, taken once per device and kept in g_scratch_addr.
constexpr size_t kScratchStateBytes = 256;
constexpr size_t kScratchBytes =
    kScratchStateBytes + (size_t)kMaxGrid * kPartStride * sizeof(double);  // 512.25 KiB
static_assert(sizeof(State) <= kScratchStateBytes, "State must fit the scratch header");
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up on first use).
rgp_status scratch_of_current_device(void** out) {
  int dev = -1;
  RGP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return RGP_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    RGP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return RGP_EHIP;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return RGP_OK;
}

}  // namespace

extern "C" {

rgp_status rgp_loss_grad(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                         const void* I_minus, rgp_dtype real_t, const void* b, double alpha,
                         double beta, double* jdsp_dev, void* grad, void* hdiag, void* hoff,
                         void* ws, size_t ws_bytes, void* stream) {
  DType di, dr;
  rgp_status st = check_loss_grad(grid, img_t, I_plus, I_minus, real_t, b, alpha, beta, hdiag,
                                  hoff, &di, &dr);
  if (st != RGP_OK) return st;
  if ((st = need_ws(RGP_OP_LOSS_GRAD, grid, real_t, nullptr, ws, ws_bytes)) != RGP_OK) return st;
  Carver c(ws);
  Control k = carve_control(c);
  return enqueue_loss_grad(grid, di, dr, I_plus, I_minus, b, alpha, beta, jdsp_dev, grad, hdiag,
                           hoff, k.st, k.slot(kPartLoss), static_cast<hipStream_t>(stream));
}

rgp_status rgp_loss_grad_noalloc(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                                 const void* I_minus, rgp_dtype real_t, const void* b,
                                 double alpha, double beta, double* jdsp_dev, void* grad,
                                 void* hdiag, void* hoff, void* stream) {
  DType di, dr;
  rgp_status st = check_loss_grad(grid, img_t, I_plus, I_minus, real_t, b, alpha, beta, hdiag,
                                  hoff, &di, &dr);
  if (st != RGP_OK) return st;
  // the launch's block sums must fit the scratch (loss_grad grids are capped at kMaxGrid blocks)
  const Launch L = plan_loss_grad(geom_of(grid), dr);
  if (L.grid < 1 || L.grid > (unsigned)kMaxGrid) return RGP_EWORKSPACE;
  void* base = nullptr;
  if ((st = scratch_of_current_device(&base)) != RGP_OK) return st;
  unsigned char* p = static_cast<unsigned char*>(base);
  return enqueue_loss_grad(grid, di, dr, I_plus, I_minus, b, alpha, beta, jdsp_dev, grad, hdiag,
                           hoff, reinterpret_cast<State*>(p),
                           reinterpret_cast<double*>(p + kScratchStateBytes),
                           static_cast<hipStream_t>(stream));
}

rgp_status rgp_gn_hvp(const rgp_grid* grid, rgp_dtype real_t, const void* hdiag,
                      const void* hoff, double alpha, const void* v, void* Hv, double* vHv_dev,
                      void* ws, size_t ws_bytes, void* stream) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  DType dr;
  if (!dtype_of(real_t, &dr)) return RGP_EINVAL;
  if (dr == DType::BF16) return RGP_EDTYPE;
  if (!hdiag || !hoff || !v || !Hv || !(alpha >= 0.0) || !std::isfinite(alpha)) return RGP_EINVAL;
  if ((st = need_ws(RGP_OP_GN_HVP, grid, real_t, nullptr, ws, ws_bytes)) != RGP_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const Geom g = geom_of(grid);
  Carver c(ws);
  Control k = carve_control(c);
  HvpArgs ha{};
  ha.g = g;
  ha.diag = hdiag;
  ha.off = hoff;
  ha.v = v;
  ha.Hv = Hv;
  ha.alpha = alpha;
  ha.part = vHv_dev ? k.slot(kPartHvp) : nullptr;
  RGP_HIP(launch_hvp(ha, dr, s));
  if (vHv_dev) RGP_HIP(launch_sum_final(k.slot(kPartHvp), plan_hvp(g, dr).grid, vHv_dev, s));
  return RGP_OK;
}

rgp_status rgp_pcg_solve(const rgp_grid* grid, rgp_dtype real_t, const void* hdiag,
                         const void* hoff, double alpha, const void* rhs, void* x, int32_t maxit,
                         double rtol, int32_t* iters_dev, double* relres_dev, void* ws,
                         size_t ws_bytes, void* stream) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  DType dr;
  if (!dtype_of(real_t, &dr)) return RGP_EINVAL;
  if (dr == DType::BF16) return RGP_EDTYPE;
  if (!hdiag || !hoff || !rhs || !x || maxit < 1 || maxit > 100000 || !(rtol >= 0.0) ||
      !(alpha >= 0.0) || !std::isfinite(alpha))
    return RGP_EINVAL;
  if ((st = need_ws(RGP_OP_PCG_SOLVE, grid, real_t, nullptr, ws, ws_bytes)) != RGP_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const Geom g = geom_of(grid);
  Carver c(ws);
  Control k = carve_control(c);
  void* vec[6];
  for (int i = 0; i < 6; ++i) vec[i] = c.take(g.nnode * dsize(dr));
  const PcgPlan L = plan_pcg(g, dr);
  for (int i = 0; i <= maxit; ++i) {
    const int in = (i + 1) & 1, out = i & 1;
    PcgScalarArgs sa{};
    sa.st = k.st;
    sa.slots = k.slots;
    sa.part_prev = k.slot(kPartPcg0 + in);
    sa.nprod = L.grid;
    sa.iter = i;
    sa.maxit = maxit;
    sa.rtol = rtol;
    sa.gn_mode = 0;
    sa.fused = L.fused;
    sa.iters_out = iters_dev;
    sa.relres_out = relres_dev;
    if (!sa.fused) RGP_HIP(launch_pcg_scalars(sa, s));
    PcgArgs pa{};
    pa.g = g;
    pa.diag = hdiag;
    pa.off = hoff;
    pa.rhs = rhs;
    pa.rhs_sign = 1.0;
    pa.x = x;
    pa.r_in = vec[3 * in + 0];
    pa.p_in = vec[3 * in + 1];
    pa.w_in = vec[3 * in + 2];
    pa.r_out = vec[3 * out + 0];
    pa.p_out = vec[3 * out + 1];
    pa.w_out = vec[3 * out + 2];
    pa.alpha = alpha;
    pa.part = k.slot(kPartPcg0 + out);
    pa.sc = sa;
    RGP_HIP(launch_pcg_step(pa, dr, s));
  }
  return RGP_OK;
}

rgp_status rgp_loss_grad_images(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                                const void* I_minus, rgp_dtype real_t, const void* b,
                                void* gI_plus, void* gI_minus, void* stream) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  DType di, dr;
  if ((st = check_types(img_t, real_t, &di, &dr)) != RGP_OK) return st;
  if (!I_plus || !I_minus || !b || !gI_plus || !gI_minus) return RGP_EINVAL;
  ImageGradArgs ia{};
  ia.g = geom_of(grid);
  ia.Ip = I_plus;
  ia.Im = I_minus;
  ia.b = b;
  ia.gIp = gI_plus;
  ia.gIm = gI_minus;
  RGP_HIP(launch_image_grad(ia, di, dr, static_cast<hipStream_t>(stream)));
  return RGP_OK;
}

rgp_status rgp_correct_lsq(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                           const void* I_minus, rgp_dtype real_t, const void* b, int32_t maxit,
                           double rtol, void* I_out, int32_t* iters_dev, void* stream) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  DType di, dr;
  if ((st = check_types(img_t, real_t, &di, &dr)) != RGP_OK) return st;
  if (!I_plus || !I_minus || !b || !I_out || maxit < 1 || maxit > 100000 || !(rtol >= 0.0))
    return RGP_EINVAL;
  if (lsq_cols_per_block((int)grid->m[grid->pe], dr) < 1) return RGP_ESHAPE;
  LsqArgs la{};
  la.g = geom_of(grid);
  la.Ip = I_plus;
  la.Im = I_minus;
  la.b = b;
  la.I_out = I_out;
  la.iters = iters_dev;
  la.maxit = maxit;
  la.rtol = rtol;
  RGP_HIP(launch_lsq(la, di, dr, static_cast<hipStream_t>(stream)));
  return RGP_OK;
}

rgp_status rgp_apply_correction(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                                const void* I_minus, rgp_dtype real_t, const void* b,
                                void* T_plus, void* T_minus, void* stream) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  DType di, dr;
  if ((st = check_types(img_t, real_t, &di, &dr)) != RGP_OK) return st;
  if (!I_plus || !I_minus || !b) return RGP_EINVAL;
  if (!T_plus && !T_minus) return RGP_OK;
  CorrectArgs ca{};
  ca.g = geom_of(grid);
  ca.Ip = I_plus;
  ca.Im = I_minus;
  ca.b = b;
  ca.Tp = T_plus;
  ca.Tm = T_minus;
  RGP_HIP(launch_correct(ca, di, dr, static_cast<hipStream_t>(stream)));
  return RGP_OK;
}

}  // extern "C"

namespace {

rgp_status check_correct(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                         const void* I_minus, rgp_dtype real_t, const rgp_solver_opts* opts,
                         const void* b_init, void* b_out, void* ws, size_t ws_bytes) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  DType di, dr;
  if ((st = check_types(img_t, real_t, &di, &dr)) != RGP_OK) return st;
  if ((st = check_opts(opts)) != RGP_OK) return st;
  if (!I_plus || !I_minus || !b_out) return RGP_EINVAL;
  if (opts->use_b_init && !b_init) return RGP_EINVAL;
  // the OT initialisation runs on the coarsest level
  Level lv[kMaxLevels];
  if (make_levels(grid, opts->levels, lv) != 0) return RGP_ESHAPE;
  if (!opts->use_b_init && !ot_column_supported(lv[opts->levels - 1].g.mp)) return RGP_ESHAPE;
  if (opts->solver == RGP_SOLVER_ADMM) {
    if (block_pcg_npl((int)grid->m[grid->pe]) == 0) return RGP_ESHAPE;
    for (int d = 0; d < 3; ++d)
      if (d != grid->pe && grid->m[d] > kDhtMaxN) return RGP_ESHAPE;
  }
  return need_ws(RGP_OP_CORRECT, grid, real_t, opts, ws, ws_bytes);
}

hipError_t copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  return launch_copy(dst, src, bytes, s);
}

// Enqueues the whole correction (arguments already validated).
rgp_status enqueue_correct(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                           const void* I_minus, rgp_dtype real_t, const rgp_solver_opts* opts,
                           const void* b_init, void* b_out, void* T_plus, void* T_minus,
                           double* stats_dev, void* ws, hipStream_t s) {
  DType di, dr;
  dtype_of(img_t, &di);
  dtype_of(real_t, &dr);
  const int L = opts->levels;
  Level lv[kMaxLevels];
  if (make_levels(grid, L, lv) != 0) return RGP_ESHAPE;
  CorrectWs w = carve_correct(ws, lv, L, dr, opts);
  const size_t rs = dsize(dr);
  const Range range("rgp: correction");

  RGP_HIP(launch_reset(SetStateArgs{w.ctl.st, w.ctl.guarded}, s));
  const int64_t nrec = (int64_t)L * opts->gn_iters;
  if (stats_dev)
    RGP_HIP(launch_fill(stats_dev, RGP_STAT_HEADER + nrec * kStatFields, std::nan(""), s));

  // Image pyramid (levels >= 1 in the arithmetic type).
  const void* imgs[kMaxLevels][2];
  DType ity[kMaxLevels];
  imgs[0][0] = I_plus;
  imgs[0][1] = I_minus;
  ity[0] = di;
  for (int l = 1; l < L; ++l) {
    const Range rl("rgp: restrict to level %d", l);
    for (int i = 0; i < 2; ++i) {
      RestrictArgs ra{};
      ra.src = imgs[l - 1][i];
      ra.dst = w.img[l][i];
      for (int d = 0; d < 3; ++d) {
        ra.mf[d] = (int32_t)lv[l - 1].m[d];
        ra.mc[d] = (int32_t)lv[l].m[d];
      }
      RGP_HIP(launch_restrict(ra, ity[l - 1], dr, s));
      imgs[l][i] = w.img[l][i];
    }
    ity[l] = dr;
  }

  // Initial field on the coarsest level.
  const Level& top = lv[L - 1];
  if (opts->use_b_init) {
    const Range ri("rgp: b_init");
    RGP_HIP(copy_d2d(w.B[0], b_init, top.g.nnode * rs, s));
    // input scan for non-finite values (the OT path does it in its shift kernel)
    RGP_HIP(launch_shift(ShiftArgs{imgs[L - 1][0], imgs[L - 1][1], top.g.ncell,
                                   w.ctl.slot(kPartShift), w.ctl.guarded},
                         ity[L - 1], s));
    RGP_HIP(launch_scan_status(w.ctl.slot(kPartShift), shift_grid(top.g.ncell), w.ctl.st, s));
  } else {
    const Range ri("rgp: OT init");
    RGP_HIP(launch_shift(ShiftArgs{imgs[L - 1][0], imgs[L - 1][1], top.g.ncell,
                                   w.ctl.slot(kPartShift), w.ctl.guarded},
                         ity[L - 1], s));
    OtArgs oa{};
    oa.g = top.g;
    oa.Ip = imgs[L - 1][0];
    oa.Im = imgs[L - 1][1];
    oa.b0 = w.B[0];
    oa.st = w.ctl.st;
    oa.shift_part = w.ctl.slot(kPartShift);
    oa.shift_nprod = shift_grid(top.g.ncell);
    oa.eps = opts->ot_eps;
    oa.guard = opts->ot_guard ? 1 : 0;
    oa.guard_slope = kGuardSlope;
    oa.guarded = w.ctl.guarded;
    RGP_HIP(launch_ot(oa, ity[L - 1], dr, s));
  }

  int cur = 0;
  if (!opts->use_b_init && opts->ot_blur) {
    BlurArgs ba{};
    ba.src = w.B[0];
    ba.dst = w.B[1];
    for (int d = 0; d < 3; ++d) ba.n[d] = (uint32_t)(top.m[d] + (d == grid->pe ? 1 : 0));
    ba.cells = top.g.ncell;
    RGP_HIP(launch_blur(ba, dr, s));
    cur = 1;
  }
  for (int l = L - 1; l >= 0; --l) {
    const Range rl("rgp: level %d", l);
    if (l < L - 1) {
      ProlongArgs pa{};
      pa.src = w.B[cur];
      pa.dst = w.B[1 - cur];
      for (int d = 0; d < 3; ++d) {
        pa.mf[d] = (int32_t)lv[l].m[d];
        pa.mc[d] = (int32_t)lv[l + 1].m[d];
      }
      pa.pe = grid->pe;
      RGP_HIP(launch_prolong(pa, dr, s));
      cur = 1 - cur;
    }
    double* rec = stats_dev ? stats_dev + RGP_STAT_HEADER +
                                  (size_t)(L - 1 - l) * opts->gn_iters * kStatFields
                            : nullptr;
    hipError_t e;
    if (opts->solver == RGP_SOLVER_LBFGS)
      e = run_level_lbfgs(w, lv[l].g, imgs[l][0], imgs[l][1], ity[l], dr, opts, cur, rec, s);
    else if (opts->solver == RGP_SOLVER_ADMM)
      e = run_level_admm(w, lv[l].g, lv[l].m, grid->pe, lv[l].h, imgs[l][0], imgs[l][1],
                         ity[l], dr, opts, cur, rec, s);
    else
      e = run_level(w, lv[l].g, imgs[l][0], imgs[l][1], ity[l], dr, opts, cur, rec, s);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      return RGP_EHIP;
    }
  }

  if (T_plus || T_minus) {
    CorrectArgs ca{};
    ca.g = lv[0].g;
    ca.Ip = I_plus;
    ca.Im = I_minus;
    ca.b = w.B[cur];
    ca.Tp = T_plus;
    ca.Tm = T_minus;
    RGP_HIP(launch_correct(ca, di, dr, s));
  }
  RGP_HIP(copy_d2d(b_out, w.B[cur], lv[0].g.nnode * rs, s));
  if (stats_dev) RGP_HIP(launch_stats_header(stats_dev, w.ctl.st, w.ctl.guarded, s));
  return RGP_OK;
}

}  // namespace

struct rgp_plan_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

rgp_status rgp_correct(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                       const void* I_minus, rgp_dtype real_t, const rgp_solver_opts* opts,
                       const void* b_init, void* b_out, void* T_plus, void* T_minus,
                       double* stats_dev, void* ws, size_t ws_bytes, void* stream) {
  rgp_status st = check_correct(grid, img_t, I_plus, I_minus, real_t, opts, b_init, b_out, ws,
                                ws_bytes);
  if (st != RGP_OK) return st;
  return enqueue_correct(grid, img_t, I_plus, I_minus, real_t, opts, b_init, b_out, T_plus,
                         T_minus, stats_dev, ws, static_cast<hipStream_t>(stream));
}

rgp_status rgp_correct_plan(const rgp_grid* grid, rgp_dtype img_t, const void* I_plus,
                            const void* I_minus, rgp_dtype real_t, const rgp_solver_opts* opts,
                            const void* b_init, void* b_out, void* T_plus, void* T_minus,
                            double* stats_dev, void* ws, size_t ws_bytes, void* stream,
                            rgp_plan* plan) {
  if (!plan) return RGP_EINVAL;
  *plan = nullptr;
  if (!stream) return RGP_EINVAL;  // the legacy default stream cannot be captured
  rgp_status st = check_correct(grid, img_t, I_plus, I_minus, real_t, opts, b_init, b_out, ws,
                                ws_bytes);
  if (st != RGP_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  RGP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  st = enqueue_correct(grid, img_t, I_plus, I_minus, real_t, opts, b_init, b_out, T_plus, T_minus,
                       stats_dev, ws, s);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &graph);
  if (st != RGP_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) g_last_hip = (int)e;
    return st != RGP_OK ? st : RGP_EHIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    (void)hipGraphDestroy(graph);
    g_last_hip = (int)e2;
    return RGP_EHIP;
  }
  rgp_plan p = new (std::nothrow) rgp_plan_s{graph, exec};
  if (!p) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return RGP_EINVAL;
  }
  *plan = p;
  return RGP_OK;
}

rgp_status rgp_plan_launch(rgp_plan plan, void* stream) {
  if (!plan) return RGP_EINVAL;
  RGP_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
  return RGP_OK;
}

rgp_status rgp_plan_destroy(rgp_plan plan) {
  if (!plan) return RGP_OK;
  const hipError_t e1 = hipGraphExecDestroy(plan->exec);
  const hipError_t e2 = hipGraphDestroy(plan->graph);
  delete plan;
  if (e1 != hipSuccess || e2 != hipSuccess) {
    g_last_hip = (int)(e1 != hipSuccess ? e1 : e2);
    return RGP_EHIP;
  }
  return RGP_OK;
}

}  // extern "C"

// ---- kernel timing ----------------------------------------------------------------------

namespace {
// Events the autotuner hands to its own launches on this thread (pairs e0[i], e1[i], taken in
// order); a caller's timing session is left alone meanwhile.
struct TuneTiming {
  hipEvent_t* e0 = nullptr;
  hipEvent_t* e1 = nullptr;
  int n = 0, used = 0;
};
thread_local TuneTiming t_tune;
}  // namespace

bool rgp::timing_slot(int kind, int tag, unsigned grid, int64_t cells, int64_t nodes,
                      hipStream_t s, hipEvent_t* e0, hipEvent_t* e1) {
  if (t_tune.e0) {
    if (t_tune.used >= t_tune.n) return false;
    *e0 = t_tune.e0[t_tune.used];
    *e1 = t_tune.e1[t_tune.used];
    ++t_tune.used;
    return true;
  }
  if (!g_timing_on.load(std::memory_order_relaxed)) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  if (!g_timing_on.load(std::memory_order_relaxed) || g_timing_used >= g_timing.size())
    return false;
  TimingRec& r = g_timing[g_timing_used++];
  r.kind = kind;
  r.tag = tag;
  r.grid = grid;
  r.cells = cells;
  r.nodes = nodes;
  *e0 = r.e0;
  *e1 = r.e1;
  return true;
}

namespace {
void timing_release_locked() {
  for (TimingRec& r : g_timing) {
    if (r.e0) (void)hipEventDestroy(r.e0);
    if (r.e1) (void)hipEventDestroy(r.e1);
  }
  g_timing.clear();
  g_timing_used = 0;
}
}  // namespace

rgp_status rgp_timing_start(int32_t capacity) {
  if (capacity < 1 || capacity > (1 << 20)) return RGP_EINVAL;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_timing_on.store(false);
  timing_release_locked();
  g_timing.resize((size_t)capacity, TimingRec{0, 0, 0, 0, 0, nullptr, nullptr});
  for (TimingRec& r : g_timing) {
    hipError_t e = hipEventCreate(&r.e0);
    if (e == hipSuccess) e = hipEventCreate(&r.e1);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      timing_release_locked();
      return RGP_EHIP;
    }
  }
  g_timing_on.store(true);
  return RGP_OK;
}

rgp_status rgp_timing_stop(rgp_timing_record* out, int32_t max, int32_t* n) {
  if (!out || !n || max < 0) return RGP_EINVAL;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_timing_on.store(false);
  rgp_status st = RGP_OK;
  int32_t k = 0;
  for (size_t i = 0; i < g_timing_used && k < max; ++i) {
    const TimingRec& r = g_timing[i];
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(r.e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.e0, r.e1);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      st = RGP_EHIP;
      break;
    }
    out[k++] = rgp_timing_record{r.kind, r.tag, r.grid, 0u, r.cells, r.nodes, (double)ms};
  }
  *n = k;
  timing_release_locked();
  return st;
}

// ---- batched correction -------------------------------------------------------------------

namespace {

constexpr int kMaxBatch = 1024;
constexpr int kBatchMaxContig = 256;  // nodes along the contiguous axis (one PCG tile shape)

struct BatchPlansScope {
  bool saved;
  int saved_march;
  explicit BatchPlansScope(int march_min) : saved(batch_plans()), saved_march(batch_march_min()) {
    batch_plans() = true;
    batch_march_min() = march_min;
  }
  ~BatchPlansScope() {
    batch_plans() = saved;
    batch_march_min() = saved_march;
  }
};
struct RecorderScope {
  Recorder* saved;
  explicit RecorderScope(Recorder* r) : saved(active_recorder()) { active_recorder() = r; }
  ~RecorderScope() { active_recorder() = saved; }
};

rgp_status check_batch_grids(int32_t n, const rgp_grid* grids, rgp_dtype real_t,
                             const rgp_solver_opts* opts) {
  if (n < 1 || n > kMaxBatch || !grids) return RGP_EINVAL;
  rgp_status st = check_opts(opts);
  if (st != RGP_OK) return st;
  if (opts->use_b_init) return RGP_EINVAL;
  DType dr;
  if (!dtype_of(real_t, &dr) || dr == DType::BF16) return RGP_EDTYPE;
  for (int p = 0; p < n; ++p) {
    if ((st = check_grid(&grids[p])) != RGP_OK) return st;
    if (grids[p].m[2] + (grids[p].pe == 2 ? 1 : 0) > kBatchMaxContig) return RGP_ESHAPE;
    Level lv[kMaxLevels];
    if (make_levels(&grids[p], opts->levels, lv) != 0) return RGP_ESHAPE;
    if (!ot_column_supported(lv[opts->levels - 1].g.mp)) return RGP_ESHAPE;
  }
  return RGP_OK;
}

size_t pair_bytes(const rgp_grid* g, const rgp_solver_opts* o, DType dr) {
  Level lv[kMaxLevels];
  make_levels(g, o->levels, lv);
  return align_up(correct_bytes(lv, o->levels, dr, o));
}

// One shared launch of the merged sequence: where its tables sit in the arena.
struct BatchSlot {
  bool shared = false;
  RecKind kind = RecKind::kOther;
  size_t tab = 0, geo = 0, starts = 0;
  unsigned grid = 0;
  size_t lds = 0;
  int var[4] = {0, 0, 0, 0};
  int64_t cells = 0, nodes = 0;  // summed over the pairs (kernel timing)
  int tag = 0;
};

// Records the correction of every pair (their workspaces laid out back to back from ws) and
// merges the sequences: returns the per-pair launches and the table arena.
rgp_status record_batch(int32_t n, const rgp_grid* grids, rgp_dtype img_t,
                        const void* const* I_plus, const void* const* I_minus, rgp_dtype real_t,
                        const rgp_solver_opts* opts, void* const* b_out, void* const* T_plus,
                        void* const* T_minus, double* const* stats, unsigned char* ws,
                        std::vector<Recorder>& recs, std::vector<BatchSlot>& slots,
                        std::vector<unsigned char>& arena, size_t& pairs_total) {
  DType dr;
  dtype_of(real_t, &dr);
  recs.assign((size_t)n, Recorder{});
  size_t off = 0;
  {
    BatchPlansScope bp(opts->batch_march);
    for (int p = 0; p < n; ++p) {
      RecorderScope rs(&recs[(size_t)p]);
      rgp_status st = enqueue_correct(&grids[p], img_t, I_plus[p], I_minus[p], real_t, opts,
                                      nullptr, b_out[p], T_plus ? T_plus[p] : nullptr,
                                      T_minus ? T_minus[p] : nullptr, stats ? stats[p] : nullptr,
                                      ws + off, nullptr);
      if (st != RGP_OK) return st;
      off += pair_bytes(&grids[p], opts, dr);
    }
  }
  pairs_total = off;
  const size_t L = recs[0].launches.size();
  for (int p = 1; p < n; ++p)
    if (recs[(size_t)p].launches.size() != L) return RGP_EINVAL;
  slots.assign(L, BatchSlot{});
  arena.clear();
  auto put = [&](const void* src, size_t bytes) {
    const size_t at = align_up(arena.size());
    arena.resize(at + bytes);
    std::memcpy(arena.data() + at, src, bytes);
    return at;
  };
  for (size_t i = 0; i < L; ++i) {
    const RecLaunch& r0 = recs[0].launches[i];
    BatchSlot& sl = slots[i];
    sl.kind = r0.kind;
    bool same = true;
    for (int p = 1; p < n && same; ++p) {
      const RecLaunch& r = recs[(size_t)p].launches[i];
      same = r.kind == r0.kind && r.block == r0.block && r.args.size() == r0.args.size() &&
             std::equal(r.var, r.var + 4, r0.var);
    }
    if (!same) {
      // the sequences must have the same shape; differing kinds mean they do not
      for (int p = 1; p < n; ++p)
        if (recs[(size_t)p].launches[i].kind != r0.kind) return RGP_EINVAL;
    }
    if (r0.kind == RecKind::kOther || n == 1 || !same) continue;
    sl.shared = true;
    std::copy(r0.var, r0.var + 4, sl.var);
    std::vector<unsigned char> tab;
    std::vector<uint32_t> starts((size_t)n + 1, 0);
    std::vector<MarchGeo> geo;
    for (int p = 0; p < n; ++p) {
      const RecLaunch& r = recs[(size_t)p].launches[i];
      tab.insert(tab.end(), r.args.begin(), r.args.end());
      starts[(size_t)p + 1] = starts[(size_t)p] + r.grid;
      sl.cells += r.cells;
      sl.nodes += r.nodes;
      sl.tag = r.tag;
      sl.lds = std::max(sl.lds, r.lds);
      geo.push_back(r.geo);
      if (r0.kind == RecKind::kPcgStep) sl.var[3] = std::max(sl.var[3], r.geo.XL);
    }
    sl.grid = starts[(size_t)n];
    sl.tab = put(tab.data(), tab.size());
    sl.starts = put(starts.data(), starts.size() * sizeof(uint32_t));
    if (r0.kind == RecKind::kPcgStep) sl.geo = put(geo.data(), geo.size() * sizeof(MarchGeo));
  }
  arena.resize(align_up(arena.size()));
  return RGP_OK;
}

hipError_t issue_batch(int32_t n, const std::vector<Recorder>& recs,
                       const std::vector<BatchSlot>& slots, const unsigned char* arena_dev,
                       hipStream_t s) {
  for (size_t i = 0; i < slots.size(); ++i) {
    const BatchSlot& sl = slots[i];
    hipError_t e = hipSuccess;
    if (!sl.shared) {
      for (int p = 0; p < n && e == hipSuccess; ++p) e = recs[(size_t)p].launches[i].replay(s);
      if (e != hipSuccess) return e;
      continue;
    }
    const void* tab = arena_dev + sl.tab;
    const uint32_t* starts = reinterpret_cast<const uint32_t*>(arena_dev + sl.starts);
    switch (sl.kind) {
      case RecKind::kLossGrad:
        e = launch_loss_grad_batch(tab, starts, n, sl.grid, (DType)sl.var[0], (DType)sl.var[1],
                                   sl.cells, sl.nodes, sl.tag, s);
        break;
      case RecKind::kTrial:
        e = launch_trial_batch(tab, starts, n, sl.grid, sl.var[2], (DType)sl.var[0],
                               (DType)sl.var[1], sl.cells, sl.nodes, s);
        break;
      case RecKind::kDecide:
        e = launch_decide_batch(tab, n, sl.var[0], s);
        break;
      case RecKind::kApply:
        e = launch_apply_step_batch(tab, starts, n, sl.grid, (DType)sl.var[0], s);
        break;
      case RecKind::kPcgScalars:
        e = launch_pcg_scalars_batch(tab, n, s);
        break;
      case RecKind::kPcgStep:
        e = launch_pcg_step_batch(tab, reinterpret_cast<const MarchGeo*>(arena_dev + sl.geo),
                                  starts, n, sl.grid, sl.lds, (DType)sl.var[0], sl.var[3],
                                  sl.cells, sl.nodes, sl.tag, s);
        break;
      default:
        e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

rgp_status rgp_batch_workspace_size(int32_t n, const rgp_grid* grids, rgp_dtype real_t,
                                    const rgp_solver_opts* opts, size_t* bytes) {
  if (!bytes) return RGP_EINVAL;
  rgp_status st = check_batch_grids(n, grids, real_t, opts);
  if (st != RGP_OK) return st;
  // a dry recording with placeholder addresses gives the size of the launch tables
  std::vector<const void*> img((size_t)n, reinterpret_cast<const void*>(kAlign));
  std::vector<void*> out((size_t)n, reinterpret_cast<void*>(kAlign));
  std::vector<Recorder> recs;
  std::vector<BatchSlot> slots;
  std::vector<unsigned char> arena;
  size_t pairs = 0;
  st = record_batch(n, grids, RGP_F32, img.data(), img.data(), real_t, opts, out.data(), nullptr,
                    nullptr, nullptr, nullptr, recs, slots, arena, pairs);
  if (st != RGP_OK) return st;
  *bytes = pairs + arena.size();
  return RGP_OK;
}

namespace {

// Checks the arguments of a batched correction, records every pair's sequence and uploads the
// shared launches' tables to the workspace (synchronising `s` once: the host tables die here).
rgp_status prepare_batch(int32_t n, const rgp_grid* grids, rgp_dtype img_t,
                         const void* const* I_plus, const void* const* I_minus, rgp_dtype real_t,
                         const rgp_solver_opts* opts, void* const* b_out, void* const* T_plus,
                         void* const* T_minus, double* const* stats_dev, void* ws, size_t ws_bytes,
                         hipStream_t s, std::vector<Recorder>& recs,
                         std::vector<BatchSlot>& slots, unsigned char** arena_dev) {
  rgp_status st = check_batch_grids(n, grids, real_t, opts);
  if (st != RGP_OK) return st;
  DType di, dr;
  if ((st = check_types(img_t, real_t, &di, &dr)) != RGP_OK) return st;
  if (!I_plus || !I_minus || !b_out) return RGP_EINVAL;
  for (int p = 0; p < n; ++p) {
    if (!I_plus[p] || !I_minus[p] || !b_out[p]) return RGP_EINVAL;
    if ((T_plus && !T_plus[p]) || (T_minus && !T_minus[p]) || (stats_dev && !stats_dev[p]))
      return RGP_EINVAL;
  }
  size_t need = 0;
  if ((st = rgp_batch_workspace_size(n, grids, real_t, opts, &need)) != RGP_OK) return st;
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
    return RGP_EWORKSPACE;
  std::vector<unsigned char> arena;
  size_t pairs = 0;
  st = record_batch(n, grids, img_t, I_plus, I_minus, real_t, opts, b_out, T_plus, T_minus,
                    stats_dev, static_cast<unsigned char*>(ws), recs, slots, arena, pairs);
  if (st != RGP_OK) return st;
  *arena_dev = static_cast<unsigned char*>(ws) + pairs;
  if (!arena.empty()) {
    RGP_HIP(hipMemcpyAsync(*arena_dev, arena.data(), arena.size(), hipMemcpyHostToDevice, s));
    RGP_HIP(hipStreamSynchronize(s));
  }
  return RGP_OK;
}

}  // namespace

rgp_status rgp_correct_batch(int32_t n, const rgp_grid* grids, rgp_dtype img_t,
                             const void* const* I_plus, const void* const* I_minus,
                             rgp_dtype real_t, const rgp_solver_opts* opts, void* const* b_out,
                             void* const* T_plus, void* const* T_minus, double* const* stats_dev,
                             void* ws, size_t ws_bytes, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  RGP_HIP(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return RGP_EINVAL;  // it synchronises the stream
  std::vector<Recorder> recs;
  std::vector<BatchSlot> slots;
  unsigned char* arena_dev = nullptr;
  rgp_status st = prepare_batch(n, grids, img_t, I_plus, I_minus, real_t, opts, b_out, T_plus,
                                T_minus, stats_dev, ws, ws_bytes, s, recs, slots, &arena_dev);
  if (st != RGP_OK) return st;
  RGP_HIP(issue_batch(n, recs, slots, arena_dev, s));
  return RGP_OK;
}

rgp_status rgp_correct_batch_plan(int32_t n, const rgp_grid* grids, rgp_dtype img_t,
                                  const void* const* I_plus, const void* const* I_minus,
                                  rgp_dtype real_t, const rgp_solver_opts* opts,
                                  void* const* b_out, void* const* T_plus, void* const* T_minus,
                                  double* const* stats_dev, void* ws, size_t ws_bytes,
                                  void* stream, rgp_plan* plan) {
  if (!plan) return RGP_EINVAL;
  *plan = nullptr;
  if (!stream) return RGP_EINVAL;  // the legacy default stream cannot be captured
  const hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<Recorder> recs;
  std::vector<BatchSlot> slots;
  unsigned char* arena_dev = nullptr;
  rgp_status st = prepare_batch(n, grids, img_t, I_plus, I_minus, real_t, opts, b_out, T_plus,
                                T_minus, stats_dev, ws, ws_bytes, s, recs, slots, &arena_dev);
  if (st != RGP_OK) return st;
  RGP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const hipError_t e = issue_batch(n, recs, slots, arena_dev, s);
  hipGraph_t graph = nullptr;
  const hipError_t e1 = hipStreamEndCapture(s, &graph);
  if (e != hipSuccess || e1 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    g_last_hip = (int)(e != hipSuccess ? e : e1);
    return RGP_EHIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    (void)hipGraphDestroy(graph);
    g_last_hip = (int)e2;
    return RGP_EHIP;
  }
  rgp_plan pl = new (std::nothrow) rgp_plan_s{graph, exec};
  if (!pl) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return RGP_EINVAL;
  }
  *plan = pl;
  return RGP_OK;
}

// ---- autotuner of the PCG march ----------------------------------------------------------

rgp_status rgp_autotune(const rgp_grid* grid, rgp_dtype real_t, const rgp_solver_opts* opts,
                        void* ws, size_t ws_bytes, void* stream, int32_t* xl_out) {
  rgp_status st = check_grid(grid);
  if (st != RGP_OK) return st;
  DType dr;
  if (!dtype_of(real_t, &dr) || dr == DType::BF16) return RGP_EDTYPE;
  rgp_solver_opts o;
  rgp_default_opts(&o);
  if (opts) o = *opts;
  if (!opts) o.levels = 1;
  if ((st = check_opts(&o)) != RGP_OK) return st;
  if ((st = need_ws(RGP_OP_CORRECT, grid, real_t, &o, ws, ws_bytes)) != RGP_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  RGP_HIP(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return RGP_EINVAL;  // timing needs eager launches
  Level lv[kMaxLevels];
  if (make_levels(grid, o.levels, lv) != 0) return RGP_ESHAPE;
  const CorrectWs w = carve_correct(ws, lv, o.levels, dr, &o);
  // Each candidate runs 2 untimed and kReps timed launches per round; a timed launch carries its
  // own pair of events, recorded by the launch at the kernel's start and end (kernel time only,
  // whatever the host's launch rate).
  constexpr int kReps = 9, kRounds = 3;
  hipEvent_t te0[kReps], te1[kReps];
  int nev = 0;
  hipError_t e = hipSuccess;
  for (; nev < kReps && e == hipSuccess; ++nev) {
    e = hipEventCreate(&te0[nev]);
    if (e == hipSuccess) {
      e = hipEventCreate(&te1[nev]);
      if (e != hipSuccess) (void)hipEventDestroy(te0[nev]);
    }
    if (e != hipSuccess) break;
  }
  for (int l = 0; l < o.levels && e == hipSuccess; ++l) {
    const Geom& g = lv[l].g;
    // a running PCG state: both slots and the previous block sums set to ones
    e = launch_fill(reinterpret_cast<double*>(w.ctl.slots), 2 * sizeof(PcgSlot) / sizeof(double),
                    1.0, s);
    if (e == hipSuccess)
      e = launch_fill(w.ctl.slot(kPartPcg0), 2 * (int64_t)kMaxGrid * kPartStride, 1.0, s);
    const PcgPlan H = plan_pcg_xl(g, dr, -1);  // the untuned choice
    set_tuned_march(g, dr, 0);
    const int64_t cap = 4096 / ((int64_t)H.block / kWave);
    // candidates, timed in kRounds interleaved rounds (so that a slow spell of the device does
    // not fall on one candidate only); a candidate's figure is the median of all its launches
    int cand[sizeof(kMarchLengths) / sizeof(int)];
    int nc = 0;
    for (int xl : kMarchLengths) {
      const PcgPlan L = plan_pcg_xl(g, dr, xl);
      if (xl > L.m.no || L.m.units > 4 * cap || (L.m.units < cap / 16 && xl != H.m.XL)) continue;
      cand[nc++] = xl;
    }
    std::vector<float> samples((size_t)nc * kRounds * kReps);
    for (int round = 0; round < kRounds && e == hipSuccess; ++round) {
      for (int ci = 0; ci < nc && e == hipSuccess; ++ci) {
        const int xl = cand[ci];
        const PcgPlan L = plan_pcg_xl(g, dr, xl);
        PcgArgs pa{};
        pa.g = g;
        pa.diag = w.Dg;
        pa.off = w.Of;
        pa.rhs = w.G;
        pa.rhs_sign = -1.0;
        pa.x = w.X;
        pa.r_in = w.R[1];
        pa.p_in = w.P[1];
        pa.w_in = w.W[1];
        pa.r_out = w.R[0];
        pa.p_out = w.P[0];
        pa.w_out = w.W[0];
        pa.alpha = o.alpha;
        pa.part = w.ctl.slot(kPartPcg0);
        pa.sc.st = w.ctl.st;
        pa.sc.slots = w.ctl.slots;
        pa.sc.part_prev = w.ctl.slot(kPartPcg1);
        pa.sc.nprod = L.grid;
        pa.sc.iter = 2;              // reads slot 1 and the sums above, writes slot 0
        pa.sc.maxit = 1 << 30;
        pa.sc.rtol = 0.0;
        pa.sc.fused = 1;
        for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch_pcg_step_plan(pa, dr, L, s);
        t_tune = TuneTiming{te0, te1, kReps, 0};
        for (int r = 0; r < kReps && e == hipSuccess; ++r) e = launch_pcg_step_plan(pa, dr, L, s);
        const int timed = t_tune.used;
        t_tune = TuneTiming{};
        if (e == hipSuccess && timed != kReps) e = hipErrorUnknown;
        for (int r = 0; r < kReps && e == hipSuccess; ++r) {
          e = hipEventSynchronize(te1[r]);
          if (e == hipSuccess)
            e = hipEventElapsedTime(&samples[((size_t)ci * kRounds + round) * kReps + r], te0[r],
                                    te1[r]);
        }
      }
    }
    int best_xl = H.m.XL;
    float best_ms = 1e30f;
    for (int ci = 0; ci < nc && e == hipSuccess; ++ci) {
      float* t = samples.data() + (size_t)ci * kRounds * kReps;
      std::sort(t, t + kRounds * kReps);
      const float ms = t[kRounds * kReps / 2];
      if (ms < best_ms) {
        best_ms = ms;
        best_xl = cand[ci];
      }
    }
    if (e == hipSuccess) {
      set_tuned_march(g, dr, best_xl);
      if (xl_out) xl_out[l] = best_xl;
    }
  }
  for (int i = 0; i < nev; ++i) {
    (void)hipEventDestroy(te0[i]);
    (void)hipEventDestroy(te1[i]);
  }
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return RGP_EHIP;
  }
  return RGP_OK;
}
