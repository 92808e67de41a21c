// Kernel argument blocks and host launchers of librgp (internal; not part of the C-ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rgp_internal.hpp"

namespace rgp {

enum class DType : int { F64 = 0, F32 = 1, BF16 = 2 };

template <typename TI>
__device__ __forceinline__ TI from_real(float v);
template <typename TI>
__device__ __forceinline__ TI from_real(double v);

template <>
__device__ __forceinline__ float from_real<float>(float v) { return v; }
template <>
__device__ __forceinline__ float from_real<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ double from_real<double>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double from_real<double>(double v) { return v; }
// round to nearest even (NaN stays NaN)
__device__ __forceinline__ bf16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  bf16_t r;
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
    r.bits = (uint16_t)((u >> 16) | 0x40u);
    return r;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  r.bits = (uint16_t)(u >> 16);
  return r;
}
template <>
__device__ __forceinline__ bf16_t from_real<bf16_t>(float v) { return f32_to_bf16(v); }
template <>
__device__ __forceinline__ bf16_t from_real<bf16_t>(double v) { return f32_to_bf16((float)v); }

// Launch shape of a tiled kernel: grid of `grid` blocks of `block` threads over `ntiles` tiles of
// 64 columns x S nodes.
struct Launch {
  unsigned grid, block;
  int S;
  int64_t ntiles;
};

struct LossGradArgs {
  Geom g;
  const void* Ip;
  const void* Im;
  const void* b_in;
  const void* q;      // step direction (used when step != 0)
  void* b_out;        // receives b_in + gamma q (step != 0)
  void* grad;         // nullable
  void* diag;         // nullable (then off is ignored)
  void* off;
  double alpha, beta;
  State* st;
  double* part;       // block sums: sum r^2, sum S terms, sum phi, violations, sum g^2
  int step;           // apply the accepted line-search step first
  int level_start;    // first GN step of a level: block 0 clears gn_stop / accepted
  int run;            // PE nodes per thread of the launch (set by the launcher)
  // ADMM's b-update (F_rho of Sec. 2.3.2): smoothness along the PE axis only, and the proximal
  // term (rho vol / 2)|b - prox_c|^2 with rho = st->admm_rho; its value joins the S sum as
  // (rho / alpha) (b - c)^2, so that J = D + alpha S + beta P stays the recorded form
  const void* prox_c;  // nullable: the plain objective of Eq. (6)
};

// Reduction of loss_grad's block sums into J, D, S, P (one block, or every PCG block of
// iteration 0 when gn_mode).
struct LossFinalArgs {
  const double* part;
  unsigned nprod;
  double vol, alpha, beta;
  State* st;
  double* jdsp;       // nullable
  double* record;     // nullable (written when the barrier is violated in gn_mode)
  int gn_mode;
};

struct ImageGradArgs {
  Geom g;
  const void* Ip;
  const void* Im;
  const void* b;
  void* gIp;          // dJ/dI+ (cells, field type)
  void* gIm;          // dJ/dI- (cells, field type)
};

// Largest number of candidate steps evaluated in one trial pass.
constexpr int kMaxTrialCand = 9;

struct TrialArgs {
  Geom g;
  const void* Ip;
  const void* Im;
  const void* b;
  const void* q;
  const void* grad;
  double alpha, beta, armijo_c;
  State* st;
  double* part;             // block sums: [gq, sbq, sqq, then (sum r^2, sum phi, violations) per candidate]
  int first, nc;            // gamma_c = 2^-(first + c), c < nc
  const void* prox_c;       // nullable: ADMM's b-update (as in LossGradArgs)
};

struct DecideArgs {
  const double* part_prev;
  unsigned nprod_prev;
  int prev_first, prev_nc, total;
  double vol, alpha, beta, armijo_c;
  State* st;
  double* record;
};

struct ApplyArgs {
  void* b;
  const void* q;
  const State* st;
  int64_t n;
};

struct CorrectArgs {
  Geom g;
  const void* Ip;
  const void* Im;
  const void* b;
  void* Tp;   // nullable
  void* Tm;   // nullable
};

struct HvpArgs {
  Geom g;
  const void* diag;
  const void* off;
  const void* v;
  void* Hv;
  double alpha;
  double* part;   // nullable: block sums of v.Hv
};

// Scalar phase of a PCG iteration: reduces the block sums of iteration iter-1 (iteration 0: of
// loss_grad, finalising the objective in Gauss-Newton mode) and derives the coefficients and
// status of iteration iter (slots[iter & 1]).  It runs either in the single-block
// k_pcg_scalars or (fused) at the start of every block of k_pcg_step, block 0 writing the slot.
struct PcgScalarArgs {
  State* st;
  PcgSlot* slots;           // [2]
  const double* part_prev;  // block sums of iteration iter-1
  unsigned nprod;           // grid of the main PCG kernels
  int iter, maxit;
  double rtol;
  int gn_mode;
  int fused;                // 1 = k_pcg_step derives the slot, 0 = k_pcg_scalars does
  int32_t* iters_out;       // nullable
  double* relres_out;       // nullable
  LossFinalArgs lf;         // gn_mode, iteration 0: J, D, S, P of the current iterate
};

struct PcgArgs {
  Geom g;
  const void* diag;
  const void* off;
  const void* rhs;
  double rhs_sign;
  void* x;
  const void* r_in;
  const void* p_in;
  const void* w_in;
  void* r_out;
  void* p_out;
  void* w_out;
  double alpha;             // smoothness weight (cross-axis couplings)
  double* part;             // block sums of this iteration
  PcgScalarArgs sc;         // iteration index, slots and the previous block sums
};

// Launch shape of the PCG step: `block` threads, npt plane positions per thread, hmax halo slots
// per thread, units of XL planes (m), `lds` bytes of dynamic LDS.
struct PcgPlan {
  unsigned grid, block;
  int npt, hmax;
  MarchGeo m;
  size_t lds;
  int fused;               // scalar phase inside k_pcg_step (else one k_pcg_scalars per iteration)
};

struct ShiftArgs {
  const void* Ip;
  const void* Im;
  int64_t n;
  double* part;                  // block min, max|.| and non-finite flag (0 or 1)
  unsigned long long* guarded;   // zeroed by block 0 (the OT kernel counts into it)
};

struct OtArgs {
  Geom g;
  const void* Ip;
  const void* Im;
  void* b0;
  State* st;                     // block 0 stores the shift
  const double* shift_part;
  unsigned shift_nprod;
  double eps;
  int guard;
  double guard_slope;
  unsigned long long* guarded;   // nullable counter (zeroed by the shift kernel)
};

struct RestrictArgs {
  const void* src;
  void* dst;
  int32_t mf[3], mc[3];
};

struct RestrictAdjArgs {
  const void* src;    // coarse cell array
  void* dst;          // fine cell array
  int32_t mf[3], mc[3];
  int32_t accumulate;  // add to dst instead of overwriting it
};

struct ProlongArgs {
  const void* src;   // coarse field
  void* dst;         // fine field
  int32_t mf[3], mc[3];
  int32_t pe;
};

struct SetStateArgs {
  State* st;
  unsigned long long* guarded;
};

Launch plan_tiles(const Geom& g, int S, int block);
Launch plan_loss_grad(const Geom& g, DType real);
Launch plan_trial(const Geom& g, DType real, int nc);
PcgPlan plan_pcg(const Geom& g, DType real);
// Candidate march lengths (planes per work unit) of the PCG step.
constexpr int kMarchLengths[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
constexpr int kMarchMax = 64;  // longest march a caller may ask for
PcgPlan plan_pcg_xl(const Geom& g, DType real, int xl);  // xl <= 0: tuned or heuristic
void set_tuned_march(const Geom& g, DType real, int xl);  // xl <= 0 forgets the entry
int tuned_march(const Geom& g, DType real);               // 0 when not tuned
Launch plan_hvp(const Geom& g, DType real);
unsigned shift_grid(int64_t n);

// Kernel timing (instrumentation behind rgp_timing_start/stop): when it is enabled and the stream
// is not being captured, timing_slot hands out a pair of HIP events that hipExtLaunchKernelGGL
// records at the start and the end of the kernel itself, and notes the launch (tag: the PCG
// iteration of a PCG step, the candidate count of a trial pass, the pass mode plus 4 times the
// line length of a Hartley pass, the iteration limit of a block PCG, the phase of an L-BFGS
// launch, else 0).
enum KernelKind : int {
  kKindPcgStep = 0,
  kKindLossGrad = 1,
  kKindTrial = 2,
  kKindHvp = 3,
  kKindOt = 4,
  kKindShift = 5,
  kKindBlur = 6,
  kKindDht = 7,
  kKindBlockPcg = 8,
  kKindLbfgs = 9,
  kKindLsq = 10,
  kKindCount = 11
};
bool timing_slot(int kind, int tag, unsigned grid, int64_t cells, int64_t nodes, hipStream_t s,
                 hipEvent_t* e0, hipEvent_t* e1);

#define RGP_LAUNCH_TN(KIND, TAG, CELLS, NODES, KERNEL, GRID, BLOCK, LDS, S, ...)             \
  do {                                                                                       \
    hipEvent_t rgp_e0_, rgp_e1_;                                                              \
    if (::rgp::timing_slot((KIND), (TAG), (GRID), (CELLS), (NODES), (S), &rgp_e0_, &rgp_e1_)) \
      hipExtLaunchKernelGGL(KERNEL, dim3(GRID), dim3(BLOCK), (LDS), (S), rgp_e0_, rgp_e1_, 0, \
                            __VA_ARGS__);                                                     \
    else                                                                                      \
      hipLaunchKernelGGL(KERNEL, dim3(GRID), dim3(BLOCK), (LDS), (S), __VA_ARGS__);           \
  } while (0)
#define RGP_LAUNCH_N(KIND, CELLS, NODES, KERNEL, GRID, BLOCK, LDS, S, ...) \
  RGP_LAUNCH_TN(KIND, 0, CELLS, NODES, KERNEL, GRID, BLOCK, LDS, S, __VA_ARGS__)
#define RGP_LAUNCH_T(KIND, TAG, G, KERNEL, GRID, BLOCK, LDS, S, ...) \
  RGP_LAUNCH_TN(KIND, TAG, (G).ncell, (G).nnode, KERNEL, GRID, BLOCK, LDS, S, __VA_ARGS__)
#define RGP_LAUNCH(KIND, G, KERNEL, GRID, BLOCK, LDS, S, ...) \
  RGP_LAUNCH_TN(KIND, 0, (G).ncell, (G).nnode, KERNEL, GRID, BLOCK, LDS, S, __VA_ARGS__)

// L-BFGS direction (lbfgs.hip): pair memory at most kLbfgsMaxMem; a pair is kept when
// s^T y > kLbfgsCurvature |s| |y|.
constexpr int kLbfgsMaxMem = 32;
constexpr double kLbfgsCurvature = 1e-10;
struct LbfgsMeta {
  double rho[kLbfgsMaxMem + 1];                    // 1 / s^T y per ring slot
  double sy[kLbfgsMaxMem + 1][kLbfgsMaxMem + 1];   // s_i^T y_j per ring slots (kept pairs valid)
  double yy[kLbfgsMaxMem + 1][kLbfgsMaxMem + 1];   // y_i^T y_j
  double cs[kLbfgsMaxMem + 1], cy[kLbfgsMaxMem + 1];  // d = cg g + sum over kept slots of
  double cg;                                       //   cs s + cy y
  double h0;                                       // s^T y / y^T y of the newest pair kept
  int32_t head;                                    // the free ring slot (the next pair goes there)
  int32_t count;                                   // pairs kept
};
// kLbDots: the new pair (s = gamma x, y = g - g_old into the free slot) and the block sums of its
// inner products with every pair of the window and of g with them; kLbScalar (one block): the
// sums, the admission of the pair, the two-loop recursion on those inner products, the direction's
// coefficients; kLbCombine: d = cg g + sum (cs s + cy y).
enum LbfgsPhase : int32_t { kLbDots = 0, kLbScalar = 1, kLbCombine = 2 };
struct LbfgsArgs {
  int64_t n;                  // field nodes
  const void* g;              // gradient at the current iterate
  const void* g_old;          // gradient at the previous iterate (kLbDots with a pair)
  void* x;                    // previous direction (kLbDots); d (kLbCombine)
  void* S;                    // ring of mem + 1 slots of n values each
  void* Y;
  LbfgsMeta* meta_prev;       // metadata of the previous step of the level
  LbfgsMeta* meta;            // metadata of this step
  double* part;               // kLbDots' column-major block sums (sum k of block b at
                              // part[k * kMaxGrid + b]), 3 + 5 (mem + 1) sums
  double* part_max;           // kLbDots' block maxima of |g|
  unsigned nprod;             // kLbDots' blocks (kLbScalar reads that many)
  State* st;
  int32_t mem;                // pairs kept at most
  int32_t phase;
  int32_t pair;               // this step forms a pair (every step but the first of a level)
  unsigned nblk;              // set by the launcher
};
unsigned lbfgs_grid(int64_t n);
unsigned lbfgs_dots_grid(int64_t n);
constexpr int kLbfgsSums(int mem) { return 3 + 5 * (mem + 1); }

// ADMM (admm.hip).
constexpr double kAdmmMu = 10.0, kAdmmTau = 2.0;  // rho adaptation: ratio and factor
constexpr int kDhtMaxN = 1024;                   // longest cross axis of the z-update
struct BlockPcgArgs {      // per-column Jacobi PCG on the tridiagonal blocks (diag, off)
  Geom g;
  const void* diag;
  const void* off;
  const void* grad;        // right-hand side -grad
  void* x;                 // solution (nodes of every column written)
  int32_t maxit;
  double rtol;
  State* st;               // gn_stop; receives the largest iteration count and residual
  double* part;            // per-block maxima (column-major, 2 sums)
  unsigned nblk;           // set by the launcher
};
enum DhtMode : int32_t { kDhtFirst = 0, kDhtScale = 1, kDhtPlain = 2, kDhtLast = 3 };
struct DhtArgs {           // one pass of the z-update (normalised Hartley transform along axis)
  int32_t n[3];            // node extents of the field array
  int32_t axis;            // transform axis (a cross axis)
  int32_t other_axis;      // the other cross axis (kDhtScale)
  int32_t mode;
  const void* src;         // input of kDhtScale / kDhtPlain / kDhtLast
  void* dst;               // output (kDhtLast: z, read first as z_old)
  const void* b;           // kDhtFirst, kDhtLast
  void* u;                 // kDhtFirst (read), kDhtLast (updated)
  void* c;                 // kDhtLast: c = z - u
  double alpha;
  double inv_h2[2];        // 1 / h^2 of axis and other_axis (kDhtScale)
  State* st;               // rho, gn_stop
  double* part;            // kDhtLast: block sums of (b - z)^2 and (z - z_old)^2
  int32_t lines_per_block; // set by the launcher
  unsigned nblk;           // set by the launcher
  FastDiv by_n, by_nu1, by_lpb, by_ngr;  // set by the launcher: divisions by n[axis], by the
                                         // faster other extent, by lines_per_block, by its pairs
};
struct AdmmRhoArgs {
  State* st;
  const double* part;
  unsigned nprod;
  double* record;          // nullable: field 11 receives the rho the iteration used
};
struct AdmmVecArgs {
  int64_t n;
  const void* b;
  void* z;
  void* u;
  void* c;
  double rho0;             // init only
  State* st;
};
int block_pcg_npl(int mp);       // nodes per lane (0: the column is too long)
unsigned block_pcg_grid(int64_t ncol);
hipError_t launch_block_pcg(const BlockPcgArgs& a, DType real, hipStream_t s);
unsigned dht_grid(const int32_t n[3], int axis, int* lines_per_block);
hipError_t launch_dht(const DhtArgs& a, DType real, hipStream_t s);
hipError_t launch_admm_rho(const AdmmRhoArgs& a, hipStream_t s);
hipError_t launch_admm_vec(const AdmmVecArgs& a, bool init, DType real, hipStream_t s);

// Least-squares correction (lsq.hip).
struct LsqArgs {
  Geom g;
  const void* Ip;
  const void* Im;
  const void* b;
  void* I_out;
  int32_t* iters;        // per column (nullable)
  int32_t maxit;
  double rtol;
  int32_t cols_per_block;  // set by the launcher
};
int lsq_cols_per_block(int mp, DType real);
hipError_t launch_lsq(const LsqArgs& a, DType img, DType real, hipStream_t s);
hipError_t launch_lbfgs(const LbfgsArgs& a, DType real, hipStream_t s);

// Runs __VA_ARGS__ with TI (image storage type) and TR (arithmetic type) bound to the supported
// combinations; returns hipErrorInvalidValue from the caller otherwise.
#define RGP_DISPATCH_TYPES(IMG, REAL, ...)                                              \
  do {                                                                                  \
    if ((REAL) == DType::F64 && (IMG) == DType::F64) {                                  \
      using TI = double; using TR = double; __VA_ARGS__;                                \
    } else if ((REAL) == DType::F32 && (IMG) == DType::F32) {                           \
      using TI = float; using TR = float; __VA_ARGS__;                                  \
    } else if ((REAL) == DType::F32 && (IMG) == DType::BF16) {                          \
      using TI = bf16_t; using TR = float; __VA_ARGS__;                                 \
    } else if ((REAL) == DType::F64 && (IMG) == DType::F32) {                           \
      using TI = float; using TR = double; __VA_ARGS__;                                 \
    } else if ((REAL) == DType::F64 && (IMG) == DType::BF16) {                          \
      using TI = bf16_t; using TR = double; __VA_ARGS__;                                \
    } else {                                                                            \
      return hipErrorInvalidValue;                                                      \
    }                                                                                   \
  } while (0)

hipError_t launch_loss_grad(const LossGradArgs& a, DType img, DType real, hipStream_t s);
hipError_t launch_loss_final(const LossFinalArgs& a, hipStream_t s);
hipError_t launch_trial(const TrialArgs& a, DType img, DType real, hipStream_t s);
hipError_t launch_decide(const DecideArgs& a, hipStream_t s);
hipError_t launch_apply_step(const ApplyArgs& a, DType real, hipStream_t s);
hipError_t launch_correct(const CorrectArgs& a, DType img, DType real, hipStream_t s);
hipError_t launch_image_grad(const ImageGradArgs& a, DType img, DType real, hipStream_t s);
hipError_t launch_hvp(const HvpArgs& a, DType real, hipStream_t s);
hipError_t launch_sum_final(const double* part, unsigned nprod, double* out, hipStream_t s);
hipError_t launch_pcg_step(const PcgArgs& a, DType real, hipStream_t s);
hipError_t launch_pcg_step_plan(const PcgArgs& a, DType real, const PcgPlan& L, hipStream_t s);
hipError_t launch_pcg_scalars(const PcgScalarArgs& a, hipStream_t s);
hipError_t launch_shift(const ShiftArgs& a, DType img, hipStream_t s);
// Sets st->status to RGP_ENONFINITE when the input scan (the shift kernel's block sums) found a
// non-finite image value.
hipError_t launch_scan_status(const double* part, unsigned nprod, State* st, hipStream_t s);
hipError_t launch_ot(const OtArgs& a, DType img, DType real, hipStream_t s);
// Optional blur of the OT field: dst = 3x3x3 Gaussian (sigma 1 voxel) of src, periodic over the
// node grid n[0] x n[1] x n[2].
struct BlurArgs {
  const void* src;
  void* dst;
  uint32_t n[3];
  int64_t cells;
};
hipError_t launch_blur(const BlurArgs& a, DType real, hipStream_t s);
// Whether the OT kernel takes columns of mp cells along the PE axis (at most 8192).
bool ot_column_supported(int mp);
hipError_t launch_restrict(const RestrictArgs& a, DType src, DType dst, hipStream_t s);
hipError_t launch_restrict_adjoint(const RestrictAdjArgs& a, DType real, hipStream_t s);
hipError_t launch_prolong(const ProlongArgs& a, DType real, hipStream_t s);
hipError_t launch_reset(const SetStateArgs& a, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_stats_header(double* stats, const State* st, const unsigned long long* guarded,
                               hipStream_t s);

}  // namespace rgp
