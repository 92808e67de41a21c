// Kernel argument blocks and host launchers of librgp (internal; not part of the C-ABI).
#pragma once

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

struct LossGradArgs {
  Geom g;
  const void* Ip;
  const void* Im;
  const void* b_in;
  const void* q;      // step direction (used when step != 0)
  void* b_out;        // receives b_in + gamma q (or b_in); may be null when step == 0
  void* grad;         // nullable
  void* diag;         // nullable (then off is ignored)
  void* off;
  double alpha, beta;
  State* st;
  double* partials;
  unsigned* counter;
  double* jdsp;       // nullable: J, D, S, P
  double* record;     // nullable: stats record of this GN step
  int step;           // apply the pending line-search step first
  int gn_mode;        // maintain gn_stop
};

struct TrialArgs {
  Geom g;
  const void* Ip;
  const void* Im;
  const void* b;
  const void* q;
  const void* grad;
  double alpha, beta, armijo_c;
  State* st;
  double* partials;
  unsigned* counter;
  double* record;
  int first;       // index of the first candidate (gamma = 2^-first)
  int last_pass;   // no candidate accepted after this pass -> stop
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
  double* partials;
  unsigned* counter;
  double* vHv;   // nullable
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
  double alpha;       // smoothness weight (cross-axis couplings)
  State* st;
  double* partials;
  unsigned* counter;
  int iter, maxit;
  double rtol;
  int gn_mode;
  int32_t* iters_out;   // nullable
  double* relres_out;   // nullable
};

struct ShiftArgs {
  const void* Ip;
  const void* Im;
  int64_t n;
  double eps;
  State* st;
  double* partials;
  unsigned* counter;
};

struct OtArgs {
  Geom g;
  const void* Ip;
  const void* Im;
  void* b0;
  const State* st;      // ot_shift
  int guard;
  double guard_slope;
  unsigned long long* guarded;   // nullable counter (zeroed by the host sequence)
};

struct RestrictArgs {
  const void* src;
  void* dst;
  int32_t mf[3], mc[3];
};

struct ProlongArgs {
  const void* src;   // coarse field
  void* dst;         // fine field
  int32_t mf[3], mc[3];
  int32_t pe;
};

struct SetStateArgs {
  State* st;
  unsigned* counter;
  unsigned long long* guarded;
};

unsigned loss_grad_blocks(const Geom& g);
unsigned trial_blocks(const Geom& g);
unsigned hvp_blocks(const Geom& g);
unsigned pcg_blocks(const Geom& g);
unsigned shift_blocks(int64_t n);

hipError_t launch_loss_grad(const LossGradArgs& a, DType img, DType real, hipStream_t s);
hipError_t launch_trial(const TrialArgs& a, int ncand, DType img, DType real, hipStream_t s);
hipError_t launch_apply_step(const ApplyArgs& a, DType real, hipStream_t s);
hipError_t launch_correct(const CorrectArgs& a, DType img, DType real, hipStream_t s);
hipError_t launch_hvp(const HvpArgs& a, DType real, hipStream_t s);
hipError_t launch_pcg_step(const PcgArgs& a, DType real, hipStream_t s);
hipError_t launch_shift(const ShiftArgs& a, DType img, hipStream_t s);
hipError_t launch_ot(const OtArgs& a, DType img, DType real, hipStream_t s);
hipError_t launch_restrict(const RestrictArgs& a, DType src, DType dst, hipStream_t s);
hipError_t launch_prolong(const ProlongArgs& a, DType real, hipStream_t s);
hipError_t launch_reset(const SetStateArgs& a, hipStream_t s);

}  // namespace rgp
