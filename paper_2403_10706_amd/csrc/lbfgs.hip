// L-BFGS direction on the device (Sec. 2.3.3: a quasi-Newton method on the explicit gradient).
//
// One L-BFGS step on a pyramid level is the objective/gradient launch of the Gauss-Newton solve
// (which also applies the previous accepted step), the kernels below, and the Armijo passes of
// the Gauss-Newton solve on the direction they leave in `x`.  The two-loop recursion (Nocedal and
// Wright, Algorithm 7.4) is a chain of streaming kernels, one per pair and loop: each applies the
// update of the previous pair (its coefficient reduced, in every block and in block order, from
// the previous kernel's FP64 block sums) and forms the block sums of the next pair's inner
// product.  The pairs live in a ring of m + 1 slots, so that a new pair can be written before it
// is known whether its curvature s^T y admits it, without overwriting the oldest pair kept.
//
// Launch sequence of step `it` (np = min(it, m) pairs at most, fixed when the solve is enqueued):
//   it >= 1: kPair (s = gamma x, y = g - g_old into the free slot; block sums s.y, y.y, s.s)
//   kLoop1 j = 0..np: j == 0 admits the new pair (metadata of this step from the previous
//     step's) and copies q = g; j >= 1 applies q -= alpha y of the (j-1)-th newest pair; then the
//     block sums of s.q of the j-th newest pair (or of max|g| when no pair is kept)
//   kMid: r = h0 q with h0 = s^T y / y^T y of the newest pair (1 / max|g| without pairs); block
//     sums of y.r of the oldest pair; records the pair count and h0 in the state
//   kLoop2 t = 1..np: r += (alpha - beta) s of the (t-1)-th oldest pair; block sums of y.r of the
//     t-th oldest
//   the last kernel of the chain writes d = -r.
// Pairs beyond the ones kept make their kernels no-ops; every kernel returns at once when the
// level has stopped (failed line search or barrier).
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "rgp_internal.hpp"
#include "rgp_launch.hpp"
#include "rgp_solver.hpp"

namespace rgp {

namespace {

constexpr int kLbBlock = 256;

__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ int ring_newest(const LbfgsMeta& m, int mem, int j) {
  // slot of the j-th newest pair kept (j = 0: the newest)
  const int r = mem + 1;
  return ((m.head - 1 - j) % r + r) % r;
}

// Block max of a non-negative value (exact: max does not depend on the order).
__device__ __forceinline__ double block_max(double v) {
  __shared__ double sh[kLbBlock];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kLbBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Max over nprod producer blocks of the column-major sum 0 of part.
__device__ __forceinline__ double reduce_max(const double* part, unsigned nprod) {
  double v = 0.0;
  for (unsigned b = threadIdx.x; b < nprod; b += kLbBlock) v = fmax(v, part[b]);
  return block_max(v);
}

// The metadata of this step: the previous step's, with the new pair admitted when its curvature
// is positive enough (t: s.y, y.y, s.s of the pair).
__device__ __forceinline__ LbfgsMeta admit(const LbfgsMeta& prev, const double (&t)[3], int mem) {
  LbfgsMeta m = prev;
  const double sy = t[0], yy = t[1], ss = t[2];
  if (sy > kLbfgsCurvature * sqrt(ss) * sqrt(yy)) {
    m.rho[m.head] = 1.0 / sy;
    m.h0 = sy / yy;
    m.head = (m.head + 1) % (mem + 1);
    m.count = m.count < mem ? m.count + 1 : mem;
  }
  return m;
}

template <typename TR>
__device__ void lbfgs_body(const LbfgsArgs& a) {
  if (load_flag(&a.st->gn_stop)) return;
  const int64_t n = a.n;
  const int64_t stride = (int64_t)gridDim.x * kLbBlock;
  const int64_t i0 = (int64_t)blockIdx.x * kLbBlock + threadIdx.x;
  TR* __restrict__ x = static_cast<TR*>(a.x);
  const TR* __restrict__ g = static_cast<const TR*>(a.g);
  TR* __restrict__ S = static_cast<TR*>(a.S);
  TR* __restrict__ Y = static_cast<TR*>(a.Y);

  if (a.phase == kLbPair) {
    const LbfgsMeta m = *a.meta_prev;
    const TR gam = (TR)a.st->gamma;
    const TR* __restrict__ go = static_cast<const TR*>(a.g_old);
    TR* __restrict__ s = S + (int64_t)m.head * n;
    TR* __restrict__ y = Y + (int64_t)m.head * n;
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0; i < n; i += stride) {
      const TR si = gam * x[i], yi = g[i] - go[i];
      s[i] = si;
      y[i] = yi;
      const double sd = (double)si, yd = (double)yi;
      v[0] = fma(sd, yd, v[0]);
      v[1] = fma(yd, yd, v[1]);
      v[2] = fma(sd, sd, v[2]);
    }
    store_partials_cm<3, kLbBlock>(v, a.part_out, blockIdx.x);
    return;
  }

  if (a.phase == kLbLoop1) {
    LbfgsMeta m;
    double coef = 0.0;   // alpha of the (j-1)-th newest pair
    if (a.j == 0) {
      if (a.np > 0) {
        double t[3];
        load_partials_cm<3>(t, a.part_in, a.nprod_in, 3);
        block_sum<3, kLbBlock>(t);
        m = admit(*a.meta_prev, t, a.mem);
      } else {
        m = LbfgsMeta{};
        m.head = 0;
        m.count = 0;
        m.h0 = 0.0;
      }
      if (blockIdx.x == 0 && threadIdx.x == 0) *a.meta = m;
    } else {
      m = *a.meta;
      if (a.j - 1 < m.count) {
        double t[1];
        load_partials_cm<1>(t, a.part_in, a.nprod_in, 1);
        block_sum<1, kLbBlock>(t);
        const int sl = ring_newest(m, a.mem, a.j - 1);
        coef = m.rho[sl] * t[0];
        if (blockIdx.x == 0 && threadIdx.x == 0) a.meta->alpha[a.j - 1] = coef;
      }
    }
    const bool upd = a.j >= 1 && a.j - 1 < m.count;
    const bool dot = a.j < m.count;
    if (a.j >= 1 && !upd) return;   // no pair left: nothing to do
    const TR* __restrict__ yu = Y + (int64_t)(upd ? ring_newest(m, a.mem, a.j - 1) : 0) * n;
    const TR* __restrict__ sd = S + (int64_t)(dot ? ring_newest(m, a.mem, a.j) : 0) * n;
    const TR c = (TR)coef;
    double v[1] = {0.0};
    double gmax = 0.0;
    for (int64_t i = i0; i < n; i += stride) {
      TR q;
      if (a.j == 0) {
        q = g[i];
        gmax = fmax(gmax, fabs((double)q));
      } else {
        q = fmad(-c, yu[i], x[i]);
      }
      x[i] = q;
      if (dot) v[0] = fma((double)sd[i], (double)q, v[0]);
    }
    if (dot) store_partials_cm<1, kLbBlock>(v, a.part_out, blockIdx.x);
    if (a.j == 0 && m.count == 0) {
      const double bm = block_max(gmax);
      if (threadIdx.x == 0) a.part_max[blockIdx.x] = bm;
    }
    return;
  }

  if (a.phase == kLbMid) {
    const LbfgsMeta m = *a.meta;
    double h;
    if (m.count > 0) {
      h = m.h0;
    } else {
      const double gm = reduce_max(a.part_max, a.nprod_in);
      h = gm > 0.0 ? 1.0 / gm : 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.st->pcg_iters = m.count;
      a.st->relres = h;
    }
    const bool dot = m.count > 0 && !a.last;
    const TR* __restrict__ yd = Y + (int64_t)(dot ? ring_newest(m, a.mem, m.count - 1) : 0) * n;
    const TR hh = (TR)h;
    double v[1] = {0.0};
    for (int64_t i = i0; i < n; i += stride) {
      const TR r = hh * x[i];
      x[i] = a.last ? -r : r;
      if (dot) v[0] = fma((double)yd[i], (double)r, v[0]);
    }
    if (dot) store_partials_cm<1, kLbBlock>(v, a.part_out, blockIdx.x);
    return;
  }

  // kLbLoop2, t = a.j >= 1: the (t-1)-th oldest pair is the (count - t)-th newest
  const LbfgsMeta m = *a.meta;
  const int t = a.j;
  const bool upd = t - 1 < m.count;
  const bool dot = t < m.count && !a.last;
  if (!upd && !a.last) return;
  double coef = 0.0;
  int su = 0;
  if (upd) {
    double tt[1];
    load_partials_cm<1>(tt, a.part_in, a.nprod_in, 1);
    block_sum<1, kLbBlock>(tt);
    const int jn = m.count - t;   // newest-first index of the pair being applied
    su = ring_newest(m, a.mem, jn);
    const double beta = m.rho[su] * tt[0];
    coef = m.alpha[jn] - beta;
  }
  const TR* __restrict__ sp = S + (int64_t)su * n;
  const TR* __restrict__ yd = Y + (int64_t)(dot ? ring_newest(m, a.mem, m.count - 1 - t) : 0) * n;
  const TR c = (TR)coef;
  double v[1] = {0.0};
  for (int64_t i = i0; i < n; i += stride) {
    TR r = x[i];
    if (upd) r = fmad(c, sp[i], r);
    x[i] = a.last ? -r : r;
    if (dot) v[0] = fma((double)yd[i], (double)r, v[0]);
  }
  if (dot) store_partials_cm<1, kLbBlock>(v, a.part_out, blockIdx.x);
}

template <typename TR>
__global__ __launch_bounds__(kLbBlock) void k_lbfgs(LbfgsArgs a) {
  lbfgs_body<TR>(a);
}

}  // namespace

unsigned lbfgs_grid(int64_t n) {
  const int64_t per = (int64_t)kLbBlock * 8;
  const int64_t b = (n + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

hipError_t launch_lbfgs(const LbfgsArgs& a0, DType real, hipStream_t s) {
  LbfgsArgs a = a0;
  a.nblk = lbfgs_grid(a.n);
  if (active_recorder())
    return record_other([a, real](hipStream_t s2) { return launch_lbfgs(a, real, s2); });
  if (real == DType::F64)
    hipLaunchKernelGGL(k_lbfgs<double>, dim3(a.nblk), dim3(kLbBlock), 0, s, a);
  else if (real == DType::F32)
    hipLaunchKernelGGL(k_lbfgs<float>, dim3(a.nblk), dim3(kLbBlock), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace rgp
