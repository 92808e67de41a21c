// L-BFGS direction on the device (Sec. 2.3.3: a quasi-Newton method on the explicit gradient).
//
// One L-BFGS step on a pyramid level is the objective/gradient launch of the Gauss-Newton solve
// (which also applies the previous accepted step), the three kernels below, and the Armijo passes
// of the Gauss-Newton solve on the direction they leave in `x`.  The two-loop recursion (Nocedal
// and Wright, Algorithm 7.4) touches the vectors only through inner products with s_i and y_i and
// through the final combination, so it runs on scalars: with the inner products s_i.g, y_i.g and
// the Gram entries s_i.y_j, y_i.y_j of the pairs kept (kept up to date as pairs arrive), every
// coefficient of both loops follows exactly as the loops would form it, and the direction is one
// combination d = cg g + sum (cs_i s_i + cy_i y_i).  Per step:
//   kLbDots: the new pair s = gamma x, y = g - g_old into the free ring slot (steps >= 1), and
//     the block sums of s.y, y.y, s.s and, for every pair of the window (the new one and those
//     kept so far), s_k.y, y_k.s, y_k.y, s_k.g, y_k.g; the block maxima of |g|
//   kLbScalar (one block): the sums; the admission of the pair (s^T y > 1e-10 |s| |y|), the Gram
//     entries of its slot, the two loops on scalars, cg, cs, cy, and the pair count and H0 scale
//     in the state (H0 = s^T y / y^T y of the newest pair, 1 / max|g| without pairs)
//   kLbCombine: d from the coefficients.
// The pairs live in a ring of m + 1 slots, so that a new pair can be written before it is known
// whether its curvature admits it, without overwriting the oldest pair kept.  Every kernel returns
// at once when the level has stopped (failed line search or barrier).
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

constexpr int kLbChunk = 4;   // window pairs per pass of kLbDots

template <typename TR>
__device__ void lbfgs_dots(const LbfgsArgs& a) {
  const int64_t n = a.n;
  const int t = threadIdx.x;
  const LbfgsMeta* mp = a.meta_prev;
  const bool pair = a.pair != 0;
  const int h = pair ? mp->head : 0;
  const int nwin = pair ? 1 + mp->count : 0;   // window: the new slot, then the kept, newest first
  const TR* __restrict__ g = static_cast<const TR*>(a.g);
  const TR* __restrict__ go = static_cast<const TR*>(a.g_old);
  const TR* __restrict__ x = static_cast<const TR*>(a.x);
  TR* __restrict__ S = static_cast<TR*>(a.S);
  TR* __restrict__ Y = static_cast<TR*>(a.Y);
  TR* __restrict__ sh = S + (int64_t)h * n;
  TR* __restrict__ yh = Y + (int64_t)h * n;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;   // a contiguous range per block
  const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
  const TR gam = pair ? (TR)a.st->gamma : TR(0);
  double v3[3] = {0.0, 0.0, 0.0};
  double gmax = 0.0;
  for (int64_t i = lo + t; i < hi; i += kLbBlock) {
    const TR gi = g[i];
    gmax = fmax(gmax, fabs((double)gi));
    if (pair) {
      const TR si = gam * x[i], yi = gi - go[i];
      sh[i] = si;
      yh[i] = yi;
      const double sd = (double)si, yd = (double)yi;
      v3[0] = fma(sd, yd, v3[0]);
      v3[1] = fma(yd, yd, v3[1]);
      v3[2] = fma(sd, sd, v3[2]);
    }
  }
  block_sum<3, kLbBlock>(v3);
  const double bm = block_max(gmax);
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) a.part[(size_t)q * kMaxGrid + blockIdx.x] = v3[q];
    a.part_max[blockIdx.x] = bm;
  }
  for (int w0 = 0; w0 < nwin; w0 += kLbChunk) {
    int sl[kLbChunk];
    bool on[kLbChunk];
#pragma unroll
    for (int c = 0; c < kLbChunk; ++c) {
      const int w = w0 + c;
      on[c] = w < nwin;
      sl[c] = !on[c] ? h : (w == 0 ? h : ring_newest(*mp, a.mem, w - 1));
    }
    double v[5 * kLbChunk];
#pragma unroll
    for (int q = 0; q < 5 * kLbChunk; ++q) v[q] = 0.0;
    for (int64_t i = lo + t; i < hi; i += kLbBlock) {
      const double gi = (double)g[i], si = (double)sh[i], yi = (double)yh[i];
#pragma unroll
      for (int c = 0; c < kLbChunk; ++c) {
        if (on[c]) {
          const double sk = (double)S[(int64_t)sl[c] * n + i], yk = (double)Y[(int64_t)sl[c] * n + i];
          v[5 * c + 0] = fma(sk, yi, v[5 * c + 0]);
          v[5 * c + 1] = fma(yk, si, v[5 * c + 1]);
          v[5 * c + 2] = fma(yk, yi, v[5 * c + 2]);
          v[5 * c + 3] = fma(sk, gi, v[5 * c + 3]);
          v[5 * c + 4] = fma(yk, gi, v[5 * c + 4]);
        }
      }
    }
    block_sum<5 * kLbChunk, kLbBlock>(v);
    if (t == 0) {
#pragma unroll
      for (int c = 0; c < kLbChunk; ++c)
        if (on[c])
#pragma unroll
          for (int q = 0; q < 5; ++q)
            a.part[(size_t)(3 + 5 * sl[c] + q) * kMaxGrid + blockIdx.x] = v[5 * c + q];
    }
  }
}

// FP64 sum over the lanes of wavefront 0 (all 64 active).
__device__ __forceinline__ double lane_sum(double v) {
  double t[1] = {v};
  wave_sums<1>(t);
  return t[0];
}

__device__ void lbfgs_scalar(const LbfgsArgs& a) {
  constexpr int R = kLbfgsMaxMem + 1;
  __shared__ double sums[3 + 5 * R];
  __shared__ double gsy[kLbfgsMaxMem][kLbfgsMaxMem], gyy[kLbfgsMaxMem][kLbfgsMaxMem];
  __shared__ double sg[kLbfgsMaxMem], yg[kLbfgsMaxMem], rh[kLbfgsMaxMem];
  __shared__ int sls[kLbfgsMaxMem];
  __shared__ int s_count, s_head;
  __shared__ double s_h0;
  const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
  const int mem = a.mem, Rm = mem + 1;
  const int K = 3 + 5 * Rm;
  const LbfgsMeta* mp = a.meta_prev;
  LbfgsMeta* m = a.meta;
  // every sum over the producer blocks: wavefront wv takes sums wv, wv + 4, ..., four at a time
  constexpr int kB = 4;
  for (int k0 = wv; k0 < K; k0 += 4 * kB) {
    double acc[kB];
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int k = k0 + 4 * q;
      acc[q] = 0.0;
      if (k < K)
        for (unsigned b = lane; b < a.nprod; b += kWave) acc[q] += a.part[(size_t)k * kMaxGrid + b];
    }
    wave_sums<kB>(acc);
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < kB; ++q)
        if (k0 + 4 * q < K) sums[k0 + 4 * q] = acc[q];
  }
  double gm = 0.0;
  for (unsigned b = t; b < a.nprod; b += kLbBlock) gm = fmax(gm, a.part_max[b]);
  gm = block_max(gm);   // synchronises: the sums are in LDS from here on
  // this step's metadata: the previous step's (zero on the first step of a level), then the pair
  const bool first = !a.pair;
  for (int i = t; i < Rm * Rm; i += kLbBlock) {
    const int r = i / Rm, c = i - r * Rm;
    m->sy[r][c] = first ? 0.0 : mp->sy[r][c];
    m->yy[r][c] = first ? 0.0 : mp->yy[r][c];
  }
  for (int i = t; i < Rm; i += kLbBlock) m->rho[i] = first ? 0.0 : mp->rho[i];
  __syncthreads();
  if (t == 0) {
    int head = first ? 0 : mp->head, count = first ? 0 : mp->count;
    double h0 = first ? 0.0 : mp->h0;
    if (a.pair) {
      const double sy = sums[0], yy = sums[1], ss = sums[2];
      if (sy > kLbfgsCurvature * sqrt(ss) * sqrt(yy)) {
        const int hs = head;
        // Gram entries of the new slot with every slot of the window (the kept and itself)
        for (int w = 0; w <= count; ++w) {
          const int k = w == 0 ? hs : ((hs - w) % Rm + Rm) % Rm;
          m->sy[k][hs] = sums[3 + 5 * k + 0];   // s_k . y_new
          m->sy[hs][k] = sums[3 + 5 * k + 1];   // s_new . y_k
          m->yy[k][hs] = sums[3 + 5 * k + 2];
          m->yy[hs][k] = sums[3 + 5 * k + 2];
        }
        m->rho[hs] = 1.0 / sy;
        h0 = sy / yy;
        head = (head + 1) % Rm;
        count = count < mem ? count + 1 : mem;
      }
    }
    m->head = head;
    m->count = count;
    m->h0 = h0;
    s_head = head;
    s_count = count;
    s_h0 = h0;
  }
  __syncthreads();
  const int count = s_count, head = s_head;
  // the kept pairs, newest first, and their inner products
  if (t < count) {
    const int sl = ((head - 1 - t) % Rm + Rm) % Rm;
    sls[t] = sl;
    sg[t] = sums[3 + 5 * sl + 3];
    yg[t] = sums[3 + 5 * sl + 4];
    rh[t] = m->rho[sl];
  }
  __syncthreads();
  for (int i = t; i < count * count; i += kLbBlock) {
    const int r = i / count, c = i - r * count;
    gsy[r][c] = m->sy[sls[r]][sls[c]];
    gyy[r][c] = m->yy[sls[r]][sls[c]];
  }
  __syncthreads();
  if (wv == 0) {
    const double hh = count > 0 ? s_h0 : (gm > 0.0 ? 1.0 / gm : 0.0);
    // first loop, newest first: alpha_j = rho_j s_j.q_j, q_j = g - sum_{j' < j} alpha_j' y_j'
    double al = 0.0;   // lane j holds alpha_j
    for (int j = 0; j < count; ++j) {
      const double part = lane < j ? al * gsy[j][lane] : 0.0;
      const double a_j = rh[j] * (sg[j] - lane_sum(part));
      if (lane == j) al = a_j;
    }
    // r = h q; second loop, oldest first: beta_j = rho_j y_j.r, r += (alpha_j - beta_j) s_j
    double cf = 0.0;   // lane j holds alpha_j - beta_j once applied
    for (int j = count - 1; j >= 0; --j) {
      const double p1 = lane < count ? al * gyy[j][lane] : 0.0;
      const double p2 = (lane > j && lane < count) ? cf * gsy[lane][j] : 0.0;
      const double yr = hh * yg[j] - hh * lane_sum(p1) + lane_sum(p2);
      const double b_j = rh[j] * yr;
      if (lane == j) cf = al - b_j;
    }
    // d = -r = -h g + h sum alpha_j y_j - sum (alpha_j - beta_j) s_j
    if (lane < count) {
      m->cy[sls[lane]] = hh * al;
      m->cs[sls[lane]] = -cf;
    }
    if (lane == 0) {
      m->cg = -hh;
      a.st->pcg_iters = count;
      a.st->relres = hh;
    }
  }
}

template <typename TR>
__device__ void lbfgs_combine(const LbfgsArgs& a) {
  __shared__ double cfs[kLbfgsMaxMem], cfy[kLbfgsMaxMem];
  __shared__ int sls[kLbfgsMaxMem];
  const LbfgsMeta* m = a.meta;
  const int count = m->count, Rm = a.mem + 1, t = threadIdx.x;
  if (t < count) {
    const int sl = ((m->head - 1 - t) % Rm + Rm) % Rm;
    sls[t] = sl;
    cfs[t] = m->cs[sl];
    cfy[t] = m->cy[sl];
  }
  const TR cg = (TR)m->cg;
  __syncthreads();
  const int64_t n = a.n;
  const TR* __restrict__ g = static_cast<const TR*>(a.g);
  const TR* __restrict__ S = static_cast<const TR*>(a.S);
  const TR* __restrict__ Y = static_cast<const TR*>(a.Y);
  TR* __restrict__ x = static_cast<TR*>(a.x);
  const int64_t stride = (int64_t)gridDim.x * kLbBlock;
  for (int64_t i = (int64_t)blockIdx.x * kLbBlock + t; i < n; i += stride) {
    TR d = cg * g[i];
    for (int j = 0; j < count; ++j) {
      const int64_t o = (int64_t)sls[j] * n + i;
      d = fmad((TR)cfy[j], Y[o], d);
      d = fmad((TR)cfs[j], S[o], d);
    }
    x[i] = d;
  }
}

template <typename TR>
__global__ __launch_bounds__(kLbBlock) void k_lbfgs(LbfgsArgs a) {
  if (load_flag(&a.st->gn_stop)) return;
  if (a.phase == kLbDots)
    lbfgs_dots<TR>(a);
  else if (a.phase == kLbScalar)
    lbfgs_scalar(a);
  else
    lbfgs_combine<TR>(a);
}

}  // namespace

unsigned lbfgs_grid(int64_t n) {
  const int64_t per = (int64_t)kLbBlock * 8;
  const int64_t b = (n + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

unsigned lbfgs_dots_grid(int64_t n) {
  const int64_t per = (int64_t)kLbBlock * 8;
  const int64_t b = (n + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : (b > 256 ? 256 : b));
}

hipError_t launch_lbfgs(const LbfgsArgs& a0, DType real, hipStream_t s) {
  LbfgsArgs a = a0;
  a.nblk = a.phase == kLbDots ? a.nprod : (a.phase == kLbScalar ? 1u : lbfgs_grid(a.n));
  if (active_recorder())
    return record_other([a, real](hipStream_t s2) { return launch_lbfgs(a, real, s2); });
  if (real == DType::F64)
    RGP_LAUNCH_TN(kKindLbfgs, a.phase, 0, a.n, k_lbfgs<double>, a.nblk, kLbBlock, 0, s, a);
  else if (real == DType::F32)
    RGP_LAUNCH_TN(kKindLbfgs, a.phase, 0, a.n, k_lbfgs<float>, a.nblk, kLbBlock, 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace rgp
