// Multilevel pyramid transfers for the coarse-to-fine schedule, and state initialisation.
//
// Restriction: a coarse cell is the mean of the existing fine cells of its 2x2x2 block
// (ceil(m/2) cells per axis, spacing doubled).  Prolongation of the staggered field map: per axis
// linear interpolation in physical coordinates - along the PE axis fine node k sits at coarse node
// coordinate k/2; across it the fine centre j sits at coarse centre coordinate (2j-1)/4, clamped
// to the outer coarse centres (constant extrapolation).  b keeps its physical units.
#include "rgp_internal.hpp"
#include "rgp_launch.hpp"
#include "batch.hpp"

namespace rgp {

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_restrict(RestrictArgs a) {
  const TI* __restrict__ src = static_cast<const TI*>(a.src);
  TO* __restrict__ dst = static_cast<TO*>(a.dst);
  const int64_t n = (int64_t)a.mc[0] * a.mc[1] * a.mc[2];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int c2 = (int)(i % a.mc[2]);
  const int c1 = (int)((i / a.mc[2]) % a.mc[1]);
  const int c0 = (int)(i / ((int64_t)a.mc[2] * a.mc[1]));
  double sum = 0.0;
  int cnt = 0;
  for (int d0 = 0; d0 < 2; ++d0) {
    const int f0 = 2 * c0 + d0;
    if (f0 >= a.mf[0]) continue;
    for (int d1 = 0; d1 < 2; ++d1) {
      const int f1 = 2 * c1 + d1;
      if (f1 >= a.mf[1]) continue;
      for (int d2 = 0; d2 < 2; ++d2) {
        const int f2 = 2 * c2 + d2;
        if (f2 >= a.mf[2]) continue;
        sum += to_real(src[((int64_t)f0 * a.mf[1] + f1) * a.mf[2] + f2], double());
        ++cnt;
      }
    }
  }
  dst[i] = from_real<TO>(sum / (double)cnt);
}

// Adjoint of the restriction: fine cell f takes the value of its coarse cell divided by the number
// of existing fine cells in that cell's 2x2x2 block (1, 2, 4 or 8, so the division is exact), and
// adds it to dst with `accumulate`.
template <typename TR>
__global__ __launch_bounds__(kBlock) void k_restrict_adjoint(RestrictAdjArgs a) {
  const TR* __restrict__ src = static_cast<const TR*>(a.src);
  TR* __restrict__ dst = static_cast<TR*>(a.dst);
  const int64_t n = (int64_t)a.mf[0] * a.mf[1] * a.mf[2];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int f2 = (int)(i % a.mf[2]);
  const int f1 = (int)((i / a.mf[2]) % a.mf[1]);
  const int f0 = (int)(i / ((int64_t)a.mf[2] * a.mf[1]));
  const int c0 = f0 >> 1, c1 = f1 >> 1, c2 = f2 >> 1;
  const int cnt = (2 * c0 + 1 < a.mf[0] ? 2 : 1) * (2 * c1 + 1 < a.mf[1] ? 2 : 1) *
                  (2 * c2 + 1 < a.mf[2] ? 2 : 1);
  const TR v = src[((int64_t)c0 * a.mc[1] + c1) * a.mc[2] + c2] / (TR)cnt;
  dst[i] = a.accumulate ? dst[i] + v : v;
}

// 1D interpolation stencil of one axis: up to two coarse indices with weights.
__device__ __forceinline__ void axis_weights(int j, int mc, bool node_axis, int& i0, int& i1,
                                             double& w1) {
  double t;
  int top;
  if (node_axis) {
    t = 0.5 * (double)j;
    top = mc;  // coarse nodes 0..mc
  } else {
    t = 0.5 * ((double)j + 0.5) - 0.5;
    top = mc - 1;  // coarse centres 0..mc-1
  }
  t = fmin(fmax(t, 0.0), (double)top);
  int f = (int)floor(t);
  if (f >= top) {
    i0 = i1 = top;
    w1 = 0.0;
    return;
  }
  i0 = f;
  i1 = f + 1;
  w1 = t - (double)f;
}

template <typename TR>
__global__ __launch_bounds__(kBlock) void k_prolong(ProlongArgs a) {
  const TR* __restrict__ src = static_cast<const TR*>(a.src);
  TR* __restrict__ dst = static_cast<TR*>(a.dst);
  int nf[3], nc[3];
  for (int d = 0; d < 3; ++d) {
    nf[d] = a.mf[d] + (d == a.pe ? 1 : 0);
    nc[d] = a.mc[d] + (d == a.pe ? 1 : 0);
  }
  const int64_t n = (int64_t)nf[0] * nf[1] * nf[2];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int f2 = (int)(i % nf[2]);
  const int f1 = (int)((i / nf[2]) % nf[1]);
  const int f0 = (int)(i / ((int64_t)nf[2] * nf[1]));
  int lo[3], hi[3];
  double w[3];
  const int fj[3] = {f0, f1, f2};
  for (int d = 0; d < 3; ++d) axis_weights(fj[d], a.mc[d], d == a.pe, lo[d], hi[d], w[d]);
  double acc = 0.0;
  for (int s0 = 0; s0 < 2; ++s0) {
    const double w0 = s0 ? w[0] : 1.0 - w[0];
    if (w0 == 0.0) continue;
    const int c0 = s0 ? hi[0] : lo[0];
    for (int s1 = 0; s1 < 2; ++s1) {
      const double w1 = s1 ? w[1] : 1.0 - w[1];
      if (w1 == 0.0) continue;
      const int c1 = s1 ? hi[1] : lo[1];
      for (int s2 = 0; s2 < 2; ++s2) {
        const double w2 = s2 ? w[2] : 1.0 - w[2];
        if (w2 == 0.0) continue;
        const int c2 = s2 ? hi[2] : lo[2];
        acc += w0 * w1 * w2 * (double)src[((int64_t)c0 * nc[1] + c1) * nc[2] + c2];
      }
    }
  }
  dst[i] = (TR)acc;
}

__global__ void k_reset(SetStateArgs a) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    State z = {};
    *a.st = z;
    if (a.guarded) *a.guarded = 0ull;
  }
}

__global__ __launch_bounds__(kBlock) void k_fill(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_stats_header(double* stats, const State* st, const unsigned long long* guarded) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    stats[0] = (double)*guarded;
    stats[1] = st->ot_shift;
    stats[2] = (double)st->status;
    stats[3] = 0.0;
  }
}

// Device-to-device copy of n 16-byte words (both ends 16-byte aligned): kU words per thread and
// round, all loads in flight before the stores.
__global__ __launch_bounds__(kBlock) void k_copy16(const uint4* __restrict__ src,
                                                   uint4* __restrict__ dst, int64_t n) {
  constexpr int kU = 4;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x; i0 < n; i0 += kU * stride) {
    uint4 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n) dst[i] = v[u];
    }
  }
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (active_recorder())
    return record_other([dst, src, bytes](hipStream_t s2) { return launch_copy(dst, src, bytes, s2); });
  if (bytes == 0) return hipSuccess;
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src) | bytes) & 15u)
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
  const int64_t n = (int64_t)(bytes / 16);
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  const unsigned grid = (unsigned)(blocks < 2048 ? blocks : 2048);
  hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kBlock), 0, s, static_cast<const uint4*>(src),
                     static_cast<uint4*>(dst), n);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (active_recorder())
    return record_other([p, n, v](hipStream_t s2) { return launch_fill(p, n, v, s2); });
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_stats_header(double* stats, const State* st, const unsigned long long* guarded,
                               hipStream_t s) {
  if (active_recorder())
    return record_other([stats, st, guarded](hipStream_t s2) {
      return launch_stats_header(stats, st, guarded, s2);
    });
  hipLaunchKernelGGL(k_stats_header, dim3(1), dim3(64), 0, s, stats, st, guarded);
  return hipGetLastError();
}

hipError_t launch_restrict(const RestrictArgs& a, DType src, DType dst, hipStream_t s) {
  if (active_recorder())
    return record_other([a, src, dst](hipStream_t s2) { return launch_restrict(a, src, dst, s2); });
  const int64_t n = (int64_t)a.mc[0] * a.mc[1] * a.mc[2];
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  if (nb == 0) return hipSuccess;
#define RGP_RESTRICT(TI, TO) hipLaunchKernelGGL((k_restrict<TI, TO>), dim3(nb), dim3(kBlock), 0, s, a)
  if (src == DType::F64 && dst == DType::F64) RGP_RESTRICT(double, double);
  else if (src == DType::F32 && dst == DType::F32) RGP_RESTRICT(float, float);
  else if (src == DType::F32 && dst == DType::F64) RGP_RESTRICT(float, double);
  else if (src == DType::BF16 && dst == DType::F32) RGP_RESTRICT(bf16_t, float);
  else if (src == DType::BF16 && dst == DType::F64) RGP_RESTRICT(bf16_t, double);
  else return hipErrorInvalidValue;
#undef RGP_RESTRICT
  return hipGetLastError();
}

hipError_t launch_restrict_adjoint(const RestrictAdjArgs& a, DType real, hipStream_t s) {
  if (active_recorder())
    return record_other([a, real](hipStream_t s2) { return launch_restrict_adjoint(a, real, s2); });
  const int64_t n = (int64_t)a.mf[0] * a.mf[1] * a.mf[2];
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  if (nb == 0) return hipSuccess;
  if (real == DType::F64)
    hipLaunchKernelGGL((k_restrict_adjoint<double>), dim3(nb), dim3(kBlock), 0, s, a);
  else if (real == DType::F32)
    hipLaunchKernelGGL((k_restrict_adjoint<float>), dim3(nb), dim3(kBlock), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_prolong(const ProlongArgs& a, DType real, hipStream_t s) {
  if (active_recorder())
    return record_other([a, real](hipStream_t s2) { return launch_prolong(a, real, s2); });
  int64_t n = 1;
  for (int d = 0; d < 3; ++d) n *= (int64_t)(a.mf[d] + (d == a.pe ? 1 : 0));
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  if (nb == 0) return hipSuccess;
  if (real == DType::F64)
    hipLaunchKernelGGL(k_prolong<double>, dim3(nb), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_prolong<float>, dim3(nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reset(const SetStateArgs& a, hipStream_t s) {
  if (active_recorder()) return record_other([a](hipStream_t s2) { return launch_reset(a, s2); });
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace rgp
