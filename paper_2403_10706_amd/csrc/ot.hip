// Column-wise 1D optimal-transport initialisation of the field map (Sec. 2.2 of the paper).
//
// Per column (m cells, m+1 nodes along the PE axis), in FP64:
//   i+- <- i+- + s                 positivity shift s = max(0, -min I) + eps max|I| (both images)
//   C_k = sum_{j<k} i_j / sum_j i_j, k = 0..m   (nodal CDFs)
//   C^{-1}(r) = linear spline through (C_k, k)  (for r in (C_i, C_{i+1}]: i + (r-C_i)/(C_{i+1}-C_i))
//   b0_k = h/4 [C+^{-1}(C-_k) - C-^{-1}(C+_k)]
// which is the average of the displacement of T- = C_half^{-1} o C- and the negated displacement
// of T+ = C_half^{-1} o C+, with C_half^{-1} = (C+^{-1} + C-^{-1}) / 2.  Guard: a column with
// some |D b0| > guard_slope gets its slopes clipped and is re-integrated from b0_0 = 0.
//
// A workgroup owns a tile of adjacent columns, each split into segments of consecutive cells, one
// per thread.  The raw sums are scanned in registers and across the segments of a wavefront; one
// FP64 CDF per column sits in LDS at a time (first C+, then C-), searched once per segment and
// walked forward from there (the queries of a segment ascend).
#include <cmath>

#include "rgp_internal.hpp"
#include "rgp_launch.hpp"
#include "batch.hpp"

namespace rgp {

// ------------------------------------------------------------------------------------------
// Positivity shift: block-wise min and max|.| over both images, and whether any value is not
// finite (NaN or an infinity); the OT kernel combines them.  This is also the input scan of a
// correction that starts from a given field.
// ------------------------------------------------------------------------------------------
template <typename TI>
__global__ __launch_bounds__(kBlock) void k_shift(ShiftArgs a) {
  const TI* __restrict__ P = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ M = static_cast<const TI*>(a.Im);
  double lo = inf_d(), hi = 0.0, bad = 0.0;
  // kU elements of each image per thread and round, all loads in flight together (indices
  // clamped into the array; the surplus ones are not counted)
  constexpr int kU = 8;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x; i0 < a.n; i0 += kU * stride) {
    TI pv[kU], mv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = min(i0 + u * stride, a.n - 1);
      pv[u] = P[i];
      mv[u] = M[i];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (i0 + u * stride < a.n) {
        const double p = to_real(pv[u], double()), m = to_real(mv[u], double());
        lo = fmin(lo, fmin(p, m));
        hi = fmax(hi, fmax(fabs(p), fabs(m)));
        // |v| < inf fails for NaN and for the infinities
        if (!(fabs(p) < inf_d()) || !(fabs(m) < inf_d())) bad = 1.0;
      }
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, kWave));
    hi = fmax(hi, __shfl_xor(hi, off, kWave));
    bad = fmax(bad, __shfl_xor(bad, off, kWave));
  }
  __shared__ double sl[kBlock / kWave], sh[kBlock / kWave], sb[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  if (lane == 0) {
    sl[wv] = lo;
    sh[wv] = hi;
    sb[wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < kBlock / kWave; ++w) {
      lo = fmin(lo, sl[w]);
      hi = fmax(hi, sh[w]);
      bad = fmax(bad, sb[w]);
    }
    a.part[(size_t)blockIdx.x * kPartStride + 0] = lo;
    a.part[(size_t)blockIdx.x * kPartStride + 1] = hi;
    a.part[(size_t)blockIdx.x * kPartStride + 2] = bad;
    if (blockIdx.x == 0 && a.guarded) *a.guarded = 0ull;
  }
}

// Status of a correction that starts from a given field (no OT kernel reads the scan): one block
// combines the non-finite flags of the input scan's blocks.
__global__ __launch_bounds__(kBlock) void k_scan_status(const double* part, unsigned nprod,
                                                        State* st) {
  double bad = 0.0;
  for (unsigned b = threadIdx.x; b < nprod; b += kBlock)
    bad = fmax(bad, part[(size_t)b * kPartStride + 2]);
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (bad > 0.0) any = 1;  // benign race: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0 && any && st->status == 0) st->status = RGP_ENONFINITE;
}

// Spline inverse of one ascending run of queries against a nodal CDF C_0..C_m held with stride NC
// in LDS.  The bracket of r is the largest i in [-1, m] with C_i < r, with c0 = C_i and c1 = C_{i+1}
// (-inf and +inf past the ends); r in (C_i, C_{i+1}] maps to i + (r - C_i)/(C_{i+1} - C_i).

// a / d for finite d > 0: reciprocal estimate, two Newton-Raphson steps y <- y (2 - d y), and one
// residual correction of the quotient (within an ulp or two of the rounded quotient).
__device__ __forceinline__ double div_pos(double a, double d) {
  double y = __builtin_amdgcn_rcp(d);
  double e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  const double q = a * y;
  return fma(fma(-d, q, a), y, q);
}

// Number of nodes whose CDF value is below r (the bracket index + 1): binary lifting over powers
// of two from P/2 down, P the smallest power of two above m + 1, so every lane runs the same steps.
template <int NC>
__device__ __forceinline__ int count_below(const double* C, int m, double r) {
  const int P = 1 << (32 - __clz(m + 1));
  int pos = 0;
  for (int step = P >> 1; step > 0; step >>= 1) {
    const int t = pos + step - 1;
    const double v = C[min(t, m) * NC];
    pos = (t <= m && v < r) ? pos + step : pos;
  }
  return pos;
}

// FIRST: x[u] = C^{-1}(q[u]) for u < n; else x[u] = f (x[u] - C^{-1}(q[u])).
template <int NC, int LMAX, bool FIRST>
__device__ __forceinline__ void invert_run(const double* C, int m, const double (&q)[LMAX], int n,
                                           double f, double (&x)[LMAX]) {
  int i = count_below<NC>(C, m, q[0]) - 1;
  double c0 = i >= 0 ? C[max(i, 0) * NC] : -inf_d();
  double c1 = i < m ? C[min(i + 1, m) * NC] : inf_d();
#pragma unroll
  for (int u = 0; u < LMAX; ++u) {
    if (u < n) {
      const double r = q[u];
      if (u > 0) {
        while (c1 < r) {  // walk forward (c1 = +inf at i = m stops it)
          ++i;
          c0 = c1;
          const double nx = C[min(i + 1, m) * NC];
          c1 = i < m ? nx : inf_d();
        }
      }
      double y = (double)i + div_pos(r - c0, c1 - c0);
      y = i < 0 ? 0.0 : (i >= m ? (double)m : y);
      x[u] = FIRST ? y : f * (x[u] - y);
    }
  }
}

// Tiles of NC adjacent columns go to the XCDs in contiguous runs (the hardware deals workgroups to
// the 8 XCDs round-robin), so the tiles that share a cache line of the images meet in one L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned G) {
  if (G < 8u) return b;
  const unsigned x = b % 8u, q = b / 8u, per = G / 8u, rem = G % 8u;
  return x < rem ? x * (per + 1u) + q : rem * (per + 1u) + (x - rem) * per + q;
}

// One workgroup per tile of NC adjacent columns.  Thread (c, seg), c = tid % NC (adjacent lanes
// read adjacent columns of a row), seg = tid / NC, owns the cells [j0, j0 + n) of its column,
// n <= L = ceil(m / NSEG) <= LMAX, and the nodes j0+1 .. j0+n (segment 0 also node 0).
//   1. Raw cell values are summed in registers; the shift s enters as S_k = R_k + k s.  Segment
//      offsets: a scan over the segments of the wavefront (lanes NC apart), then the wavefront
//      totals through LDS, in the same barrier as the block extrema that give s.
//   2. C+ of the own nodes goes to LDS; the own C- values are its queries (b+ = C+^{-1}(C-_k)).
//      Then C- replaces C+ in the same LDS array and the own C+ values are the queries.  One
//      FP64 array per column keeps a full-resolution grid resident in a single round.
//   3. Guard: the slope of the first own cell takes the previous segment's last node through LDS.
template <typename TI, typename TR, int NC, int LMAX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LMAX <= 12 ? 4 : LMAX <= 16 ? 3 : 1))) void k_ot(OtArgs a) {
  constexpr int NSEG = kBlock / NC;
  constexpr int NW = kBlock / kWave;
  static_assert(NC >= 1 && NC <= kWave && kWave % NC == 0, "columns per tile");
  extern __shared__ double lds[];  // one nodal CDF per column, node k of column c at [k * NC + c]
  __shared__ double wtot[2][NW][NC];
  __shared__ double ext[3][NW];
  __shared__ double segx[NSEG][NC];  // last node of each segment, then clipped segment sums
  __shared__ int colflag[NC];
  __shared__ unsigned long long blockclip;

  const Geom g = a.g;
  const int mp = g.mp;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int c = tid % NC, seg = tid / NC;
  const int64_t col = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * NC + c;
  const bool colok = col < g.ncol;
  const uint32_t colc = (uint32_t)(colok ? col : g.ncol - 1);
  const uint32_t ix = fdiv(colc, g.by_ny), iy = colc - ix * (uint32_t)g.ny;
  const int L = (mp + NSEG - 1) / NSEG;
  const int j0 = min(mp, seg * L), n = min(mp, j0 + L) - j0;

  // 1. loads of the own cells (all in flight together), then the block extrema of the shift kernel
  const TI* __restrict__ srcp =
      static_cast<const TI*>(a.Ip) + ((int64_t)ix * g.cxs + (int64_t)iy * g.cys + (int64_t)j0 * g.cps);
  const TI* __restrict__ srcm =
      static_cast<const TI*>(a.Im) + ((int64_t)ix * g.cxs + (int64_t)iy * g.cys + (int64_t)j0 * g.cps);
  TI vp[LMAX], vm[LMAX];
#pragma unroll
  for (int u = 0; u < LMAX; ++u) {
    if (u < n) {
      vp[u] = srcp[(int64_t)u * g.cps];
      vm[u] = srcm[(int64_t)u * g.cps];
    }
  }
  double lo = inf_d(), hi = 0.0, bad = 0.0;
  for (unsigned b = tid; b < a.shift_nprod; b += kBlock) {
    lo = fmin(lo, a.shift_part[(size_t)b * kPartStride + 0]);
    hi = fmax(hi, a.shift_part[(size_t)b * kPartStride + 1]);
    bad = fmax(bad, a.shift_part[(size_t)b * kPartStride + 2]);
  }
  if (tid < NC) colflag[tid] = 0;
  if (tid == 0) blockclip = 0ull;

  double Cp[LMAX], Cm[LMAX];  // raw inclusive prefixes of the segment, later the own CDF values
  double accp = 0.0, accm = 0.0;
#pragma unroll
  for (int u = 0; u < LMAX; ++u) {
    if (u < n) {
      accp += to_real(vp[u], double());
      accm += to_real(vm[u], double());
    }
    Cp[u] = accp;
    Cm[u] = accm;
  }
  double incp = accp, incm = accm;
#pragma unroll
  for (int d = NC; d < kWave; d <<= 1) {
    const double tp = __shfl_up(incp, d, kWave), tm = __shfl_up(incm, d, kWave);
    if (lane >= d) {
      incp += tp;
      incm += tm;
    }
  }
  double offp = __shfl_up(incp, NC, kWave), offm = __shfl_up(incm, NC, kWave);
  if (lane < NC) offp = offm = 0.0;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, d, kWave));
    hi = fmax(hi, __shfl_xor(hi, d, kWave));
    bad = fmax(bad, __shfl_xor(bad, d, kWave));
  }
  if (lane >= kWave - NC) {
    wtot[0][w][c] = incp;
    wtot[1][w][c] = incm;
  }
  if (lane == 0) {
    ext[0][w] = lo;
    ext[1][w] = hi;
    ext[2][w] = bad;
  }
  __syncthreads();
  double totp = 0.0, totm = 0.0;
  lo = inf_d();
  hi = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const double xp = wtot[0][q][c], xm = wtot[1][q][c];
    if (q < w) {
      offp += xp;
      offm += xm;
    }
    totp += xp;
    totm += xm;
    lo = fmin(lo, ext[0][q]);
    hi = fmax(hi, ext[1][q]);
    bad = fmax(bad, ext[2][q]);
  }
  const double s = fmax(0.0, -lo) + a.eps * hi;
  if (blockIdx.x == 0 && tid == 0) {
    a.st->ot_shift = s;
    if (bad > 0.0 && a.st->status == 0) a.st->status = RGP_ENONFINITE;
  }
  const double Sp = totp + (double)mp * s, Sm = totm + (double)mp * s;
  // images with a non-finite value give the zero field (as a column without mass does)
  const bool massok = Sp > 0.0 && Sm > 0.0 && bad == 0.0;
  const double rSp = 1.0 / Sp, rSm = 1.0 / Sm;
#pragma unroll
  for (int u = 0; u < LMAX; ++u) {  // C_k = S_k / S_m for k = j0+1+u, C_m = 1 exactly
    const int k = j0 + 1 + u;
    Cp[u] = k >= mp ? 1.0 : ((offp + Cp[u]) + (double)k * s) * rSp;
    Cm[u] = k >= mp ? 1.0 : ((offm + Cm[u]) + (double)k * s) * rSm;
  }

  // 2. b+ = C+^{-1}(C-_k) against C+ in LDS, then b- = C-^{-1}(C+_k) against C- in LDS
  double* C = lds + c;
  double bv[LMAX];  // C+^{-1}(C-_k), then b0_k
#pragma unroll
  for (int u = 0; u < LMAX; ++u) bv[u] = 0.0;
  if (seg == 0) C[0] = 0.0;
#pragma unroll
  for (int u = 0; u < LMAX; ++u)
    if (u < n) C[(j0 + 1 + u) * NC] = Cp[u];
  __syncthreads();
  if (massok && n > 0) invert_run<NC, LMAX, true>(C, mp, Cm, n, 0.0, bv);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < LMAX; ++u)
    if (u < n) C[(j0 + 1 + u) * NC] = Cm[u];
  __syncthreads();
  const double hp = g.hp;
  if (massok && n > 0) invert_run<NC, LMAX, false>(C, mp, Cp, n, 0.25 * hp, bv);

  // 3. guard: clip slopes beyond +-guard_slope and re-integrate the column from b0_0 = 0
  if (a.guard) {
    double last = 0.0;
#pragma unroll
    for (int u = 0; u < LMAX; ++u)
      if (u == n - 1) last = bv[u];
    if (n > 0) segx[seg][c] = last;
    __syncthreads();
    const double b00 = (seg == 0 || n == 0) ? 0.0 : segx[seg - 1][c];
    unsigned long long nclip = 0;
    const double dmax = a.guard_slope * hp;  // |D b0| > slope  <=>  |b0_{k+1} - b0_k| > slope h
    double prev = b00;
#pragma unroll
    for (int u = 0; u < LMAX; ++u) {
      if (u < n) {
        if (fabs(bv[u] - prev) > dmax) ++nclip;
        prev = bv[u];
      }
    }
    if (nclip) {
      atomicOr(&colflag[c], 1);
      if (colok) atomicAdd(&blockclip, nclip);
    }
    __syncthreads();
    if (blockclip) {
      const bool flagged = colflag[c] != 0;
      if (flagged) {
        double acc = 0.0;
        prev = b00;
#pragma unroll
        for (int u = 0; u < LMAX; ++u) {
          if (u < n) {
            const double d = fmin(fmax(bv[u] - prev, -dmax), dmax);
            prev = bv[u];
            acc += d;
            bv[u] = acc;
          }
        }
        segx[seg][c] = acc;
      }
      __syncthreads();
      if (flagged) {
        double off = 0.0;
        for (int q = 0; q < seg; ++q) off += segx[q][c];
#pragma unroll
        for (int u = 0; u < LMAX; ++u) bv[u] += off;
      }
      if (tid == 0 && a.guarded) atomicAdd(a.guarded, blockclip);
    }
  }

  if (colok) {
    TR* __restrict__ out = static_cast<TR*>(a.b0) + ((int64_t)ix * g.nxs + (int64_t)iy * g.nys);
    if (seg == 0) out[0] = (TR)0.0;
#pragma unroll
    for (int u = 0; u < LMAX; ++u)
      if (u < n) out[(int64_t)(j0 + 1 + u) * g.nps] = (TR)bv[u];
  }
}

// ------------------------------------------------------------------------------------------
// Optional blur of the OT field: the 3x3x3 Gaussian of standard deviation 1 voxel, normalised
// to sum 1, is the product of three 1D factors [a, 1, a] / (1 + 2a) with a = exp(-1/2); neighbour
// indices wrap around every axis (the paper applies the blur as an FFT convolution).  One node
// per thread, adjacent lanes on adjacent nodes of the contiguous axis; the node index splits with
// multiply-shift divisions and the 27 taps hit L1/L2.  Measured alternatives: runs of 8 nodes per
// thread (3x slower: lanes 8 nodes apart break the coalescing) and taking the two neighbours
// along the contiguous axis from the adjacent lanes (DPP; 7 % slower).
// ------------------------------------------------------------------------------------------
template <typename TR>
__global__ __launch_bounds__(kBlock) void k_blur(BlurArgs a, TR we, TR wc, FastDiv by_n2,
                                                 FastDiv by_n1) {
  const uint32_t n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n0 * n1 * n2) return;
  const TR* __restrict__ src = static_cast<const TR*>(a.src);
  const TR w[3] = {we, wc, we};
  const uint32_t r = fdiv(t, by_n2), i2 = t - r * n2, i0 = fdiv(r, by_n1), i1 = r - i0 * n1;
  const uint32_t j0[3] = {i0 == 0 ? n0 - 1 : i0 - 1, i0, i0 + 1 == n0 ? 0u : i0 + 1};
  const uint32_t j1[3] = {i1 == 0 ? n1 - 1 : i1 - 1, i1, i1 + 1 == n1 ? 0u : i1 + 1};
  const uint32_t j2[3] = {i2 == 0 ? n2 - 1 : i2 - 1, i2, i2 + 1 == n2 ? 0u : i2 + 1};
  TR v[3][3][3];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int u = 0; u < 3; ++u) v[p][q][u] = src[(j0[p] * n1 + j1[q]) * n2 + j2[u]];
  TR acc = TR(0);
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    TR s1 = TR(0);
#pragma unroll
    for (int q = 0; q < 3; ++q)
      s1 += w[q] * (w[0] * v[p][q][0] + w[1] * v[p][q][1] + w[2] * v[p][q][2]);
    acc += w[p] * s1;
  }
  static_cast<TR*>(a.dst)[t] = acc;
}

hipError_t launch_blur(const BlurArgs& a, DType real, hipStream_t s) {
  if (active_recorder())
    return record_other([a, real](hipStream_t s2) { return launch_blur(a, real, s2); });
  const int64_t total = (int64_t)a.n[0] * a.n[1] * a.n[2];
  if (total < 1 || total > (int64_t(1) << 30)) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)((total + kBlock - 1) / kBlock);
  const double ea = std::exp(-0.5), z = 1.0 + 2.0 * ea;
  const FastDiv d2 = make_fastdiv(a.n[2]), d1 = make_fastdiv(a.n[1]);
  if (real == DType::F64)
    RGP_LAUNCH_N(kKindBlur, a.cells, total, k_blur<double>, nb, kBlock, 0, s, a, ea / z, 1.0 / z,
                 d2, d1);
  else if (real == DType::F32)
    RGP_LAUNCH_N(kKindBlur, a.cells, total, k_blur<float>, nb, kBlock, 0, s, a, (float)(ea / z),
                 (float)(1.0 / z), d2, d1);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

unsigned shift_grid(int64_t n) {
  int64_t nb = (n + kBlock * 16 - 1) / (kBlock * 16);
  if (nb < 1) nb = 1;
  if (nb > 256) nb = 256;  // every OT block combines these block extrema
  return (unsigned)nb;
}

hipError_t launch_scan_status(const double* part, unsigned nprod, State* st, hipStream_t s) {
  if (active_recorder())
    return record_other([part, nprod, st](hipStream_t s2) {
      return launch_scan_status(part, nprod, st, s2);
    });
  hipLaunchKernelGGL(k_scan_status, dim3(1), dim3(kBlock), 0, s, part, nprod, st);
  return hipGetLastError();
}

hipError_t launch_shift(const ShiftArgs& a, DType img, hipStream_t s) {
  if (active_recorder())
    return record_other([a, img](hipStream_t s2) { return launch_shift(a, img, s2); });
  const unsigned nb = shift_grid(a.n);
  if (img == DType::F64)
    RGP_LAUNCH_N(kKindShift, a.n, 0, k_shift<double>, nb, kBlock, 0, s, a);
  else if (img == DType::F32)
    RGP_LAUNCH_N(kKindShift, a.n, 0, k_shift<float>, nb, kBlock, 0, s, a);
  else
    RGP_LAUNCH_N(kKindShift, a.n, 0, k_shift<bf16_t>, nb, kBlock, 0, s, a);
  return hipGetLastError();
}

// Columns per tile and register slots per segment: 16 threads per column while the segments
// hold at most 16 cells, fewer columns (longer segments) for longer columns.
struct OtShape {
  int nc, lmax;
};
OtShape ot_shape(int mp) {
  if (mp <= 128) return {16, 8};
  if (mp <= 192) return {16, 12};
  if (mp <= 256) return {16, 16};
  if (mp <= 512) return {8, 16};
  if (mp <= 1024) return {4, 16};
  if (mp <= 4096) return {1, 16};
  if (mp <= 8192) return {1, 32};
  return {0, 0};
}

bool ot_column_supported(int mp) { return ot_shape(mp).nc != 0; }

template <typename TI, typename TR, int NC, int LMAX>
hipError_t launch_ot_tile(const OtArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)((a.g.ncol + NC - 1) / NC);
  const size_t lds = (size_t)(a.g.mp + 1) * NC * sizeof(double);
  if (lds > 48 * 1024) {  // long columns: raise the dynamic LDS limit of the kernel
    const hipError_t e = hipFuncSetAttribute((const void*)k_ot<TI, TR, NC, LMAX>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  RGP_LAUNCH(kKindOt, a.g, (k_ot<TI, TR, NC, LMAX>), nb, kBlock, lds, s, a);
  return hipGetLastError();
}

template <typename TI, typename TR>
hipError_t launch_ot_typed(const OtArgs& a, hipStream_t s) {
  const OtShape sh = ot_shape(a.g.mp);
  if (sh.nc == 16 && sh.lmax == 8) return launch_ot_tile<TI, TR, 16, 8>(a, s);
  if (sh.nc == 16 && sh.lmax == 12) return launch_ot_tile<TI, TR, 16, 12>(a, s);
  if (sh.nc == 16) return launch_ot_tile<TI, TR, 16, 16>(a, s);
  if (sh.nc == 8) return launch_ot_tile<TI, TR, 8, 16>(a, s);
  if (sh.nc == 4) return launch_ot_tile<TI, TR, 4, 16>(a, s);
  if (sh.nc == 1 && sh.lmax == 16) return launch_ot_tile<TI, TR, 1, 16>(a, s);
  if (sh.nc == 1) return launch_ot_tile<TI, TR, 1, 32>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_ot(const OtArgs& a, DType img, DType real, hipStream_t s) {
  if (active_recorder())
    return record_other([a, img, real](hipStream_t s2) { return launch_ot(a, img, real, s2); });
  if (ot_shape(a.g.mp).nc == 0 || a.shift_nprod > (unsigned)kMaxGrid) return hipErrorInvalidValue;
  if (real == DType::F64 && img == DType::F64) return launch_ot_typed<double, double>(a, s);
  if (real == DType::F32 && img == DType::F32) return launch_ot_typed<float, float>(a, s);
  if (real == DType::F32 && img == DType::BF16) return launch_ot_typed<bf16_t, float>(a, s);
  if (real == DType::F64 && img == DType::F32) return launch_ot_typed<float, double>(a, s);
  if (real == DType::F64 && img == DType::BF16) return launch_ot_typed<bf16_t, double>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace rgp
