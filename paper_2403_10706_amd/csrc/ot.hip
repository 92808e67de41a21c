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
// A workgroup owns NC adjacent columns; each column is split into NSEG = 256/NC segments, one per
// thread.  Both CDFs are scanned in LDS (segment scan + segment offsets); the inverse for the
// first node of a segment is a binary search, later nodes advance monotonically (merge path).
#include "rgp_internal.hpp"
#include "rgp_launch.hpp"
#include "batch.hpp"

namespace rgp {

// ------------------------------------------------------------------------------------------
// Positivity shift: block-wise min and max|.| over both images; the OT kernel combines them.
// ------------------------------------------------------------------------------------------
template <typename TI>
__global__ __launch_bounds__(kBlock) void k_shift(ShiftArgs a) {
  const TI* __restrict__ P = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ M = static_cast<const TI*>(a.Im);
  double lo = inf_d(), hi = 0.0;
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
      }
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, kWave));
    hi = fmax(hi, __shfl_xor(hi, off, kWave));
  }
  __shared__ double sl[kBlock / kWave], sh[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  if (lane == 0) {
    sl[wv] = lo;
    sh[wv] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < kBlock / kWave; ++w) {
      lo = fmin(lo, sl[w]);
      hi = fmax(hi, sh[w]);
    }
    a.part[(size_t)blockIdx.x * kPartStride + 0] = lo;
    a.part[(size_t)blockIdx.x * kPartStride + 1] = hi;
    if (blockIdx.x == 0 && a.guarded) *a.guarded = 0ull;
  }
}

// Shift from the block-wise extrema (every thread of the calling block gets it).
__device__ __forceinline__ double shift_from(const double* part, unsigned nprod, double eps,
                                             bool empty) {
  __shared__ double sl[kBlock / kWave], sh[kBlock / kWave];
  double lo = inf_d(), hi = 0.0;
  for (unsigned b = threadIdx.x; b < nprod; b += blockDim.x) {
    lo = fmin(lo, part[(size_t)b * kPartStride + 0]);
    hi = fmax(hi, part[(size_t)b * kPartStride + 1]);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, kWave));
    hi = fmax(hi, __shfl_xor(hi, off, kWave));
  }
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  if (lane == 0) {
    sl[wv] = lo;
    sh[wv] = hi;
  }
  __syncthreads();
  lo = inf_d();
  hi = 0.0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
    lo = fmin(lo, sl[w]);
    hi = fmax(hi, sh[w]);
  }
  __syncthreads();
  if (empty) lo = 0.0;
  return fmax(0.0, -lo) + eps * hi;
}

// Largest i in [-1, m] with C[i] < r (C[-1] = -inf), i.e. lower_bound - 1.
__device__ __forceinline__ int lower_idx(const double* C, int stride, int m, double r) {
  int lo = 0, hi = m + 1;  // search first index with C >= r in [0, m+1)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (C[mid * stride] < r) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

// Spline inverse in index units, starting the search at i (monotone advance).
__device__ __forceinline__ double inv_from(const double* C, int stride, int m, double r, int& i) {
  while (i + 1 <= m && C[(i + 1) * stride] < r) ++i;
  if (i < 0) return 0.0;
  if (i >= m) return (double)m;
  const double c0 = C[i * stride], c1 = C[(i + 1) * stride];
  return (double)i + (r - c0) / (c1 - c0);
}

template <typename TI, typename TR>
__global__ __launch_bounds__(kBlock) void k_ot(OtArgs a, int nc) {
  extern __shared__ double lds[];
  const Geom g = a.g;
  const int mp = g.mp;
  const int nseg = kBlock / nc;
  const int stride = nc;                         // LDS layout X[k * nc + c]
  double* Cp = lds;                              // CDF of I+ (then scratch)
  double* Cm = Cp + (size_t)(mp + 1) * nc;       // CDF of I- (then guard scan)
  double* B0 = Cm + (size_t)(mp + 1) * nc;       // b0 per node
  double* segp = B0 + (size_t)(mp + 1) * nc;     // [nseg][nc] segment sums
  double* segm = segp + (size_t)nseg * nc;
  __shared__ int colflag[kBlock];
  __shared__ unsigned long long blockclip;

  const TI* __restrict__ Ip = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ Im = static_cast<const TI*>(a.Im);
  TR* __restrict__ b0 = static_cast<TR*>(a.b0);
  const double hp = g.hp;

  const int c = threadIdx.x % nc;
  const int seg = threadIdx.x / nc;
  const int64_t col = (int64_t)blockIdx.x * nc + c;
  const bool colok = col < g.ncol;
  const int64_t colc = colok ? col : g.ncol - 1;
  const int64_t ix = colc / g.ny, iy = colc - (colc / g.ny) * g.ny;
  const int64_t cb = ix * g.cxs + iy * g.cys;
  const int64_t nb = ix * g.nxs + iy * g.nys;
  double* cp = Cp + c;
  double* cm = Cm + c;
  double* bz = B0 + c;

  colflag[threadIdx.x] = 0;
  if (threadIdx.x == 0) blockclip = 0ull;

  // 1. shifted cell values, local inclusive scans per segment: C[j+1] = sum_{j0 <= j' <= j}.
  //    The cells of a segment are loaded kChunk at a time, all loads of a chunk in flight
  //    together (indices clamped into the column, surplus values unused); the first chunk is
  //    issued before the positivity shift is reduced, so the two overlap.
  const int L = (mp + nseg - 1) / nseg;
  const int j0 = min(mp, seg * L), j1 = min(mp, j0 + L);
  constexpr int kChunk = 16;
  TI vp[kChunk], vm[kChunk];
  auto load_chunk = [&](int jb) {
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int j = max(0, min(jb + u, j1 - 1));
      vp[u] = Ip[cb + (int64_t)j * g.cps];
      vm[u] = Im[cb + (int64_t)j * g.cps];
    }
  };
  load_chunk(j0);
  const double s = shift_from(a.shift_part, a.shift_nprod, a.eps, g.ncell == 0);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.st->ot_shift = s;
  double accp = 0.0, accm = 0.0;
  for (int jb = j0; jb < j1; jb += kChunk) {
    if (jb != j0) load_chunk(jb);
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int j = jb + u;
      if (j < j1) {
        accp += to_real(vp[u], double()) + s;
        accm += to_real(vm[u], double()) + s;
        cp[(j + 1) * stride] = accp;
        cm[(j + 1) * stride] = accm;
      }
    }
  }
  segp[seg * nc + c] = accp;
  segm[seg * nc + c] = accm;
  if (seg == 0) {
    cp[0] = 0.0;
    cm[0] = 0.0;
  }
  __syncthreads();
  {
    double offp = 0.0, offm = 0.0;
    for (int q = 0; q < seg; ++q) {
      offp += segp[q * nc + c];
      offm += segm[q * nc + c];
    }
    for (int j = j0; j < j1; ++j) {
      cp[(j + 1) * stride] += offp;
      cm[(j + 1) * stride] += offm;
    }
  }
  __syncthreads();
  const double Sp = cp[mp * stride], Sm = cm[mp * stride];
  const bool massok = Sp > 0.0 && Sm > 0.0;
  __syncthreads();
  if (massok) {  // C_k = S_k / S_m with C_0 = 0 and C_m = 1 exactly
    for (int j = j0; j < j1; ++j) {
      cp[(j + 1) * stride] = (j + 1 == mp) ? 1.0 : cp[(j + 1) * stride] / Sp;
      cm[(j + 1) * stride] = (j + 1 == mp) ? 1.0 : cm[(j + 1) * stride] / Sm;
    }
  }
  __syncthreads();

  // 2. b0 at the nodes of this segment (nodes split evenly over the segments).
  const int L2 = (mp + 1 + nseg - 1) / nseg;
  const int k0 = min(mp + 1, seg * L2), k1 = min(mp + 1, k0 + L2);
  {
    int ip = -2, im = -2;
    for (int k = k0; k < k1; ++k) {
      double v = 0.0;
      if (massok) {
        const double rm = cm[k * stride], rp = cp[k * stride];
        if (ip == -2) ip = lower_idx(cp, stride, mp, rm);
        if (im == -2) im = lower_idx(cm, stride, mp, rp);
        const double xp = inv_from(cp, stride, mp, rm, ip);
        const double xm = inv_from(cm, stride, mp, rp, im);
        v = 0.25 * hp * (xp - xm);
      }
      bz[k * stride] = v;
    }
  }
  __syncthreads();

  // 3. guard: clip slopes beyond +-guard_slope and re-integrate the column from b0_0 = 0.
  if (a.guard) {
    unsigned long long nclip = 0;
    for (int j = k0; j < k1 && j < mp; ++j) {
      const double sl = (bz[(j + 1) * stride] - bz[j * stride]) / hp;
      if (fabs(sl) > a.guard_slope) ++nclip;
    }
    if (nclip) {
      atomicOr(&colflag[c], 1);
      if (colok) atomicAdd(&blockclip, nclip);
    }
    __syncthreads();
    const bool flagged = colflag[c] != 0;
    if (flagged) {
      double acc = 0.0;
      for (int j = k0; j < k1 && j < mp; ++j) {
        double sl = (bz[(j + 1) * stride] - bz[j * stride]) / hp;
        sl = fmin(fmax(sl, -a.guard_slope), a.guard_slope);
        acc += sl * hp;
        cm[(j + 1) * stride] = acc;
      }
      segm[seg * nc + c] = acc;
    }
    __syncthreads();
    if (flagged) {
      double off = 0.0;
      for (int q = 0; q < seg; ++q) off += segm[q * nc + c];
      for (int k = k0; k < k1; ++k) bz[k * stride] = (k == k0) ? off : off + cm[k * stride];
    }
    if (threadIdx.x == 0 && blockclip && a.guarded) atomicAdd(a.guarded, blockclip);
    __syncthreads();
  }

  if (colok) {
    for (int k = k0; k < k1; ++k) b0[nb + (int64_t)k * g.nps] = (TR)bz[k * stride];
  }
}

unsigned shift_grid(int64_t n) {
  int64_t nb = (n + kBlock * 16 - 1) / (kBlock * 16);
  if (nb < 1) nb = 1;
  if (nb > 256) nb = 256;  // every OT block combines these block extrema
  return (unsigned)nb;
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

size_t ot_lds_bytes(int mp, int nc) {
  const int nseg = kBlock / nc;
  return ((size_t)(mp + 1) * nc * 3 + (size_t)nseg * nc * 2) * sizeof(double);
}

// Columns per workgroup: the most (up to 16) whose three FP64 column arrays leave room for four
// workgroups per CU (160 KB of LDS); the inverse-CDF phase is chains of dependent LDS reads, so
// resident workgroups matter more than columns per workgroup.  Long columns fall back to the most
// that fit at all.
int ot_cols_per_block(int mp) {
  for (int nc = 16; nc >= 1; nc >>= 1)
    if (ot_lds_bytes(mp, nc) <= 40 * 1024) return nc;
  for (int nc = 16; nc >= 1; nc >>= 1)
    if (ot_lds_bytes(mp, nc) <= 150 * 1024) return nc;
  return 0;
}

hipError_t launch_ot(const OtArgs& a, DType img, DType real, hipStream_t s) {
  if (active_recorder())
    return record_other([a, img, real](hipStream_t s2) { return launch_ot(a, img, real, s2); });
  const int nc = ot_cols_per_block(a.g.mp);
  if (nc == 0) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)((a.g.ncol + nc - 1) / nc);
  const size_t lds = ot_lds_bytes(a.g.mp, nc);
#define RGP_OT_LAUNCH(TI, TR)                                                         \
  do {                                                                                \
    hipFuncSetAttribute((const void*)k_ot<TI, TR>,                                   \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);        \
    RGP_LAUNCH(kKindOt, a.g, (k_ot<TI, TR>), nb, kBlock, lds, s, a, nc);              \
  } while (0)
  if (real == DType::F64 && img == DType::F64) RGP_OT_LAUNCH(double, double);
  else if (real == DType::F32 && img == DType::F32) RGP_OT_LAUNCH(float, float);
  else if (real == DType::F32 && img == DType::BF16) RGP_OT_LAUNCH(bf16_t, float);
  else if (real == DType::F64 && img == DType::F32) RGP_OT_LAUNCH(float, double);
  else if (real == DType::F64 && img == DType::BF16) RGP_OT_LAUNCH(bf16_t, double);
  else return hipErrorInvalidValue;
#undef RGP_OT_LAUNCH
  return hipGetLastError();
}

}  // namespace rgp
