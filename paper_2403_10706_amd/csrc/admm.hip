// ADMM (Sec. 2.3.2, Eq. 8-11): the column-parallel b-update solve, the z-update by a separable
// orthogonal transform, the multiplier update and the adaptation of rho.
//
// b-update.  One Gauss-Newton step on F_rho = D + alpha S3 + beta P + (rho vol / 2)|b - c|^2
// (c = z - u): loss_grad and the Armijo passes run in their proximal mode; the search direction
// solves the Gauss-Newton system of F_rho, one tridiagonal block per PE column, with
// Jacobi-preconditioned CG on every column independently (k_block_pcg).  A 16-lane row of a
// wavefront owns one column, each lane a run of NPL consecutive nodes held in registers for the
// whole solve; a column's inner products are row sums by DPP (every lane of the row gets the
// total, in a fixed order) and the neighbours of a run's end nodes come from the adjacent lanes
// (DPP row shifts).  Each column has its own step sizes and its own stop.  T p is accumulated in
// FP64 (for smooth p the Laplacian terms nearly cancel).
//
// z-update.  (alpha L12 + rho I) z = rho (b + u) with L12 the Laplacian of periodic differences
// across the PE axis: the normalised discrete Hartley transforms H_A, H_B along the two cross
// axes (H = cas(2 pi j l / n) / sqrt(n), cas = cos + sin) diagonalise the periodic second
// differences of their axis, are symmetric and are their own inverses, so
// z = (H_A x H_B) diag(1 / (alpha (lambda_A + lambda_B) + rho)) (H_A x H_B) rho (b + u) with
// lambda(k) = (2 - 2 cos(2 pi k / n)) / h^2 - the same solution as the FFT of the paper.  Four
// passes of k_dht, each transforming lines along one axis in LDS (a table of n cosine and sine
// pairs indexed by j l mod n; the cosine and sine sums of frequency l give H x at l and at n - l):
// B (from rho (b + u)), A with the scaling, A, B (fused with the multiplier update and the
// residual sums of the rho adaptation).
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "rgp_internal.hpp"
#include "rgp_launch.hpp"
#include "rgp_solver.hpp"

namespace rgp {

namespace {

constexpr int kBpBlock = 256;          // 4 wavefronts, 16 columns per block
constexpr int kBpColsPerBlock = 16;
constexpr int kDhtBlock = 256;
constexpr int kDhtElems = 2048;        // line elements per workgroup (LDS)
constexpr int kDhtLines = 2;           // lines per Hartley work item (they share the table index)

__device__ __forceinline__ double fmad64(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int CTRL>
__device__ __forceinline__ float dpp_edge(float v, float edge) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_edge(double v, double edge) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(edge), __double2loint(v), CTRL, 0xF,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(edge), __double2hiint(v), CTRL, 0xF,
                                             0xF, false);
  return __hiloint2double(hi, lo);
}
// value of the previous / next lane of the same 16-lane row (edge on the row's first / last lane)
template <typename T>
__device__ __forceinline__ T row_prev(T v, T edge) { return dpp_edge<0x111>(v, edge); }
template <typename T>
__device__ __forceinline__ T row_next(T v, T edge) { return dpp_edge<0x101>(v, edge); }

// Sum over the 16 lanes of a row, every lane receiving it (same order in every row).
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_row<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_row<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_row<0x141>(v);  // row_half_mirror
  v += dpp_row<0x140>(v);  // row_mirror
  return v;
}

template <typename TR, int NPL>
__global__ __launch_bounds__(kBpBlock) void k_block_pcg(BlockPcgArgs a) {
  if (load_flag(&a.st->gn_stop)) return;
  const Geom g = a.g;
  const int mp = g.mp;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int seg = lane & 15;
  const TR* __restrict__ dg = static_cast<const TR*>(a.diag);
  const TR* __restrict__ og = static_cast<const TR*>(a.off);
  const TR* __restrict__ gg = static_cast<const TR*>(a.grad);
  TR* __restrict__ xg = static_cast<TR*>(a.x);
  double mit = 0.0, mrel = 0.0;   // this block's largest iteration count and relative residual
  const int64_t ngroups = (g.ncol + kBpColsPerBlock - 1) / kBpColsPerBlock;
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t col = grp * kBpColsPerBlock + wv * 4 + (lane >> 4);
    const bool colok = col < g.ncol;
    const int64_t cc = colok ? col : 0;
    const int64_t ix = cc / g.ny, iy = cc - ix * g.ny;
    const int64_t nb = ix * g.nxs + iy * g.nys;
    TR d[NPL], di[NPL], o[NPL], r[NPL], x[NPL], p[NPL];   // di = 1/d: the Jacobi step is r di
    double rr0 = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int k = seg * NPL + i;
      const bool ok = colok && k <= mp;
      const int64_t e = nb + (int64_t)(ok ? k : 0) * g.nps;
      d[i] = ok ? dg[e] : TR(1);
      di[i] = TR(1) / d[i];
      o[i] = ok && k < mp ? og[e] : TR(0);
      r[i] = ok ? -gg[e] : TR(0);
      x[i] = TR(0);
      rr0 = fmad64((double)r[i], (double)r[i], rr0);
    }
    const double nbv = sqrt(row_sum(rr0));
    double rz = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      p[i] = r[i] * di[i];
      rz = fmad64((double)r[i], (double)p[i], rz);
    }
    rz = row_sum(rz);
    bool active = nbv > 0.0;
    int its = 0;
    double relres = active ? 1.0 : 0.0;
    for (int it = 0; it < a.maxit; ++it) {
      if (!__any(active)) break;
      // q = T p with the neighbours of the run's end nodes from the adjacent lanes
      const TR pl = row_prev(p[NPL - 1], TR(0)), ol = row_prev(o[NPL - 1], TR(0));
      const TR pn = row_next(p[0], TR(0));
      TR q[NPL];
      double pq = 0.0;
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        const TR pm = i > 0 ? p[i - 1] : pl, pp = i < NPL - 1 ? p[i + 1] : pn;
        const TR om = i > 0 ? o[i - 1] : ol;
        double w = (double)d[i] * (double)p[i];
        w = fmad64((double)o[i], (double)pp, w);
        w = fmad64((double)om, (double)pm, w);
        q[i] = (TR)w;
        pq = fmad64((double)p[i], (double)q[i], pq);
      }
      pq = row_sum(pq);
      active = active && pq > 0.0;
      const TR al = active ? (TR)(rz / pq) : TR(0);
      double rr = 0.0;
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        x[i] = fma(al, p[i], x[i]);
        r[i] = fma(-al, q[i], r[i]);
        rr = fmad64((double)r[i], (double)r[i], rr);
      }
      rr = row_sum(rr);
      if (active) {
        ++its;
        relres = sqrt(rr) / nbv;
      }
      const bool cont = active && !(relres < a.rtol);
      double rzn = 0.0;
      TR z[NPL];
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        z[i] = r[i] * di[i];
        rzn = fmad64((double)r[i], (double)z[i], rzn);
      }
      rzn = row_sum(rzn);
      const TR be = cont ? (TR)(rzn / rz) : TR(0);
#pragma unroll
      for (int i = 0; i < NPL; ++i)
        if (cont) p[i] = fma(be, p[i], z[i]);
      if (cont) rz = rzn;
      active = cont;
    }
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int k = seg * NPL + i;
      if (colok && k <= mp) xg[nb + (int64_t)k * g.nps] = x[i];
    }
    if (colok) {
      mit = fmax(mit, (double)its);
      mrel = fmax(mrel, relres);
    }
  }
  // block maxima (order-independent), column-major partials
  __shared__ double sh[2][kBpBlock];
  sh[0][threadIdx.x] = mit;
  sh[1][threadIdx.x] = mrel;
  __syncthreads();
  for (int w = kBpBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
      sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = sh[0][0];
    a.part[kMaxGrid + blockIdx.x] = sh[1][0];
  }
}

// The largest column iteration count and relative residual into the state (one block).
__global__ __launch_bounds__(kBpBlock) void k_block_pcg_stats(BlockPcgArgs a) {
  if (load_flag(&a.st->gn_stop)) return;
  double mit = 0.0, mrel = 0.0;
  for (unsigned b = threadIdx.x; b < a.nblk; b += kBpBlock) {
    mit = fmax(mit, a.part[b]);
    mrel = fmax(mrel, a.part[kMaxGrid + b]);
  }
  __shared__ double sh[2][kBpBlock];
  sh[0][threadIdx.x] = mit;
  sh[1][threadIdx.x] = mrel;
  __syncthreads();
  for (int w = kBpBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
      sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.st->pcg_iters = (int32_t)sh[0][0];
    a.st->relres = sh[1][0];
  }
}

// ---- z-update ---------------------------------------------------------------------------------

// A tile of consecutive lines (line stride n | 1, odd) sits in LDS; a work item is two lines and
// one frequency pair, with the line pairs varying fastest across the lanes, so the lanes of a
// wavefront read few distinct table entries (multicast) and lines in distinct banks.  Element,
// line and work-item indices split by multiply-shift divisions in 32 bits (a field has at most
// 2^28 nodes).
template <typename TR>
__global__ __launch_bounds__(kDhtBlock) void k_dht(DhtArgs a) {
  if (load_flag(&a.st->gn_stop)) return;
  const int t = a.axis;
  const int n = a.n[t], ns = n | 1;
  const bool scale = a.mode == kDhtScale;
  // LDS sized to n: the scaling pass's eigenvalue terms of this axis (n doubles), the table of
  // cos, sin of 2 pi j / n (scaled by 1/sqrt(n), interleaved), the tile
  extern __shared__ __align__(16) unsigned char dht_lds[];
  double* __restrict__ lt = reinterpret_cast<double*>(dht_lds);
  TR* __restrict__ cs = reinterpret_cast<TR*>(lt + (scale ? n : 0));
  TR* __restrict__ xs = cs + 2 * n;
  // the two other axes, slower first
  const int u0 = t == 0 ? 1 : 0, u1 = t == 2 ? 1 : 2;
  const uint32_t st3[3] = {(uint32_t)a.n[1] * (uint32_t)a.n[2], (uint32_t)a.n[2], 1u};
  const uint32_t su0 = st3[u0], su1 = st3[u1], sj = st3[t];
  const uint32_t nu1 = (uint32_t)a.n[u1];
  const uint32_t nlines = (uint32_t)a.n[u0] * nu1;
  const int lpb = a.lines_per_block;
  const double rho = a.st->admm_rho;
  for (int j = threadIdx.x; j < n; j += kDhtBlock) {
    double sv, cv;
    sincospi(2.0 * (double)j / (double)n, &sv, &cv);
    const double rn = 1.0 / sqrt((double)n);
    cs[2 * j] = (TR)(cv * rn);
    cs[2 * j + 1] = (TR)(sv * rn);
    if (scale) lt[j] = (2.0 - 2.0 * cospi(2.0 * j / (double)n)) * a.inv_h2[0];
  }
  const bool contig = sj == 1;
  const TR* __restrict__ src = static_cast<const TR*>(a.src);
  const TR* __restrict__ b = static_cast<const TR*>(a.b);
  TR* __restrict__ u = static_cast<TR*>(a.u);
  TR* __restrict__ dst = static_cast<TR*>(a.dst);
  TR* __restrict__ zc = static_cast<TR*>(a.c);
  const TR trho = (TR)rho;
  double acc[2] = {0.0, 0.0};   // final pass: sum (b - z)^2, sum (z - z_old)^2
  for (uint32_t l0 = blockIdx.x * (uint32_t)lpb; l0 < nlines; l0 += gridDim.x * (uint32_t)lpb) {
    const int nl = (int)(nlines - l0 < (uint32_t)lpb ? nlines - l0 : (uint32_t)lpb);
    // element (li, j) of the tile: consecutive threads take consecutive addresses (along the
    // line when it is contiguous, across lines otherwise; e = li + lpb j there, with li >= nl
    // skipped in the last tile)
    auto split = [&](uint32_t e, int& li, int& j) {
      if (contig) {
        li = (int)fdiv(e, a.by_n);
        j = (int)e - li * n;
      } else {
        j = (int)fdiv(e, a.by_lpb);
        li = (int)e - j * lpb;
      }
    };
    auto addr = [&](int li, int j) -> uint32_t {
      const uint32_t L = l0 + (uint32_t)li;
      const uint32_t c0 = fdiv(L, a.by_nu1), c1 = L - c0 * nu1;
      return c0 * su0 + c1 * su1 + (uint32_t)j * sj;
    };
    const uint32_t nel = (uint32_t)(contig ? nl : lpb) * (uint32_t)n;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < nel; e += kDhtBlock) {
      int li, j;
      split(e, li, j);
      if (li >= nl) continue;
      const uint32_t ad = addr(li, j);
      xs[li * ns + j] = a.mode == kDhtFirst ? trho * (b[ad] + u[ad]) : src[ad];
    }
    __syncthreads();
    // the scaling pass's eigenvalue term of the other cross axis for line li (its coordinate
    // there is the line's frequency along that axis)
    auto other_term = [&](int li) -> double {
      const uint32_t L = l0 + (uint32_t)li;
      const uint32_t c0 = fdiv(L, a.by_nu1), c1 = L - c0 * nu1;
      const int ko = (int)(a.other_axis == u0 ? c0 : c1);
      const int no = a.n[a.other_axis];
      return (2.0 - 2.0 * cospi(2.0 * ko / (double)no)) * a.inv_h2[1];
    };
    // output v at position l of line li (lo: other_term(li) in the scaling pass)
    auto emit = [&](int li, int l, TR v, double lo) {
      const uint32_t ad = addr(li, l);
      if (scale) v = (TR)((double)v / (a.alpha * (lt[l] + lo) + rho));
      if (a.mode == kDhtLast) {
        // z_new = v; u <- u + b - z; c = z - u; residual sums
        const TR zo = dst[ad], bv = b[ad];
        const TR un = u[ad] + (bv - v);
        dst[ad] = v;
        u[ad] = un;
        zc[ad] = v - un;
        const double pr = (double)bv - (double)v, du = (double)v - (double)zo;
        acc[0] = fmad64(pr, pr, acc[0]);
        acc[1] = fmad64(du, du, acc[1]);
      } else {
        dst[ad] = v;
      }
    };
    // H x at frequency l is C + S and at n - l it is C - S, with C and S the sums of x_j times
    // cos and sin of 2 pi j l / n: one pass over j serves both frequencies, and the index j l mod n
    // is shared by the kDhtLines lines of a work item
    const int nh = n / 2 + 1;
    const int ngr = (lpb + kDhtLines - 1) / kDhtLines;   // line pairs of a full tile
    const int ngl = (nl + kDhtLines - 1) / kDhtLines;    // of this tile
    for (uint32_t e = threadIdx.x; e < (uint32_t)(ngr * nh); e += kDhtBlock) {
      const int l = (int)fdiv(e, a.by_ngr), gi = (int)e - l * ngr;
      if (gi >= ngl) continue;
      const TR* xl[kDhtLines];
      TR C[kDhtLines], S[kDhtLines];
#pragma unroll
      for (int q = 0; q < kDhtLines; ++q) {
        const int li = gi * kDhtLines + q;
        xl[q] = xs + (li < nl ? li : nl - 1) * ns;   // past the tile: a valid line, not stored
        C[q] = S[q] = TR(0);
      }
      int idx = 0;
      for (int j = 0; j < n; ++j) {
        const TR c = cs[2 * idx], sn = cs[2 * idx + 1];
#pragma unroll
        for (int q = 0; q < kDhtLines; ++q) {
          const TR x = xl[q][j];
          C[q] = fma(x, c, C[q]);
          S[q] = fma(x, sn, S[q]);
        }
        idx += l;
        if (idx >= n) idx -= n;
      }
#pragma unroll
      for (int q = 0; q < kDhtLines; ++q) {
        const int li = gi * kDhtLines + q;
        if (li >= nl) continue;
        const double lo = scale ? other_term(li) : 0.0;
        const int nout = (l > 0 && 2 * l != n) ? 2 : 1;
        for (int o = 0; o < nout; ++o) {
          const int lout = o == 0 ? l : n - l;
          emit(li, lout, o == 0 ? C[q] + S[q] : C[q] - S[q], lo);
        }
      }
    }
  }
  if (a.mode == kDhtLast) store_partials_cm<2, kDhtBlock>(acc, a.part, blockIdx.x);
}

// rho adaptation (one block): primal r = |b - z|, dual s = rho |z - z_old|; rho doubles (u
// halves) when r > 10 s, halves (u doubles) when s > 10 r.  The record of the iteration gets
// the rho it used.
__global__ __launch_bounds__(kReduceBlock) void k_admm_rho(AdmmRhoArgs a) {
  State* st = a.st;
  if (load_flag(&st->gn_stop)) return;
  double t[2];
  load_partials_cm<2>(t, a.part, a.nprod, 2);
  block_sum<2, kReduceBlock>(t);
  if (threadIdx.x == 0) {
    const double rho = st->admm_rho;
    const double r = sqrt(t[0]), s = rho * sqrt(t[1]);
    double f = 1.0;
    if (r > kAdmmMu * s) {
      st->admm_rho = rho * kAdmmTau;
      f = 1.0 / kAdmmTau;
    } else if (s > kAdmmMu * r) {
      st->admm_rho = rho / kAdmmTau;
      f = kAdmmTau;
    }
    st->admm_ufac = f;
    if (a.record) a.record[11] = rho;
  }
}

// u <- f u and c = z - u after an adaptation of rho (f = 1: nothing to do).
template <typename TR>
__global__ __launch_bounds__(kBlock) void k_admm_rescale(AdmmVecArgs a) {
  if (load_flag(&a.st->gn_stop)) return;
  const double f = a.st->admm_ufac;
  if (f == 1.0) return;
  TR* __restrict__ u = static_cast<TR*>(a.u);
  TR* __restrict__ c = static_cast<TR*>(a.c);
  const TR* __restrict__ z = static_cast<const TR*>(a.z);
  const TR tf = (TR)f;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock) {
    const TR un = tf * u[i];
    u[i] = un;
    c[i] = z[i] - un;
  }
}

// Level start: z = b, u = 0, c = b, rho = rho0.
template <typename TR>
__global__ __launch_bounds__(kBlock) void k_admm_init(AdmmVecArgs a) {
  const TR* __restrict__ b = static_cast<const TR*>(a.b);
  TR* __restrict__ u = static_cast<TR*>(a.u);
  TR* __restrict__ c = static_cast<TR*>(a.c);
  TR* __restrict__ z = static_cast<TR*>(a.z);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.st->admm_rho = a.rho0;
    a.st->admm_ufac = 1.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock) {
    const TR bv = b[i];
    z[i] = bv;
    u[i] = TR(0);
    c[i] = bv;
  }
}

unsigned vec_grid(int64_t n) {
  const int64_t b = (n + kBlock * 4 - 1) / (kBlock * 4);
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

// Nodes per lane: the shortest run in kBpRuns whose 16 lanes cover the column (169 nodes take
// 12 per lane, 192 slots, where powers of two alone would take 16, 256 slots).
constexpr int kBpRuns[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
int block_pcg_npl(int mp) {
  const int n = mp + 1;
  for (int npl : kBpRuns)
    if (16 * npl >= n) return npl;
  return 0;
}

unsigned block_pcg_grid(int64_t ncol) {
  const int64_t b = (ncol + kBpColsPerBlock - 1) / kBpColsPerBlock;
  return (unsigned)(b > kMaxGrid ? kMaxGrid : b);
}

hipError_t launch_block_pcg(const BlockPcgArgs& a0, DType real, hipStream_t s) {
  BlockPcgArgs a = a0;
  a.nblk = block_pcg_grid(a.g.ncol);
  if (active_recorder())
    return record_other([a, real](hipStream_t s2) { return launch_block_pcg(a, real, s2); });
  const int npl = block_pcg_npl(a.g.mp);
#define RGP_BP(TR, NPL)                                                                \
  RGP_LAUNCH_T(kKindBlockPcg, a.maxit, a.g, (k_block_pcg<TR, NPL>), a.nblk, kBpBlock, 0, s, a)
#define RGP_BP_T(TR)                           \
  switch (npl) {                               \
    case 1: RGP_BP(TR, 1); break;              \
    case 2: RGP_BP(TR, 2); break;              \
    case 3: RGP_BP(TR, 3); break;              \
    case 4: RGP_BP(TR, 4); break;              \
    case 6: RGP_BP(TR, 6); break;              \
    case 8: RGP_BP(TR, 8); break;              \
    case 12: RGP_BP(TR, 12); break;            \
    case 16: RGP_BP(TR, 16); break;            \
    case 24: RGP_BP(TR, 24); break;            \
    case 32: RGP_BP(TR, 32); break;            \
    default: return hipErrorInvalidValue;      \
  }
  if (real == DType::F64) {
    RGP_BP_T(double);
  } else if (real == DType::F32) {
    RGP_BP_T(float);
  } else {
    return hipErrorInvalidValue;
  }
#undef RGP_BP_T
#undef RGP_BP
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_block_pcg_stats, dim3(1), dim3(kBpBlock), 0, s, a);
  return hipGetLastError();
}

unsigned dht_grid(const int32_t n[3], int axis, int* lines_per_block) {
  const int u0 = axis == 0 ? 1 : 0, u1 = axis == 2 ? 1 : 2;
  const int64_t nlines = (int64_t)n[u0] * n[u1];
  const int lpb = kDhtElems / (n[axis] | 1) < 1 ? 1 : kDhtElems / (n[axis] | 1);
  *lines_per_block = lpb;
  const int64_t b = (nlines + lpb - 1) / lpb;
  return (unsigned)(b > kMaxGrid ? kMaxGrid : b);
}

hipError_t launch_dht(const DhtArgs& a0, DType real, hipStream_t s) {
  DhtArgs a = a0;
  if (a.n[a.axis] > kDhtMaxN) return hipErrorInvalidValue;
  a.nblk = dht_grid(a.n, a.axis, &a.lines_per_block);
  const int u1 = a.axis == 2 ? 1 : 2;
  a.by_n = make_fastdiv((uint32_t)a.n[a.axis]);
  a.by_nu1 = make_fastdiv((uint32_t)a.n[u1]);
  a.by_lpb = make_fastdiv((uint32_t)a.lines_per_block);
  a.by_ngr = make_fastdiv((uint32_t)((a.lines_per_block + kDhtLines - 1) / kDhtLines));
  if (active_recorder())
    return record_other([a, real](hipStream_t s2) { return launch_dht(a, real, s2); });
  const int64_t nodes = (int64_t)a.n[0] * a.n[1] * a.n[2];
  const int tag = a.mode + 4 * a.n[a.axis];
  const int n = a.n[a.axis];
  const size_t e = real == DType::F64 ? 8 : 4;
  const size_t lds = (a.mode == kDhtScale ? (size_t)n * 8 : 0) + (size_t)(2 * n + kDhtElems) * e;
  if (real == DType::F64)
    RGP_LAUNCH_TN(kKindDht, tag, 0, nodes, k_dht<double>, a.nblk, kDhtBlock, lds, s, a);
  else if (real == DType::F32)
    RGP_LAUNCH_TN(kKindDht, tag, 0, nodes, k_dht<float>, a.nblk, kDhtBlock, lds, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_admm_rho(const AdmmRhoArgs& a, hipStream_t s) {
  if (active_recorder())
    return record_other([a](hipStream_t s2) { return launch_admm_rho(a, s2); });
  hipLaunchKernelGGL(k_admm_rho, dim3(1), dim3(kReduceBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_admm_vec(const AdmmVecArgs& a, bool init, DType real, hipStream_t s) {
  if (active_recorder())
    return record_other(
        [a, init, real](hipStream_t s2) { return launch_admm_vec(a, init, real, s2); });
  const unsigned gridn = vec_grid(a.n);
  if (real == DType::F64) {
    if (init)
      hipLaunchKernelGGL(k_admm_init<double>, dim3(gridn), dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL(k_admm_rescale<double>, dim3(gridn), dim3(kBlock), 0, s, a);
  } else if (real == DType::F32) {
    if (init)
      hipLaunchKernelGGL(k_admm_init<float>, dim3(gridn), dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL(k_admm_rescale<float>, dim3(gridn), dim3(kBlock), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rgp
