// Least-squares correction (Sec. 2.4.7): per PE column, the field map defines the push-forward
// matrices M+ and M- that carry the true image to the two distorted inputs (the mass-conserving
// remap of the distortion model: true cell j, between the nodes x_j and x_{j+1}, moves to
// [y_j, y_{j+1}] with y_k = x_k +- b_k, and M(i, j) is its overlap with output cell i divided by
// its moved length), and the corrected image minimises |M+ I - I+|^2 + |M- I - I-|^2.  It is
// found by CGLS from I = 0 (conjugate gradients on the normal equations, Hestenes-Stiefel form).
//
// Columns of up to 512 cells: one wavefront (one workgroup) per column.  Lane l owns the cells
// l*CPL .. l*CPL+CPL-1 (CPL = 1, 2, 3, 4, 6 or 8, the fewest that cover the column) and keeps
// their CGLS vectors in registers; the moved node positions of both
// polarities and the vectors that other lanes read (p, r+, r-) sit in LDS.  M^T r is a gather over
// each owned cell's (at most three) output cells; M p is a gather too: output cell i sums w(i, j) p_j
// over the moved cells j that overlap it, in ascending j - the order in which a scatter over j would
// add them - starting from the first j whose moved interval ends beyond i (a binary search over the
// monotone moved nodes, once per solve).  Each moved cell's overlaps are formed once per solve
// (registers for its own lane, LDS for the others).  Inner products are FP64 (per lane in cell
// order, then across the wavefront in a fixed tree).
// Longer columns: one thread owns one column, its field, iterate and CGLS vectors in LDS for the
// whole solve, laid out [vector][k][thread] so that the lanes of a wavefront touch consecutive
// words whenever they index the same k; every sweep recomputes each moved cell's overlaps from the
// field there.
#include <hip/hip_runtime.h>

#include "rgp_internal.hpp"
#include "rgp_launch.hpp"

namespace rgp {

namespace {

constexpr int kLsqMaxCols = 64;    // columns (threads) per workgroup
constexpr int kLsqLds = 64 * 1024;  // LDS bytes per workgroup

// The overlaps of moved cell j (interval [lo, hi], in cells) with output cells i0, i0+1, i0+2:
// weights w[t] (0 outside the column or without overlap).
template <typename TR>
__device__ __forceinline__ void overlaps(TR lo, TR hi, int m, int& i0, TR (&w)[3]) {
  const TR len = hi - lo;
  const TR fl = floor(lo);
  i0 = (int)fl;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const TR a = fmax(lo, fl + TR(t)), b = fmin(hi, fl + TR(t + 1));
    const int i = i0 + t;
    w[t] = (len > TR(0) && b > a && i >= 0 && i < m) ? (b - a) / len : TR(0);
  }
}

template <typename TI, typename TR>
__global__ __launch_bounds__(kLsqMaxCols) void k_lsq(LsqArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Geom g = a.g;
  const int m = g.mp;
  const int nc = a.cols_per_block;
  const int tid = threadIdx.x;
  const int64_t col = (int64_t)blockIdx.x * nc + tid;
  const bool live = tid < nc && col < g.ncol;
  TR* lds = reinterpret_cast<TR*>(lds_raw);
  // [vector][k][thread]: field b (m + 1 nodes), then x, p, r+, r-, t+, t- (m cells each)
  auto at = [&](int vec, int k) -> TR& {
    const int base = vec == 0 ? 0 : (m + 1) + (vec - 1) * m;
    return lds[(size_t)(base + k) * nc + tid];
  };
  enum { B = 0, X = 1, P = 2, RP = 3, RM = 4, TP = 5, TM = 6 };
  if (!live) return;   // nothing below synchronises the workgroup

  const int ix = (int)(col / g.ny), iy = (int)(col - (int64_t)ix * g.ny);
  const int64_t cb = ix * g.cxs + iy * g.cys, nb = ix * g.nxs + iy * g.nys;
  const TI* __restrict__ Ip = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ Im = static_cast<const TI*>(a.Im);
  const TR* __restrict__ bg = static_cast<const TR*>(a.b);
  const TR inv_hp = TR(1) / (TR)g.hp;
  for (int k = 0; k <= m; ++k) at(B, k) = bg[nb + (int64_t)k * g.nps] * inv_hp;  // in cells
  for (int i = 0; i < m; ++i) {
    at(X, i) = TR(0);
    at(RP, i) = to_real(Ip[cb + (int64_t)i * g.cps], TR());
    at(RM, i) = to_real(Im[cb + (int64_t)i * g.cps], TR());
  }
  // moved interval of cell j for polarity sgn: [j + sgn b_j, j + 1 + sgn b_{j+1}] (cells)
  auto moved = [&](int j, TR sgn, TR& lo, TR& hi) {
    lo = TR(j) + sgn * at(B, j);
    hi = TR(j + 1) + sgn * at(B, j + 1);
  };
  // s = M+^T r+ + M-^T r- into `dst`; returns |s|^2
  auto grad = [&](int dst) -> double {
    double gg = 0.0;
    for (int j = 0; j < m; ++j) {
      TR s = TR(0);
#pragma unroll
      for (int pol = 0; pol < 2; ++pol) {
        const TR sgn = pol == 0 ? TR(1) : TR(-1);
        TR lo, hi, w[3];
        int i0;
        moved(j, sgn, lo, hi);
        overlaps(lo, hi, m, i0, w);
#pragma unroll
        for (int t = 0; t < 3; ++t)
          if (w[t] != TR(0)) s += w[t] * at(pol == 0 ? RP : RM, i0 + t);
      }
      at(dst, j) = s;
      gg += (double)s * (double)s;
    }
    return gg;
  };

  double gam = grad(P);
  const double gam0 = gam;
  int it = 0;
  bool active = gam > 0.0;
  while (active && it < a.maxit) {
    // t = M p (both polarities), delta = |t|^2
    for (int i = 0; i < m; ++i) {
      at(TP, i) = TR(0);
      at(TM, i) = TR(0);
    }
    for (int j = 0; j < m; ++j) {
      const TR pj = at(P, j);
#pragma unroll
      for (int pol = 0; pol < 2; ++pol) {
        const TR sgn = pol == 0 ? TR(1) : TR(-1);
        TR lo, hi, w[3];
        int i0;
        moved(j, sgn, lo, hi);
        overlaps(lo, hi, m, i0, w);
#pragma unroll
        for (int t = 0; t < 3; ++t)
          if (w[t] != TR(0)) at(pol == 0 ? TP : TM, i0 + t) += w[t] * pj;
      }
    }
    double delta = 0.0;
    for (int i = 0; i < m; ++i) {
      const double tp = (double)at(TP, i), tm = (double)at(TM, i);
      delta += tp * tp + tm * tm;
    }
    if (!(delta > 0.0)) break;
    const TR al = (TR)(gam / delta);
    for (int i = 0; i < m; ++i) {
      at(X, i) += al * at(P, i);
      at(RP, i) -= al * at(TP, i);
      at(RM, i) -= al * at(TM, i);
    }
    ++it;
    const double gnew = grad(TP);   // s into TP (free until the next M p)
    if (sqrt(gnew) < a.rtol * sqrt(gam0)) break;
    const TR be = (TR)(gnew / gam);
    for (int j = 0; j < m; ++j) at(P, j) = at(TP, j) + be * at(P, j);
    gam = gnew;
  }

  TI* __restrict__ out = static_cast<TI*>(a.I_out);
  for (int i = 0; i < m; ++i) out[cb + (int64_t)i * g.cps] = from_real<TI>(at(X, i));
  if (a.iters) a.iters[col] = it;
}

// FP64 sum over the 64 lanes of a wavefront in a fixed order (DPP stages; every lane gets it).
__device__ __forceinline__ double wave_sum(double v) {
  double t[1] = {v};
  wave_sums<1>(t);
  return t[0];
}

template <typename TI, typename TR, int CPL>
__global__ __launch_bounds__(kWave) void k_lsq_wave(LsqArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Geom g = a.g;
  const int m = g.mp;
  const int64_t col = blockIdx.x;
  const int lane = threadIdx.x;
  TR* yv[2];
  yv[0] = reinterpret_cast<TR*>(lds_raw);  // moved node positions (cells), + polarity: m + 1
  yv[1] = yv[0] + (m + 1);                 // - polarity
  TR* sp = yv[1] + (m + 1);                // p, read by the lanes that gather it: m
  TR* sr[2] = {sp + m, sp + 2 * m};        // r+, r-: m each
  TR* ww = sp + 3 * m;                     // overlap weights of moved cell j: [pol][j][3]
  int* wi = reinterpret_cast<int*>(ww + 6 * m);   // and its first output cell: [pol][j]

  const int ix = (int)(col / g.ny), iy = (int)(col - (int64_t)ix * g.ny);
  const int64_t cb = ix * g.cxs + iy * g.cys, nb = ix * g.nxs + iy * g.nys;
  const TI* __restrict__ Ip = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ Im = static_cast<const TI*>(a.Im);
  const TR* __restrict__ bg = static_cast<const TR*>(a.b);
  const TR inv_hp = TR(1) / (TR)g.hp;
  for (int k = lane; k <= m; k += kWave) {
    const TR bk = bg[nb + (int64_t)k * g.nps] * inv_hp;   // in cells
    yv[0][k] = TR(k) + bk;
    yv[1][k] = TR(k) - bk;
  }
  const int j0 = lane * CPL;
  TR x[CPL], p[CPL], r[2][CPL], t[2][CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int j = j0 + c;
    const bool own = j < m;
    x[c] = TR(0);
    r[0][c] = own ? to_real(Ip[cb + (int64_t)j * g.cps], TR()) : TR(0);
    r[1][c] = own ? to_real(Im[cb + (int64_t)j * g.cps], TR()) : TR(0);
  }
  __syncthreads();
  // overlaps of the owned moved cells, once per solve: in registers for M^T r, in LDS for the
  // lanes whose output cells they reach (M p)
  TR wo[2][CPL][3];
  int io[2][CPL];
#pragma unroll
  for (int pol = 0; pol < 2; ++pol) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int j = j0 + c;
      io[pol][c] = 0;
      wo[pol][c][0] = wo[pol][c][1] = wo[pol][c][2] = TR(0);
      if (j < m) {
        overlaps(yv[pol][j], yv[pol][j + 1], m, io[pol][c], wo[pol][c]);
        wi[pol * m + j] = io[pol][c];
#pragma unroll
        for (int tt = 0; tt < 3; ++tt) ww[(pol * m + j) * 3 + tt] = wo[pol][c][tt];
      }
    }
  }
  // first moved cell whose interval ends beyond each owned output cell, per polarity
  int jlo[2][CPL];
#pragma unroll
  for (int pol = 0; pol < 2; ++pol) {
    const TR* y = yv[pol];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const TR i = TR(j0 + c);
      int lo = 1, hi = m + 1;   // smallest k in [1, m] with y[k] > i (m + 1: none)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (y[mid] > i) hi = mid; else lo = mid + 1;
      }
      jlo[pol][c] = lo - 1;
    }
  }
  // s = M+^T r+ + M-^T r- for the owned cells (r staged in LDS); returns the wavefront's |s|^2
  auto grad = [&](TR (&s)[CPL]) -> double {
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int j = j0 + c;
      if (j < m) {
        sr[0][j] = r[0][c];
        sr[1][j] = r[1][c];
      }
    }
    __syncthreads();
    double gg = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int j = j0 + c;
      TR acc = TR(0);
      if (j < m) {
#pragma unroll
        for (int pol = 0; pol < 2; ++pol) {
          const int i0 = io[pol][c];
#pragma unroll
          for (int tt = 0; tt < 3; ++tt)
            if (wo[pol][c][tt] != TR(0)) acc += wo[pol][c][tt] * sr[pol][i0 + tt];
        }
      }
      s[c] = acc;
      gg += (double)acc * (double)acc;
    }
    __syncthreads();   // the staging area is rewritten next
    return wave_sum(gg);
  };

  TR s[CPL];
  double gam = grad(s);
  const double gam0 = gam;
#pragma unroll
  for (int c = 0; c < CPL; ++c) p[c] = s[c];
  int it = 0;
  bool active = gam > 0.0;
  while (active && it < a.maxit) {
    // t = M p for the owned output cells (p staged in LDS), delta = |t|^2
#pragma unroll
    for (int c = 0; c < CPL; ++c)
      if (j0 + c < m) sp[j0 + c] = p[c];
    __syncthreads();
    double dl = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int i = j0 + c;
#pragma unroll
      for (int pol = 0; pol < 2; ++pol) {
        TR acc = TR(0);
        if (i < m) {
          const TR* y = yv[pol];
          for (int j = jlo[pol][c]; j < m && y[j] < TR(i + 1); ++j) {
            const int tt = i - wi[pol * m + j];
            const TR wt = (tt >= 0 && tt < 3) ? ww[(pol * m + j) * 3 + tt] : TR(0);
            if (wt != TR(0)) acc += wt * sp[j];
          }
        }
        t[pol][c] = acc;
        dl += (double)acc * (double)acc;
      }
    }
    __syncthreads();
    const double delta = wave_sum(dl);
    if (!(delta > 0.0)) break;
    const TR al = (TR)(gam / delta);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      x[c] += al * p[c];
      r[0][c] -= al * t[0][c];
      r[1][c] -= al * t[1][c];
    }
    ++it;
    const double gnew = grad(s);
    if (sqrt(gnew) < a.rtol * sqrt(gam0)) break;
    const TR be = (TR)(gnew / gam);
#pragma unroll
    for (int c = 0; c < CPL; ++c) p[c] = s[c] + be * p[c];
    gam = gnew;
  }

  TI* __restrict__ out = static_cast<TI*>(a.I_out);
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int j = j0 + c;
    if (j < m) out[cb + (int64_t)j * g.cps] = from_real<TI>(x[c]);
  }
  if (a.iters && lane == 0) a.iters[col] = it;
}

}  // namespace

// Columns per workgroup so that one workgroup's vectors fit kLsqLds bytes (0: a column alone
// does not fit).
int lsq_cols_per_block(int mp, DType real) {
  const size_t per = (size_t)(7 * mp + 1) * (real == DType::F64 ? 8 : 4);
  const size_t n = kLsqLds / per;
  return (int)(n > (size_t)kLsqMaxCols ? kLsqMaxCols : n);
}

hipError_t launch_lsq(const LsqArgs& a0, DType img, DType real, hipStream_t s) {
  const int m = a0.g.mp;
  if (m <= 8 * kWave) {   // one wavefront per column
    const unsigned grid = (unsigned)a0.g.ncol;
    const size_t lds = (size_t)(11 * m + 2) * (real == DType::F64 ? 8 : 4) + (size_t)2 * m * 4;
#define RGP_LSQ_W(CPL)                                                                  \
  RGP_DISPATCH_TYPES(img, real, RGP_LAUNCH(kKindLsq, a0.g, (k_lsq_wave<TI, TR, CPL>), grid, \
                                           kWave, lds, s, a0))
    if (m <= kWave)
      RGP_LSQ_W(1);
    else if (m <= 2 * kWave)
      RGP_LSQ_W(2);
    else if (m <= 3 * kWave)
      RGP_LSQ_W(3);
    else if (m <= 4 * kWave)
      RGP_LSQ_W(4);
    else if (m <= 6 * kWave)
      RGP_LSQ_W(6);
    else
      RGP_LSQ_W(8);
#undef RGP_LSQ_W
    return hipGetLastError();
  }
  LsqArgs a = a0;
  a.cols_per_block = lsq_cols_per_block(a.g.mp, real);
  if (a.cols_per_block < 1) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((a.g.ncol + a.cols_per_block - 1) / a.cols_per_block);
  const size_t lds = (size_t)(7 * a.g.mp + 1) * a.cols_per_block * (real == DType::F64 ? 8 : 4);
  RGP_DISPATCH_TYPES(img, real, RGP_LAUNCH(kKindLsq, a.g, (k_lsq<TI, TR>), grid, kLsqMaxCols,
                                           lds, s, a));
  return hipGetLastError();
}

}  // namespace rgp
