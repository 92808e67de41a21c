// Least-squares correction (Sec. 2.4.7): per PE column, the field map defines the push-forward
// matrices M+ and M- that carry the true image to the two distorted inputs (the mass-conserving
// remap of the distortion model: true cell j, between the nodes x_j and x_{j+1}, moves to
// [y_j, y_{j+1}] with y_k = x_k +- b_k, and M(i, j) is its overlap with output cell i divided by
// its moved length), and the corrected image minimises |M+ I - I+|^2 + |M- I - I-|^2.  It is
// found by CGLS from I = 0 (conjugate gradients on the normal equations, Hestenes-Stiefel form).
//
// One thread owns one column: the field, the iterate and the CGLS vectors of its column live in
// LDS for the whole solve, laid out [vector][k][thread] so that the lanes of a wavefront touch
// consecutive words whenever they index the same k.  The matrices are never stored: every sweep
// recomputes each moved cell's (at most three) overlaps from the field.  Inner products are
// accumulated in FP64.
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

}  // namespace

// Columns per workgroup so that one workgroup's vectors fit kLsqLds bytes (0: a column alone
// does not fit).
int lsq_cols_per_block(int mp, DType real) {
  const size_t per = (size_t)(7 * mp + 1) * (real == DType::F64 ? 8 : 4);
  const size_t n = kLsqLds / per;
  return (int)(n > (size_t)kLsqMaxCols ? kLsqMaxCols : n);
}

hipError_t launch_lsq(const LsqArgs& a0, DType img, DType real, hipStream_t s) {
  LsqArgs a = a0;
  a.cols_per_block = lsq_cols_per_block(a.g.mp, real);
  if (a.cols_per_block < 1) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((a.g.ncol + a.cols_per_block - 1) / a.cols_per_block);
  const size_t lds = (size_t)(7 * a.g.mp + 1) * a.cols_per_block * (real == DType::F64 ? 8 : 4);
  RGP_DISPATCH_TYPES(img, real, hipLaunchKernelGGL((k_lsq<TI, TR>), dim3(grid),
                                                   dim3(kLsqMaxCols), lds, s, a));
  return hipGetLastError();
}

}  // namespace rgp
