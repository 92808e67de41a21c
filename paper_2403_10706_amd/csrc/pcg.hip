// Gauss-Newton Hessian-vector products and the Jacobi-preconditioned CG of Sec. 2.3.1.
//
// H v at node k of a column = diag_k v_k + off_{k-1} v_{k-1} + off_k v_{k+1}
//                             - (alpha vol / h_x^2)(v_{x-} + v_{x+}) - (alpha vol / h_y^2)(v_{y-} + v_{y+})
// (existing neighbours only).  diag/off come from loss_grad; diag is also the Jacobi
// preconditioner.
//
// One PCG iteration is one kernel.  It first applies the update of the previous iteration
// pointwise (x += a p, r -= a w, p = r/d + b p), recomputing p at the stencil halo from the
// previous vectors (which therefore live in ping-pong buffers), then forms w = H p and the five
// FP64 inner products p.w, r.w/d, w.w/d, r.w, w.w.  The next r^T z and r^T r follow from the
// recurrences r'.z' = r.z - 2a r.w/d + a^2 w.w/d and r'.r' = r.r - 2a r.w + a^2 w.w
// (Chronopoulos-Gear), so one grid-wide reduction per iteration suffices.  In exact arithmetic
// the iterates are those of textbook PCG.
#include "rgp_internal.hpp"
#include "rgp_launch.hpp"

namespace rgp {

namespace {
constexpr int kRun = 8;
}

template <typename TR, int S>
__global__ __launch_bounds__(kBlock) void k_hvp(HvpArgs a) {
  const Geom g = a.g;
  const TR* __restrict__ dg = static_cast<const TR*>(a.diag);
  const TR* __restrict__ of = static_cast<const TR*>(a.off);
  const TR* __restrict__ v = static_cast<const TR*>(a.v);
  TR* __restrict__ Hv = static_cast<TR*>(a.Hv);
  const unsigned nblocks = gridDim.x;
  const unsigned bid = xcd_remap(blockIdx.x, nblocks);
  const int64_t nct = (g.ncol + kWave - 1) / kWave;
  const int64_t coltile = bid % nct;
  const int64_t petile = bid / nct;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int64_t col = coltile * kWave + lane;
  const bool colok = col < g.ncol;
  const int64_t colc = colok ? col : g.ncol - 1;
  const int64_t ix = colc / g.ny, iy = colc - (colc / g.ny) * g.ny;
  const int k0 = (int)((petile * kWaves + wv) * S);
  const int mp = g.mp;
  const int64_t nb = ix * g.nxs + iy * g.nys;
  const TR cx = (TR)(a.alpha * g.vol / (g.hx * g.hx));
  const TR cy = (TR)(a.alpha * g.vol / (g.hy * g.hy));
  const bool hasxm = ix > 0, hasxp = ix < g.nx - 1, hasym = iy > 0, hasyp = iy < g.ny - 1;

  TR vv[S + 2], oo[S + 1];
#pragma unroll
  for (int i = 0; i < S + 2; ++i) {
    int k = k0 - 1 + i;
    k = k < 0 ? 0 : (k > mp ? mp : k);
    vv[i] = v[nb + (int64_t)k * g.nps];
    if (i < S + 1) oo[i] = of[nb + (int64_t)k * g.nps];
  }
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int k = k0 + s;
    const bool nodeok = k <= mp;
    const int kc = nodeok ? k : mp;
    const int64_t n = nb + (int64_t)kc * g.nps;
    const TR vk = vv[s + 1];
    TR vym = __shfl_up(vk, 1, kWave);
    TR vyp = __shfl_down(vk, 1, kWave);
    if (lane == 0 && hasym) vym = v[n - g.nys];
    if (lane == kWave - 1 && hasyp) vyp = v[n + g.nys];
    TR h = dg[n] * vk;
    if (k > 0) h += oo[s] * vv[s];
    if (k < mp) h += oo[s + 1] * vv[s + 2];
    TR cross = TR(0);
    if (hasxm) cross += v[n - g.nxs];
    if (hasxp) cross += v[n + g.nxs];
    h -= cx * cross;
    TR crossy = TR(0);
    if (hasym) crossy += vym;
    if (hasyp) crossy += vyp;
    h -= cy * crossy;
    if (nodeok && colok) {
      Hv[n] = h;
      acc += (double)vk * (double)h;
    }
  }
  double part[1] = {acc};
  if (publish_partials<1>(part, a.partials, a.counter, bid, nblocks)) {
    double t[1];
    reduce_partials<1>(t, a.partials, nblocks);
    if (threadIdx.x == 0) {
      if (a.vHv) *a.vHv = t[0];
      *a.counter = 0u;
    }
  }
}

template <typename TR, int S>
__global__ __launch_bounds__(kBlock) void k_pcg_step(PcgArgs a) {
  State* st = a.st;
  if (a.gn_mode && st->gn_stop) return;
  const int status = st->pcg_status;
  if (status == kPcgDone) return;
  const bool first = a.iter == 0;
  const bool finishing = status == kPcgFinish;
  const TR al = (TR)st->alpha, be = (TR)st->beta;

  const Geom g = a.g;
  const TR* __restrict__ dg = static_cast<const TR*>(a.diag);
  const TR* __restrict__ of = static_cast<const TR*>(a.off);
  const TR* __restrict__ rhs = static_cast<const TR*>(a.rhs);
  TR* __restrict__ x = static_cast<TR*>(a.x);
  const TR* __restrict__ ri = static_cast<const TR*>(a.r_in);
  const TR* __restrict__ pi = static_cast<const TR*>(a.p_in);
  const TR* __restrict__ wi = static_cast<const TR*>(a.w_in);
  TR* __restrict__ ro = static_cast<TR*>(a.r_out);
  TR* __restrict__ po = static_cast<TR*>(a.p_out);
  TR* __restrict__ wo = static_cast<TR*>(a.w_out);
  const TR sgn = (TR)a.rhs_sign;

  const unsigned nblocks = gridDim.x;
  const unsigned bid = xcd_remap(blockIdx.x, nblocks);
  const int64_t nct = (g.ncol + kWave - 1) / kWave;
  const int64_t coltile = bid % nct;
  const int64_t petile = bid / nct;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int64_t col = coltile * kWave + lane;
  const bool colok = col < g.ncol;
  const int64_t colc = colok ? col : g.ncol - 1;
  const int64_t ix = colc / g.ny, iy = colc - (colc / g.ny) * g.ny;
  const int k0 = (int)((petile * kWaves + wv) * S);
  const int mp = g.mp;
  const int64_t nb = ix * g.nxs + iy * g.nys;

  // Updated search direction at an arbitrary node (same arithmetic as for owned nodes).
  auto pnew = [&](int64_t n) -> TR {
    if (first) return sgn * rhs[n] / dg[n];
    const TR r = ri[n] - al * wi[n];
    return r / dg[n] + be * pi[n];
  };

  if (finishing) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int k = k0 + s;
      if (colok && k <= mp) {
        const int64_t n = nb + (int64_t)k * g.nps;
        x[n] = x[n] + al * pi[n];
      }
    }
    double dummy[1] = {0.0};
    if (publish_partials<1>(dummy, a.partials, a.counter, bid, nblocks)) {
      if (threadIdx.x == 0) {
        st->pcg_status = kPcgDone;
        if (a.iters_out) *a.iters_out = st->pcg_iters;
        if (a.relres_out) *a.relres_out = st->relres;
        *a.counter = 0u;
      }
    }
    return;
  }

  const TR cx = (TR)(a.alpha * g.vol / (g.hx * g.hx));
  const TR cy = (TR)(a.alpha * g.vol / (g.hy * g.hy));
  const bool hasxm = ix > 0, hasxp = ix < g.nx - 1, hasym = iy > 0, hasyp = iy < g.ny - 1;

  // p at nodes k0-1 .. k0+S (index i <-> node k0-1+i), off at k0-1 .. k0+S-1.
  TR pp[S + 2], oo[S + 1];
#pragma unroll
  for (int i = 0; i < S + 2; ++i) {
    int k = k0 - 1 + i;
    k = k < 0 ? 0 : (k > mp ? mp : k);
    const int64_t n = nb + (int64_t)k * g.nps;
    if (i == 0 || i == S + 1) {
      pp[i] = pnew(n);
    }
    if (i < S + 1) oo[i] = of[n];
  }
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  TR rl[S], dl[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int k = k0 + s;
    const bool nodeok = k <= mp;
    const int kc = nodeok ? k : mp;
    const int64_t n = nb + (int64_t)kc * g.nps;
    const TR d = dg[n];
    TR r, xn, p;
    if (first) {
      r = sgn * rhs[n];
      xn = TR(0);
      p = r / d;
    } else {
      const TR pold = pi[n];
      r = ri[n] - al * wi[n];
      xn = x[n] + al * pold;
      p = r / d + be * pold;
    }
    pp[s + 1] = p;
    rl[s] = r;
    dl[s] = d;
    if (nodeok && colok) {
      x[n] = xn;
      ro[n] = r;
      po[n] = p;
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int k = k0 + s;
    const bool nodeok = k <= mp;
    const int kc = nodeok ? k : mp;
    const int64_t n = nb + (int64_t)kc * g.nps;
    const TR pk = pp[s + 1];
    TR pym = __shfl_up(pk, 1, kWave);
    TR pyp = __shfl_down(pk, 1, kWave);
    if (lane == 0 && hasym) pym = pnew(n - g.nys);
    if (lane == kWave - 1 && hasyp) pyp = pnew(n + g.nys);
    const TR d = dl[s];
    TR w = d * pk;
    if (k > 0) w += oo[s] * pp[s];
    if (k < mp) w += oo[s + 1] * pp[s + 2];
    TR crx = TR(0);
    if (hasxm) crx += pnew(n - g.nxs);
    if (hasxp) crx += pnew(n + g.nxs);
    TR cry = TR(0);
    if (hasym) cry += pym;
    if (hasyp) cry += pyp;
    w -= cx * crx + cy * cry;
    if (nodeok && colok) {
      wo[n] = w;
      const double rr = (double)rl[s];
      const double ww = (double)w, dd = (double)d;
      acc[0] += (double)pk * ww;
      acc[1] += rr * ww / dd;
      acc[2] += ww * ww / dd;
      acc[3] += rr * ww;
      acc[4] += ww * ww;
      if (first) {
        acc[5] += rr * rr / dd;
        acc[6] += rr * rr;
      }
    }
  }
  if (publish_partials<7>(acc, a.partials, a.counter, bid, nblocks)) {
    double t[7];
    reduce_partials<7>(t, a.partials, nblocks);
    if (threadIdx.x == 0) {
      if (first) {
        st->rz = t[5];
        st->rr = t[6];
        st->bnorm2 = t[6];
        st->relres = t[6] > 0.0 ? 1.0 : 0.0;
      }
      const double pw = t[0];
      if (!(st->bnorm2 > 0.0) || !(pw > 0.0)) {
        // zero right-hand side or p^T H p <= 0: stop with the current x
        st->pcg_status = kPcgDone;
        st->pcg_iters = a.iter;
        if (a.iters_out) *a.iters_out = a.iter;
        if (a.relres_out) *a.relres_out = st->relres;
      } else {
        const double rz = st->rz;
        const double al2 = rz / pw;
        const double rzn = rz - 2.0 * al2 * t[1] + al2 * al2 * t[2];
        const double rrn = st->rr - 2.0 * al2 * t[3] + al2 * al2 * t[4];
        st->alpha = al2;
        st->beta = rzn / rz;
        st->rz = rzn;
        st->rr = rrn;
        st->pcg_iters = a.iter + 1;
        st->relres = sqrt(fmax(rrn, 0.0) / st->bnorm2);
        if (st->relres < a.rtol || a.iter + 1 >= a.maxit) st->pcg_status = kPcgFinish;
      }
      *a.counter = 0u;
    }
  }
}

unsigned hvp_blocks(const Geom& g) {
  const int64_t nct = (g.ncol + kWave - 1) / kWave;
  const int64_t npt = (g.mp + 1 + kWaves * kRun - 1) / (kWaves * kRun);
  return (unsigned)(nct * npt);
}
unsigned pcg_blocks(const Geom& g) { return hvp_blocks(g); }

hipError_t launch_hvp(const HvpArgs& a, DType real, hipStream_t s) {
  const unsigned nb = hvp_blocks(a.g);
  if (real == DType::F64)
    hipLaunchKernelGGL((k_hvp<double, kRun>), dim3(nb), dim3(kBlock), 0, s, a);
  else if (real == DType::F32)
    hipLaunchKernelGGL((k_hvp<float, kRun>), dim3(nb), dim3(kBlock), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_pcg_step(const PcgArgs& a, DType real, hipStream_t s) {
  const unsigned nb = pcg_blocks(a.g);
  if (real == DType::F64)
    hipLaunchKernelGGL((k_pcg_step<double, kRun>), dim3(nb), dim3(kBlock), 0, s, a);
  else if (real == DType::F32)
    hipLaunchKernelGGL((k_pcg_step<float, kRun>), dim3(nb), dim3(kBlock), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace rgp
