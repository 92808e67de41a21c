// Gauss-Newton Hessian-vector products and the Jacobi-preconditioned CG of Sec. 2.3.1.
//
// H v at node k of a column = diag_k v_k + off_{k-1} v_{k-1} + off_k v_{k+1}
//                             - (alpha vol / h_x^2)(v_{x-} + v_{x+}) - (alpha vol / h_y^2)(v_{y-} + v_{y+})
// (existing neighbours only).  diag/off come from loss_grad; diag is also the Jacobi
// preconditioner.
//
// One PCG iteration is one kernel.  Kernel i first reduces the block sums of kernel i-1 (every
// block does it, in block order, so all agree bitwise) to get a_{i-1} = r.z / p.w and the next
// r^T z and r^T r from the recurrences r'.z' = r.z - 2a r.w/d + a^2 w.w/d and
// r'.r' = r.r - 2a r.w + a^2 w.w (Chronopoulos-Gear), so one grid-wide reduction per iteration
// suffices and no kernel needs atomics or fences.  It then applies the update pointwise
// (x += a p, r -= a w, p = r/d + b p), recomputing p at the stencil halo from the previous
// vectors (which therefore live in ping-pong buffers), forms w = H p and stores its block sums of
// p.w, r.w/d, w.w/d, r.w and w.w.  In exact arithmetic the iterates are those of textbook PCG.
#include "rgp_internal.hpp"
#include "rgp_launch.hpp"
#include "rgp_solver.hpp"

namespace rgp {

namespace {
constexpr int kRun = 8;
}

template <typename TR, int S, int BLK>
__global__ __launch_bounds__(BLK) void k_hvp(HvpArgs a) {
  const Geom g = a.g;
  const TR* __restrict__ dg = static_cast<const TR*>(a.diag);
  const TR* __restrict__ of = static_cast<const TR*>(a.off);
  const TR* __restrict__ v = static_cast<const TR*>(a.v);
  TR* __restrict__ Hv = static_cast<TR*>(a.Hv);
  const int mp = g.mp;
  const int64_t nct = (g.ncol + kWave - 1) / kWave;
  const int64_t ntiles = nct * ((mp + 1 + S - 1) / S);
  const int lane = threadIdx.x & (kWave - 1);
  const TR cx = (TR)(a.alpha * g.vol / (g.hx * g.hx));
  const TR cy = (TR)(a.alpha * g.vol / (g.hy * g.hy));
  double acc[1] = {0.0};
  for (WaveIter it = wave_iter(ntiles); it.t < it.end; it.t += it.stride) {
    const int64_t col = (it.t % nct) * kWave + lane;
    const int k0 = (int)(it.t / nct) * S;
    const bool colok = col < g.ncol;
    const int64_t colc = colok ? col : g.ncol - 1;
    const int64_t ix = colc / g.ny, iy = colc - (colc / g.ny) * g.ny;
    const int64_t nb = ix * g.nxs + iy * g.nys;
    const bool hasxm = ix > 0, hasxp = ix < g.nx - 1, hasym = iy > 0, hasyp = iy < g.ny - 1;
    TR vv[S + 2], oo[S + 1];
#pragma unroll
    for (int i = 0; i < S + 2; ++i) {
      int k = k0 - 1 + i;
      k = k < 0 ? 0 : (k > mp ? mp : k);
      vv[i] = v[nb + (int64_t)k * g.nps];
      if (i < S + 1) oo[i] = of[nb + (int64_t)k * g.nps];
    }
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
      TR crx = TR(0), cry = TR(0);
      if (hasxm) crx += v[n - g.nxs];
      if (hasxp) crx += v[n + g.nxs];
      if (hasym) cry += vym;
      if (hasyp) cry += vyp;
      h -= cx * crx + cy * cry;
      if (nodeok && colok) {
        Hv[n] = h;
        acc[0] += (double)vk * (double)h;
      }
    }
  }
  if (a.part) store_partials<1>(acc, a.part);
}

// out = sum of one slot of block sums (one block).
__global__ __launch_bounds__(kBlock) void k_sum_final(const double* part, unsigned nprod,
                                                      double* out) {
  double t[1];
  reduce_partials<1>(t, part, nprod);
  if (threadIdx.x == 0) *out = t[0];
}

template <typename TR, int S, int BLK>
__global__ __launch_bounds__(BLK) void k_pcg_step(PcgArgs a) {
  State* st = a.st;
  const int it_ = a.iter;
  const bool first = it_ == 0;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;

  // ---- scalar phase: the recurrence of iteration it_-1 (identical in every block) ----------
  TR al = TR(0), be = TR(0);
  bool finish = false;
  if (first) {
    if (a.gn_mode) {
      if (load_flag(&st->gn_stop)) return;
      // J, D, S, P of the current iterate (loss_grad's block sums); stop on a violated barrier.
      if (finalize_loss(a.lf, blockIdx.x == 0)) return;
    }
  } else {
    if (a.gn_mode && load_flag(&st->gn_stop)) return;
    const PcgSlot prev = a.slots[(it_ - 1) & 1];
    PcgSlot cur = prev;
    if (prev.status == kPcgDone) {  // carry the final slot forward
      if (lead) {
        a.slots[it_ & 1] = prev;
        if (it_ == a.maxit) {
          st->pcg_iters = prev.iters;
          st->relres = prev.relres;
          if (a.iters_out) *a.iters_out = prev.iters;
          if (a.relres_out) *a.relres_out = prev.relres;
        }
      }
      return;
    }
    double t[7];
    reduce_partials<7>(t, a.part_prev, a.nprod);
    double rz = prev.rz, rr = prev.rr, bn = prev.bnorm2;
    if (it_ == 1) {
      rz = t[5];
      rr = t[6];
      bn = t[6];
    }
    const double pw = t[0];
    bool done = false;
    if (!(bn > 0.0) || !(pw > 0.0)) {  // zero right-hand side or p^T H p <= 0: keep x
      cur.status = kPcgDone;
      cur.iters = it_ - 1;
      cur.relres = it_ == 1 ? (bn > 0.0 ? 1.0 : 0.0) : prev.relres;
      cur.bnorm2 = bn;
      done = true;
    } else {
      const double a2 = rz / pw;
      const double rzn = rz - 2.0 * a2 * t[1] + a2 * a2 * t[2];
      const double rrn = rr - 2.0 * a2 * t[3] + a2 * a2 * t[4];
      al = (TR)a2;
      be = (TR)(rzn / rz);
      cur.rz = rzn;
      cur.rr = rrn;
      cur.bnorm2 = bn;
      cur.iters = it_;
      cur.relres = sqrt(fmax(rrn, 0.0) / bn);
      finish = cur.relres < a.rtol || it_ >= a.maxit;
      cur.status = finish ? kPcgDone : kPcgRunning;
    }
    if (lead) {
      a.slots[it_ & 1] = cur;
      if (done || finish) {
        st->pcg_iters = cur.iters;
        st->relres = cur.relres;
        if (a.iters_out) *a.iters_out = cur.iters;
        if (a.relres_out) *a.relres_out = cur.relres;
      }
    }
    if (done) return;
  }

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
  const int mp = g.mp;
  const int64_t nct = (g.ncol + kWave - 1) / kWave;
  const int64_t ntiles = nct * ((mp + 1 + S - 1) / S);
  const int lane = threadIdx.x & (kWave - 1);

  if (finish) {  // last update x += a p of the previous iteration, then stop
    for (WaveIter it = wave_iter(ntiles); it.t < it.end; it.t += it.stride) {
      const int64_t col = (it.t % nct) * kWave + lane;
      const int k0 = (int)(it.t / nct) * S;
      if (col >= g.ncol) continue;
      const int64_t nb = node_base(g, col);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int k = k0 + s;
        if (k <= mp) {
          const int64_t n = nb + (int64_t)k * g.nps;
          x[n] = x[n] + al * pi[n];
        }
      }
    }
    return;
  }

  // Updated search direction at an arbitrary node (same arithmetic as for owned nodes).
  auto pnew = [&](int64_t n) -> TR {
    if (first) return sgn * rhs[n] / dg[n];
    const TR r = ri[n] - al * wi[n];
    return r / dg[n] + be * pi[n];
  };
  const TR cx = (TR)(a.alpha * g.vol / (g.hx * g.hx));
  const TR cy = (TR)(a.alpha * g.vol / (g.hy * g.hy));

  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (WaveIter it = wave_iter(ntiles); it.t < it.end; it.t += it.stride) {
    const int64_t col = (it.t % nct) * kWave + lane;
    const int k0 = (int)(it.t / nct) * S;
    const bool colok = col < g.ncol;
    const int64_t colc = colok ? col : g.ncol - 1;
    const int64_t ix = colc / g.ny, iy = colc - (colc / g.ny) * g.ny;
    const int64_t nb = ix * g.nxs + iy * g.nys;
    const bool hasxm = ix > 0, hasxp = ix < g.nx - 1, hasym = iy > 0, hasyp = iy < g.ny - 1;

    // p at nodes k0-1 .. k0+S (index i <-> node k0-1+i), off at k0-1 .. k0+S-1.
    TR pp[S + 2], oo[S + 1];
#pragma unroll
    for (int i = 0; i < S + 2; ++i) {
      int k = k0 - 1 + i;
      k = k < 0 ? 0 : (k > mp ? mp : k);
      const int64_t n = nb + (int64_t)k * g.nps;
      if (i == 0 || i == S + 1) pp[i] = pnew(n);
      if (i < S + 1) oo[i] = of[n];
    }
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
  }
  store_partials<7>(acc, a.part);
  if (first && lead) {
    PcgSlot s0{};
    s0.status = kPcgRunning;
    a.slots[0] = s0;
  }
}

Launch plan_hvp(const Geom& g, DType real) {
  return plan_tiles(g, kRun, (real == DType::F32 && plan_tiles(g, kRun, 256).ntiles > 1024) ? 1024 : 256);
}
Launch plan_pcg(const Geom& g, DType real) { return plan_hvp(g, real); }

hipError_t launch_hvp(const HvpArgs& a, DType real, hipStream_t s) {
  const Launch L = plan_hvp(a.g, real);
  if (real == DType::F64)
    hipLaunchKernelGGL((k_hvp<double, kRun, 256>), dim3(L.grid), dim3(256), 0, s, a);
  else if (L.block == 1024)
    hipLaunchKernelGGL((k_hvp<float, kRun, 1024>), dim3(L.grid), dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL((k_hvp<float, kRun, 256>), dim3(L.grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sum_final(const double* part, unsigned nprod, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, part, nprod, out);
  return hipGetLastError();
}

hipError_t launch_pcg_step(const PcgArgs& a, DType real, hipStream_t s) {
  const Launch L = plan_pcg(a.g, real);
  if (L.grid != a.nprod) return hipErrorInvalidValue;
  if (real == DType::F64)
    hipLaunchKernelGGL((k_pcg_step<double, kRun, 256>), dim3(L.grid), dim3(256), 0, s, a);
  else if (L.block == 1024)
    hipLaunchKernelGGL((k_pcg_step<float, kRun, 1024>), dim3(L.grid), dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL((k_pcg_step<float, kRun, 256>), dim3(L.grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace rgp
