// Gauss-Newton Hessian-vector products and the Jacobi-preconditioned CG of Sec. 2.3.1.
//
// H v at node k of a column = diag_k v_k + off_{k-1} v_{k-1} + off_k v_{k+1}
//                             - (alpha vol / h_x^2)(v_{x-} + v_{x+}) - (alpha vol / h_y^2)(v_{y-} + v_{y+})
// (existing neighbours only).  diag/off come from loss_grad; diag is also the Jacobi
// preconditioner.
//
// One PCG iteration is two kernels.  A single-block scalar kernel reduces the block sums of
// iteration i-1 in block order (bitwise reproducible) to a_{i-1} = r.z / p.w and the next r^T z
// and r^T r from the recurrences r'.z' = r.z - 2a r.w/d + a^2 w.w/d and
// r'.r' = r.r - 2a r.w + a^2 w.w (Chronopoulos-Gear), so one grid-wide reduction per iteration
// suffices and nothing needs atomics or fences.  The main kernel then applies the update
// pointwise (x += a p, r -= a w, p = r/d + b p), recomputing p at the stencil halo from the
// previous vectors (which therefore live in ping-pong buffers), forms w = H p and stores its
// block sums of p.w, r.w/d, w.w/d, r.w and w.w.  In exact arithmetic the iterates are those of
// textbook PCG.
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

// Tiling of the PCG step: a wavefront owns a slab of X consecutive x-rows, a chunk of 64
// consecutive y columns (one per lane) and a run of S consecutive PE nodes, and marches along x:
// the p values of the rows x-1, x and x+1 stay in registers, y neighbours come from lane
// shuffles, and only the slab's outer rows (and the PE run ends) are recomputed from the previous
// vectors.
struct SlabTiles {
  int nslab, nchunk, nrun;
  int64_t ntiles;
};
__host__ __device__ inline SlabTiles slab_tiles(const Geom& g, int S, int X) {
  SlabTiles T;
  T.nslab = (g.nx + X - 1) / X;
  T.nchunk = (g.ny + kWave - 1) / kWave;
  T.nrun = (g.mp + 1 + S - 1) / S;
  T.ntiles = (int64_t)T.nslab * T.nchunk * T.nrun;
  return T;
}

// ---- scalar phase of iteration `iter` (one block) ------------------------------------------
__global__ __launch_bounds__(kBlock) void k_pcg_scalars(PcgScalarArgs a) {
  State* st = a.st;
  const int it_ = a.iter;
  const bool lead = threadIdx.x == 0;
  auto finish_outputs = [&](const PcgSlot& c) {
    st->pcg_iters = c.iters;
    st->relres = c.relres;
    if (a.iters_out) *a.iters_out = c.iters;
    if (a.relres_out) *a.relres_out = c.relres;
  };
  if (a.gn_mode && load_flag(&st->gn_stop)) {
    if (lead) {
      PcgSlot d{};
      d.status = kPcgDone;
      a.slots[it_ & 1] = d;
    }
    return;
  }
  if (it_ == 0) {
    bool viol = false;
    // J, D, S, P of the current iterate; a violated barrier stops the GN solve on this level.
    if (a.gn_mode) viol = finalize_loss(a.lf, true);
    if (lead) {
      PcgSlot s0{};
      s0.status = viol ? kPcgDone : kPcgRunning;
      a.slots[0] = s0;
    }
    return;
  }
  const PcgSlot prev = a.slots[(it_ - 1) & 1];
  if (prev.status != kPcgRunning) {  // the solve has ended: carry the final slot forward
    if (lead) {
      PcgSlot c = prev;
      c.status = kPcgDone;
      a.slots[it_ & 1] = c;
      if (it_ == a.maxit) finish_outputs(c);
    }
    return;
  }
  double t[7];
  reduce_partials<7>(t, a.part_prev, a.nprod);
  if (!lead) return;
  PcgSlot cur = prev;
  double rz = prev.rz, rr = prev.rr, bn = prev.bnorm2;
  if (it_ == 1) {
    rz = t[5];
    rr = t[6];
    bn = t[6];
  }
  const double pw = t[0];
  cur.bnorm2 = bn;
  if (!(bn > 0.0) || !(pw > 0.0)) {  // zero right-hand side or p^T H p <= 0: keep x
    cur.status = kPcgDone;
    cur.iters = it_ - 1;
    cur.relres = it_ == 1 ? (bn > 0.0 ? 1.0 : 0.0) : prev.relres;
    finish_outputs(cur);
  } else {
    const double a2 = rz / pw;
    const double rzn = rz - 2.0 * a2 * t[1] + a2 * a2 * t[2];
    const double rrn = rr - 2.0 * a2 * t[3] + a2 * a2 * t[4];
    cur.alpha = a2;
    cur.beta = rzn / rz;
    cur.rz = rzn;
    cur.rr = rrn;
    cur.iters = it_;
    cur.relres = sqrt(fmax(rrn, 0.0) / bn);
    const bool finish = cur.relres < a.rtol || it_ >= a.maxit;
    cur.status = finish ? kPcgFinish : kPcgRunning;
    if (finish) finish_outputs(cur);
  }
  a.slots[it_ & 1] = cur;
}

// ---- main phase of iteration `iter`: update, w = H p, block sums ---------------------------
template <typename TR, int S, int X, int BLK>
__global__ __launch_bounds__(BLK) void k_pcg_step(PcgArgs a) {
  const PcgSlot sl = *a.slot;
  if (sl.status == kPcgDone) return;
  const int it_ = a.iter;
  const bool first = it_ == 0;
  const TR al = (TR)sl.alpha, be = (TR)sl.beta;

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

  if (sl.status == kPcgFinish) {  // last update x += a p of the previous iteration (pointwise)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.nnode; i += stride)
      x[i] = x[i] + al * pi[i];
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
  const int lane = threadIdx.x & (kWave - 1);
  const SlabTiles T = slab_tiles(g, S, X);

  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (WaveIter it = wave_iter(T.ntiles); it.t < it.end; it.t += it.stride) {
    const int chunk = (int)(it.t % T.nchunk);
    const int64_t rest = it.t / T.nchunk;
    const int run = (int)(rest % T.nrun);
    const int slab = (int)(rest / T.nrun);
    const int iy = chunk * kWave + lane;
    const bool yok = iy < g.ny;
    const int64_t iyc = yok ? iy : g.ny - 1;
    const bool hasym = iyc > 0, hasyp = iyc < g.ny - 1;
    const int k0 = run * S;
    const int ix0 = slab * X;
    const int nrow = min(X, g.nx - ix0);
    const int64_t ybase = iyc * g.nys;

    // Own update of row ix: x, r, p at the S owned nodes (stored), p at the two PE halo nodes.
    auto own_row = [&](int ix, TR (&P)[S + 2], TR (&D)[S], TR (&R)[S]) {
      const int64_t base = (int64_t)ix * g.nxs + ybase;
#pragma unroll
      for (int i = 0; i < S + 2; ++i) {
        int k = k0 - 1 + i;
        const bool own = i >= 1 && i <= S;
        const bool nodeok = k >= 0 && k <= mp;
        k = k < 0 ? 0 : (k > mp ? mp : k);
        const int64_t n = base + (int64_t)k * g.nps;
        if (!own) {
          P[i] = pnew(n);
          continue;
        }
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
        P[i] = p;
        D[i - 1] = d;
        R[i - 1] = r;
        if (nodeok && yok) {
          x[n] = xn;
          ro[n] = r;
          po[n] = p;
        }
      }
    };
    // p of a neighbouring row outside the slab (owned nodes only).
    auto halo_row = [&](int ix, TR (&P)[S + 2]) {
      const int64_t base = (int64_t)ix * g.nxs + ybase;
#pragma unroll
      for (int i = 1; i <= S; ++i) {
        int k = k0 - 1 + i;
        k = k > mp ? mp : k;
        P[i] = pnew(base + (int64_t)k * g.nps);
      }
    };

    TR Pm[S + 2], Pc[S + 2], Pn[S + 2];
    TR Dc[S], Rc[S], Dn[S], Rn[S];
#pragma unroll
    for (int i = 0; i < S + 2; ++i) Pm[i] = Pc[i] = Pn[i] = TR(0);
#pragma unroll
    for (int i = 0; i < S; ++i) Dn[i] = Rn[i] = TR(1);
    if (ix0 > 0) halo_row(ix0 - 1, Pm);
    own_row(ix0, Pc, Dc, Rc);
#pragma unroll
    for (int j = 0; j < X; ++j) {
      if (j >= nrow) break;
      const int ix = ix0 + j;
      const bool hasxm = ix > 0, hasxp = ix + 1 < g.nx;
      if (j + 1 < nrow) {
        own_row(ix + 1, Pn, Dn, Rn);
      } else if (hasxp) {
        halo_row(ix + 1, Pn);
      }
      const int64_t base = (int64_t)ix * g.nxs + ybase;
      // off at nodes k0-1 .. k0+S-1
      TR oo[S + 1];
#pragma unroll
      for (int i = 0; i < S + 1; ++i) {
        int k = k0 - 1 + i;
        k = k < 0 ? 0 : (k > mp ? mp : k);
        oo[i] = of[base + (int64_t)k * g.nps];
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int k = k0 + s;
        const bool nodeok = k <= mp;
        const int kc = nodeok ? k : mp;
        const int64_t n = base + (int64_t)kc * g.nps;
        const TR pk = Pc[s + 1];
        TR pym = __shfl_up(pk, 1, kWave);
        TR pyp = __shfl_down(pk, 1, kWave);
        if (lane == 0 && hasym) pym = pnew(n - g.nys);
        if (lane == kWave - 1 && hasyp) pyp = pnew(n + g.nys);
        const TR d = Dc[s];
        TR w = d * pk;
        if (k > 0) w += oo[s] * Pc[s];
        if (k < mp) w += oo[s + 1] * Pc[s + 2];
        TR crx = TR(0), cry = TR(0);
        if (hasxm) crx += Pm[s + 1];
        if (hasxp) crx += Pn[s + 1];
        if (hasym) cry += pym;
        if (hasyp) cry += pyp;
        w -= cx * crx + cy * cry;
        if (nodeok && yok) {
          wo[n] = w;
          // FP64 products and sums; one reciprocal of the diagonal per node
          const double r = (double)Rc[s], ww = (double)w, id = (double)(TR(1) / d);
          const double wd = ww * id;
          acc[0] += (double)pk * ww;
          acc[1] += r * wd;
          acc[2] += ww * wd;
          acc[3] += r * ww;
          acc[4] += ww * ww;
          if (first) {
            acc[5] += r * r * id;
            acc[6] += r * r;
          }
        }
      }
#pragma unroll
      for (int i = 0; i < S + 2; ++i) {
        Pm[i] = Pc[i];
        Pc[i] = Pn[i];
      }
#pragma unroll
      for (int i = 0; i < S; ++i) {
        Dc[i] = Dn[i];
        Rc[i] = Rn[i];
      }
    }
  }
  store_partials<7>(acc, a.part);
}

Launch plan_hvp(const Geom& g, DType real) {
  return plan_tiles(g, kRun, (real == DType::F32 && plan_tiles(g, kRun, 256).ntiles > 1024) ? 1024 : 256);
}

// PCG launch shape: slab depth X = 2, run length S = 4, 256-thread blocks, one wavefront per
// tile up to kMaxGrid blocks (measured best on 144x168x111; full occupancy needs the large grid,
// which the single-block scalar kernel makes affordable).
namespace {
constexpr int kPcgS = 4;
constexpr int kPcgX = 2;
constexpr int kPcgBlock = 256;
}
Launch plan_pcg(const Geom& g, DType real) {
  (void)real;
  Launch L;
  L.S = kPcgS;
  L.block = kPcgBlock;
  L.ntiles = slab_tiles(g, kPcgS, kPcgX).ntiles;
  const int64_t wpb = kPcgBlock / kWave;
  int64_t grid = (L.ntiles + wpb - 1) / wpb;
  if (grid > kMaxGrid) grid = kMaxGrid;
  if (grid > 8) grid = (grid + 7) / 8 * 8;
  if (grid > kMaxGrid) grid = kMaxGrid;
  L.grid = (unsigned)(grid < 1 ? 1 : grid);
  return L;
}

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
  if (real == DType::F64)
    hipLaunchKernelGGL((k_pcg_step<double, kPcgS, kPcgX, kPcgBlock>), dim3(L.grid),
                       dim3(kPcgBlock), 0, s, a);
  else if (real == DType::F32)
    hipLaunchKernelGGL((k_pcg_step<float, kPcgS, kPcgX, kPcgBlock>), dim3(L.grid),
                       dim3(kPcgBlock), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_pcg_scalars(const PcgScalarArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace rgp
