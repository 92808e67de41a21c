// Gauss-Newton Hessian-vector products and the Jacobi-preconditioned CG of Sec. 2.3.1.
//
// H v at node k of a column = diag_k v_k + off_{k-1} v_{k-1} + off_k v_{k+1}
//                             - (alpha vol / h_x^2)(v_{x-} + v_{x+}) - (alpha vol / h_y^2)(v_{y-} + v_{y+})
// (existing neighbours only).  diag/off come from loss_grad; diag is also the Jacobi
// preconditioner.
//
// One PCG iteration is one kernel.  Every block first reduces the block sums of iteration i-1
// in block order (bitwise reproducible) to a_{i-1} = r.z / p.w and the next r^T z and r^T r
// from one step of the recurrences r'.z' = r.z - 2a r.w/d + a^2 w.w/d and
// r'.r' = r.r - 2a r.w + a^2 w.w (Chronopoulos-Gear), so one grid-wide reduction per iteration
// suffices and nothing needs atomics or fences.  r.z and r.r on the right are the sums of the
// stored residual of iteration i-1 itself, never earlier recurrence values, so rounding errors
// of early iterations (when |r| is large) do not accumulate into the stop test and the CG
// coefficient of late ones.  It then applies the update (x += a p, r -= a w, p = r/d + b p),
// recomputing p at the stencil halo from the previous vectors (which therefore live in
// ping-pong buffers), forms w = H p and stores its block sums of p.w, r.w/d, w.w/d, r.w, w.w,
// and r.z and r.r of the residual it stored.  In exact arithmetic the iterates are those of
// textbook PCG.
//
// The compiler does not fuse multiplies and adds in this file (contraction off below); the
// arithmetic spells out every fused multiply-add.  Each kernel variant (march shape, prefetch
// depth, plain or batched launch) therefore rounds exactly alike and a volume gets bitwise the
// same result whichever variant runs it.
#include "rgp_internal.hpp"
#include "rgp_launch.hpp"
#include "rgp_solver.hpp"
#include "batch.hpp"

#include <map>
#include <mutex>
#include <tuple>

#pragma clang fp contract(off)

namespace rgp {

__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

namespace {
constexpr int kRun = 4;
}

// Per tile every lane issues all loads of its run first (v and off at nodes k0-1 .. k0+S, diag,
// the x neighbours, and on the first / last lane of the wavefront the y neighbours, which the
// other lanes take from the adjacent lane); missing neighbours load 0 through kNullOff.
template <typename TR, int S, int BLK>
__global__ __launch_bounds__(BLK) void k_hvp(HvpArgs a) {
  const Geom g = a.g;
  const int mp = g.mp;
  const int64_t ntiles = (int64_t)g.by_nct.d * ((mp + 1 + S - 1) / S);
  const int lane = threadIdx.x & (kWave - 1);
  constexpr uint32_t kSr = sizeof(TR);
  const uint32_t nbytes = (uint32_t)(g.nnode * (int64_t)kSr);
  const BRes rD = bres(a.diag, nbytes), rO = bres(a.off, nbytes);
  const BRes rV = bres(a.v, nbytes), rH = bres(a.Hv, nbytes);
  const uint32_t nps = (uint32_t)g.nps, nxs = (uint32_t)g.nxs, nys = (uint32_t)g.nys;
  const TR cx = (TR)(a.alpha * g.vol / (g.hx * g.hx));
  const TR cy = (TR)(a.alpha * g.vol / (g.hy * g.hy));
  double acc[1] = {0.0};
  for (WaveIter it = wave_iter(ntiles, hw_block()); it.t < it.end; it.t += it.stride) {
    const ColTile c = col_tile(g, it.t, S);
    const int k0 = c.k0;
    TR vv[S + 2], oo[S + 1], dd[S], xm[S], xp[S], ym[S], yp[S];
#pragma unroll
    for (int i = 0; i < S + 2; ++i) {
      const uint32_t o = (c.nb + (uint32_t)min(max(k0 - 1 + i, 0), mp) * nps) * kSr;
      vv[i] = bld<TR>(rV, o);
      if (i < S + 1) oo[i] = bld<TR>(rO, o);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t n = c.nb + (uint32_t)min(k0 + s, mp) * nps;
      dd[s] = bld<TR>(rD, n * kSr);
      xm[s] = bld<TR>(rV, c.hasxm ? (n - nxs) * kSr : kNullOff);
      xp[s] = bld<TR>(rV, c.hasxp ? (n + nxs) * kSr : kNullOff);
      ym[s] = bld<TR>(rV, (lane == 0 && c.hasym) ? (n - nys) * kSr : kNullOff);
      yp[s] = bld<TR>(rV, (lane == kWave - 1 && c.hasyp) ? (n + nys) * kSr : kNullOff);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int k = k0 + s;
      const bool out = k <= mp && c.colok;
      const TR vk = vv[s + 1];
      const TR vym = from_lower_lane(vk, ym[s]), vyp = from_upper_lane(vk, yp[s]);
      // accumulated in FP64 and rounded once, as in the PCG step
      double hd = (double)dd[s] * (double)vk;
      if (k > 0) hd = fmad((double)oo[s], (double)vv[s], hd);
      if (k < mp) hd = fmad((double)oo[s + 1], (double)vv[s + 2], hd);
      const double crx = (double)xm[s] + (double)xp[s];  // missing x neighbours read 0
      const double cry = (c.hasym ? (double)vym : 0.0) + (c.hasyp ? (double)vyp : 0.0);
      hd = fmad(-(double)cx, crx, hd);
      hd = fmad(-(double)cy, cry, hd);
      const TR h = (TR)hd;
      bst<TR>(rH, out ? (c.nb + (uint32_t)k * nps) * kSr : kNullOff, h);
      if (out) acc[0] = fmad((double)vk, (double)h, acc[0]);
    }
  }
  if (a.part) store_partials<1, BLK>(acc, a.part, blockIdx.x);
}

// out = sum of one slot of block sums (one block).
__global__ __launch_bounds__(kReduceBlock) void k_sum_final(const double* part, unsigned nprod,
                                                      double* out) {
  double t[1];
  reduce_partials<1, kReduceBlock>(t, part, nprod);
  if (threadIdx.x == 0) *out = t[0];
}

// ---- scalar phase ---------------------------------------------------------------------------
__device__ __forceinline__ void pcg_outputs(const PcgScalarArgs& a, const PcgSlot& c) {
  a.st->pcg_iters = c.iters;
  a.st->relres = c.relres;
  if (a.iters_out) *a.iters_out = c.iters;
  if (a.relres_out) *a.relres_out = c.relres;
}

// Slot of iteration it >= 1 from the running slot of iteration it-1 and the block sums t of
// iteration it-1: [0] p.w, [1] r.w/d, [2] w.w/d, [3] r.w, [4] w.w, [5] r.r/d and [6] r.r of the
// residual that iteration stored (at it == 1 the right-hand side, whose r.r is |rhs|^2).  `fin`
// is set when the solve ends here.
__device__ __forceinline__ PcgSlot pcg_advance(const PcgSlot& prev, const double (&t)[7], int it,
                                               int maxit, double rtol, bool& fin) {
  PcgSlot cur = prev;
  const double rz = t[5], rr = t[6];
  const double bn = it == 1 ? t[6] : prev.bnorm2;
  const double pw = t[0];
  cur.bnorm2 = bn;
  if (!(bn > 0.0) || !(pw > 0.0)) {  // zero right-hand side or p^T H p <= 0: keep x
    cur.status = kPcgDone;
    cur.iters = it - 1;
    cur.relres = it == 1 ? (bn > 0.0 ? 1.0 : 0.0) : prev.relres;
    fin = true;
    return cur;
  }
  const double a2 = rz / pw;
  const double rzn = rz - 2.0 * a2 * t[1] + a2 * a2 * t[2];
  const double rrn = rr - 2.0 * a2 * t[3] + a2 * a2 * t[4];
  cur.alpha = a2;
  cur.beta = rzn / rz;
  cur.rz = rzn;
  cur.rr = rrn;
  cur.iters = it;
  cur.relres = sqrt(fmax(rrn, 0.0) / bn);
  fin = cur.relres < rtol || it >= maxit;
  cur.status = fin ? kPcgFinish : kPcgRunning;
  return cur;
}

// Slot of iteration a.iter >= 1 from the previous slot and this thread's partial sums t of the
// previous block sums (load_partials_cm); identical in every block, since the block sums are
// reduced in a fixed order.  Block 0 stores it and, when the solve ends, the iteration count and
// residual.
template <int BLK>
__device__ __forceinline__ PcgSlot pcg_scalar_phase(const PcgScalarArgs& a, const PcgSlot& prev,
                                                    double (&t)[7], VBlock vb) {
  const int it = a.iter;
  PcgSlot cur;
  bool fin = false;
  // reduced before the status is tested, so that the reduction need not wait for the slot
  // (after the end of the solve the sums are stale and unused)
  block_sum<7, BLK>(t);
  if (prev.status != kPcgRunning) {  // the solve has ended: carry the final slot forward
    cur = prev;
    cur.status = kPcgDone;
    fin = it == a.maxit;
  } else {
    cur = pcg_advance(prev, t, it, a.maxit, a.rtol, fin);
  }
  if (vb.id == 0 && threadIdx.x == 0) {
    a.slots[it & 1] = cur;
    if (fin) pcg_outputs(a, cur);
  }
  return cur;
}

// Status of iteration 0 from this thread's share `l` of loss_grad's block sums (loaded with
// load_partials_rm when gn_mode): in Gauss-Newton mode a stopped solve or a violated barrier at
// the current iterate (J = +inf) gives Done.  Block 0 finalises J, D, S, P into the state (unless
// the solve has stopped) and stores slot 0 for iteration 1.
template <int BLK>
__device__ __forceinline__ PcgSlot pcg_first_phase(const PcgScalarArgs& a, double (&l)[5],
                                                   VBlock vb) {
  bool stop = false, viol = false;
  if (a.gn_mode) {
    stop = load_flag(&a.st->gn_stop);
    block_sum<5, BLK>(l);
    viol = finalize_loss_sums(a.lf, l, !stop && vb.id == 0);
  }
  PcgSlot s0{};
  s0.status = (stop || viol) ? kPcgDone : kPcgRunning;
  if (vb.id == 0 && threadIdx.x == 0) a.slots[0] = s0;
  return s0;
}

// One block.  Iteration 0: in Gauss-Newton mode, a stopped solve or a violated barrier at the
// current iterate (J = +inf, finalised here from loss_grad's block sums) gives status Done.
// Later iterations (when not fused into k_pcg_step): the scalar phase.
__device__ __forceinline__ void pcg_scalars_body(const PcgScalarArgs& a) {
  State* st = a.st;
  if (a.iter > 0) {
    const PcgSlot prev = a.slots[(a.iter - 1) & 1];
    double t[7];
    load_partials_cm<7>(t, a.part_prev, a.nprod, 7);
    pcg_scalar_phase<kReduceBlock>(a, prev, t, VBlock{0u, 1u});
    return;
  }
  if (a.gn_mode && load_flag(&st->gn_stop)) {
    if (threadIdx.x == 0) {
      PcgSlot d{};
      d.status = kPcgDone;
      a.slots[0] = d;
    }
    return;
  }
  bool viol = false;
  if (a.gn_mode) viol = finalize_loss(a.lf, true);
  if (threadIdx.x == 0) {
    PcgSlot s0{};
    s0.status = viol ? kPcgDone : kPcgRunning;
    a.slots[0] = s0;
  }
}
__global__ __launch_bounds__(kReduceBlock) void k_pcg_scalars(PcgScalarArgs a) {
  pcg_scalars_body(a);
}
__global__ __launch_bounds__(kReduceBlock) void k_pcg_scalars_batch(
    const PcgScalarArgs* __restrict__ tab) {
  pcg_scalars_body(tab[blockIdx.x]);
}

// Slot i of the array through vector loads: a scalar load would share its wait counter with the
// LDS operations of the block reduction, which would then wait for the slot as well.
__device__ __forceinline__ PcgSlot load_slot(const PcgSlot* slots, int i) {
  static_assert(sizeof(PcgSlot) == 7 * sizeof(double), "slot layout");
  const BRes r = bres(slots, (uint32_t)(2 * sizeof(PcgSlot)));
  const uint32_t o = (uint32_t)(i * sizeof(PcgSlot));
  PcgSlot v;
  v.rz = bld<double>(r, o);
  v.rr = bld<double>(r, o + 8);
  v.bnorm2 = bld<double>(r, o + 16);
  v.relres = bld<double>(r, o + 24);
  v.alpha = bld<double>(r, o + 32);
  v.beta = bld<double>(r, o + 40);
  v.status = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)(o + 48), 0, 0);
  v.iters = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)(o + 52), 0, 0);
  return v;
}

// ---- main phase: plane-march PCG step -------------------------------------------------------
// Raw values of one node read by the update (x only on owned planes).
template <typename TR>
struct NodeRaw {
  TR d, r, w, p, x;
};
// The loads of one march step that stay in flight while the current plane is computed: the raw
// values of the plane after next, and the couplings and halo rows of the next plane.  Two sets
// alternate between the steps, so that no register with a pending load is ever copied.
template <typename TR, int NPT, int HMAX>
struct Ahead {
  NodeRaw<TR> raw[NPT];
  TR oc[NPT], ob[NPT];
  NodeRaw<TR> halo[HMAX];
};

// One PCG iteration over the units of a plane march (see MarchGeo).  Per plane o of a unit every
// thread owns npt plane positions: it applies the update (x += a p, r -= a w, p = r/d + b p,
// stored) one plane ahead (o+1) so that the o-neighbours of p stay in registers, writes p of plane
// o into an LDS plane buffer together with the two halo rows (nb positions on each side of the
// unit's flat run, recomputed from the previous vectors), and forms w = H p at plane o from LDS
// (a and b neighbours) and registers (o neighbours).  PF = 1: the raw values of plane o+2 and the
// halo rows and couplings of plane o+1 are loaded while plane o is computed (two register sets
// in turn).  PF = 3, for marches of at most 3 planes: every plane of the unit is loaded before
// the first is computed, together with the previous iteration's block sums.  Every step issues
// the same loads and stores whether or not a lane or plane needs them (unneeded ones go to
// kNullOff), so each wait covers only the loads the step consumes.  The LDS plane buffer is
// double-buffered so that one barrier per plane suffices.  Planes just outside the unit
// contribute p only (recomputed).
template <typename TR, int ROLE, int BLK, int NPT, int HMAX, int PF>
__device__ __forceinline__ void pcg_step_body(const PcgArgs& a, const MarchGeo& m, VBlock vb) {
  static_assert(PF == 1 || PF == 3, "prefetch: one plane ahead, or whole units of <= 3 planes");
  extern __shared__ unsigned char lds_raw[];
  TR* lds = reinterpret_cast<TR*>(lds_raw);
  const int it = a.sc.iter;
  const bool first = it == 0;
  const Geom g = a.g;
  const uint32_t nbytes = (uint32_t)(g.nnode * (int64_t)sizeof(TR));
  const BRes rD = bres(a.diag, nbytes), rO = bres(a.off, nbytes);
  // iteration 0 reads the right-hand side where later iterations read r (and no w, p, x)
  const BRes rR = bres(first ? a.rhs : a.r_in, nbytes);
  const BRes rX = bres(a.x, nbytes), rPi = bres(a.p_in, nbytes), rWi = bres(a.w_in, nbytes);
  const BRes rRo = bres(a.r_out, nbytes), rPo = bres(a.p_out, nbytes);
  const BRes rWo = bres(a.w_out, nbytes);
  const int no = m.no, na = m.na, nb = m.nb;
  const int64_t P = m.P;
  const int T = m.T;
  const int t = threadIdx.x;
  constexpr uint32_t kSz = sizeof(TR);
  auto off_at = [&](bool ok, int64_t n) -> uint32_t { return ok ? (uint32_t)n * kSz : kNullOff; };

  auto load_raw = [&](uint32_t bo, bool with_x) -> NodeRaw<TR> {
    NodeRaw<TR> v;
    const uint32_t bv = first ? kNullOff : bo;
    v.d = bld<TR>(rD, bo);
    v.r = bld<TR>(rR, bo);
    v.w = bld<TR>(rWi, bv);
    v.p = bld<TR>(rPi, bv);
    v.x = bld<TR>(rX, with_x ? bv : kNullOff);
    return v;
  };

  // units: 8 contiguous ranges, one per XCD (blocks are dealt to the XCDs round-robin), with the
  // o-chunk fastest so that units sharing halo planes run together on one XCD
  const unsigned G = vb.n;
  unsigned nxcd = 1, xcd = 0, lb = vb.id, gl = G;
  if (G >= 8u && G % 8u == 0u) {
    nxcd = 8u;
    xcd = vb.id % 8u;
    lb = vb.id / 8u;
    gl = G / 8u;
  }
  const int64_t ulo = m.units * xcd / nxcd, uhi = m.units * (xcd + 1) / nxcd;

  // state of the current unit and the loads of its first planes
  int64_t f0 = 0;
  int Teff = 0, o0 = 0, oe = 0;
  int fl[NPT], ia[NPT], ib[NPT];
  bool own[NPT];
  int64_t hpos[HMAX];
  NodeRaw<TR> A0[NPT], M0[NPT];
  Ahead<TR, NPT, HMAX> S0, S1, S2;
  TR Om[NPT];
  auto node = [&](int o, int i) -> int64_t { return (int64_t)o * P + f0 + fl[i]; };
  // PE-lower coupling of node n when the PE axis is a or b (0 at the lower boundary)
  auto off_lower = [&](bool ok, int64_t n, int i) -> TR {
    if (ROLE == 1) return bld<TR>(rO, off_at(ok && ia[i] > 0, n - nb));
    if (ROLE == 2) return bld<TR>(rO, off_at(ok && ib[i] > 0, n - 1));
    return TR(0);
  };
  // loads of plane q into a set: raw values of q (owned planes and the halo plane after the
  // unit), couplings and halo rows of q - 1 (owned planes)
  auto issue = [&](int q, Ahead<TR, NPT, HMAX>& s) {
    const bool raw_ok = q < no && q <= oe, cpl_ok = q - 1 < oe;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      s.raw[i] = load_raw(off_at(raw_ok, node(q, i)), q < oe);
      const int64_t n = node(q - 1, i);
      s.oc[i] = bld<TR>(rO, off_at(cpl_ok, n));
      s.ob[i] = off_lower(cpl_ok, n, i);
    }
#pragma unroll
    for (int j = 0; j < HMAX; ++j)
      s.halo[j] = load_raw(off_at(cpl_ok && hpos[j] >= 0, (int64_t)(q - 1) * P + hpos[j]), false);
  };
  // geometry of unit uu and the loads of planes o0-1, o0 and (sets S0.. ) o0+1 .. o0+PF
  auto begin_unit = [&](int64_t uu) {
    const int ti = (int)(uu / m.noc), oc = (int)(uu - (int64_t)ti * m.noc);
    f0 = (int64_t)ti * T;
    Teff = (int)min<int64_t>(T, P - f0);
    o0 = oc * m.XL;
    oe = min(o0 + m.XL, no);
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int l = t + i * BLK;
      own[i] = l < Teff;
      fl[i] = own[i] ? l : Teff - 1;
      const int64_t f = f0 + fl[i];
      ia[i] = (int)(f / nb);
      ib[i] = (int)(f - (int64_t)ia[i] * nb);
    }
#pragma unroll
    for (int j = 0; j < HMAX; ++j) {
      const int h = t + j * BLK;
      int64_t hp = -1;
      if (h < 2 * nb) {
        hp = h < nb ? f0 - nb + h : f0 + Teff + (h - nb);
        if (hp < 0 || hp >= P) hp = -1;
      }
      hpos[j] = hp;
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      A0[i] = load_raw(off_at(true, node(o0, i)), true);
      M0[i] = load_raw(off_at(o0 > 0, node(o0 - 1, i)), false);
      Om[i] = ROLE == 0 ? bld<TR>(rO, off_at(o0 > 0, node(o0 - 1, i))) : TR(0);
    }
    issue(o0 + 1, S0);
    if (PF == 3) {
      issue(o0 + 2, S1);
      issue(o0 + 3, S2);
    }
  };

  // Fused: the previous iteration's block sums are loaded first, then the first unit's planes, so
  // that the reduction waits for the former only and the latter arrive meanwhile.
  const bool fused = a.sc.fused;
  const PcgSlot prev = load_slot(a.sc.slots, (fused && !first) ? (it - 1) & 1 : it & 1);
  double tsum[7], lsum[5];
  if (fused && !first) load_partials_cm<7>(tsum, a.sc.part_prev, a.sc.nprod, 7);
  int64_t u = ulo + lb;
  if (u < uhi) begin_unit(u);
  // iteration 0: loss_grad's block sums after the unit's loads, so that one round trip covers
  // both (their loop waits for everything issued before it)
  if (fused && first && a.sc.gn_mode) load_partials_rm<5>(lsum, a.sc.lf.part, a.sc.lf.nprod);
  const PcgSlot sl = !fused ? prev
                            : (first ? pcg_first_phase<BLK>(a.sc, lsum, vb)
                                     : pcg_scalar_phase<BLK>(a.sc, prev, tsum, vb));
  if (sl.status == kPcgDone) return;
  const TR al = first ? TR(0) : (TR)sl.alpha, be = first ? TR(0) : (TR)sl.beta;
  if (sl.status == kPcgFinish) {  // last update x += a p of the previous iteration (pointwise)
    // kFin nodes per thread and round, all loads in flight together (past the end: kNullOff)
    constexpr int kFin = 8;
    const int64_t stride = (int64_t)vb.n * blockDim.x;
    for (int64_t i0 = (int64_t)vb.id * blockDim.x + threadIdx.x; i0 < g.nnode;
         i0 += kFin * stride) {
      uint32_t o[kFin];
      TR xv[kFin], pv[kFin];
#pragma unroll
      for (int u = 0; u < kFin; ++u) {
        const int64_t i = i0 + u * stride;
        o[u] = off_at(i < g.nnode, i);
        xv[u] = bld<TR>(rX, o[u]);
        pv[u] = bld<TR>(rPi, o[u]);
      }
#pragma unroll
      for (int u = 0; u < kFin; ++u) bst<TR>(rX, o[u], xv[u] + al * pv[u]);
    }
    return;
  }
  const TR sgn = (TR)a.rhs_sign;
  const TR cx = (TR)(a.alpha * g.vol / (g.hx * g.hx));
  const TR cy = (TR)(a.alpha * g.vol / (g.hy * g.hy));
  // constant couplings along the non-PE directions of the march
  const TR c_o = ROLE == 0 ? TR(0) : cx;
  const TR c_a = ROLE == 0 ? cx : (ROLE == 1 ? TR(0) : cy);
  const TR c_b = ROLE == 2 ? TR(0) : cy;
  // The update of one node from its raw values: r -= a w (iteration 0: r = sign * rhs), the
  // Jacobi step z = r / d (as r times 1/d, which the sums reuse) and p = z + b p.  Owned nodes
  // and recomputed halo nodes go through this same arithmetic, so both give bitwise the same p.
  // Iteration 0 loads w = p = x = 0 and runs with a = b = 0.
  const TR sg = first ? sgn : TR(1);
  auto upd_of = [&](const NodeRaw<TR>& v, TR& r, TR& z, TR& rd) -> TR {
    r = fmad(-al, v.w, sg * v.r);
    rd = TR(1) / v.d;
    z = r * rd;
    return fmad(be, v.p, z);
  };
  auto p_of = [&](const NodeRaw<TR>& v) -> TR {
    TR r, z, rd;
    return upd_of(v, r, z, rd);
  };
  // per plane position: p, d, r, z and 1/d of the previous (m), current (c) and next (n) plane
  TR Pm[NPT], Pc[NPT], Pn[NPT], Dc[NPT], Rc[NPT], Zc[NPT], Ic[NPT];
  TR Dn[NPT], Rn[NPT], Zn[NPT], In[NPT];
  // update of plane o (stored where `store` holds for an owned position)
  auto update = [&](int o, bool store, const NodeRaw<TR> (&R)[NPT], TR (&Pq)[NPT], TR (&Dq)[NPT],
                    TR (&Rq)[NPT], TR (&Zq)[NPT], TR (&Iq)[NPT]) {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      TR r, z, rd;
      const TR p = upd_of(R[i], r, z, rd);
      const TR xn = fmad(al, R[i].p, R[i].x);
      Pq[i] = p;
      // d is carried into the next step, which reloads this register set: adding +0 (kept under
      // IEEE rules) gives it a register of its own, so the reload never waits on a copy
      Dq[i] = R[i].d + TR(0);
      Rq[i] = r;
      Zq[i] = z;
      Iq[i] = rd;
      const uint32_t bo = off_at(store && own[i], node(o, i));
      bst<TR>(rX, bo, xn);
      bst<TR>(rRo, bo, r);
      bst<TR>(rPo, bo, p);
    }
  };

  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  // plane o: `cur` holds the raw values of o+1 and the couplings and halo rows of o; `nxt`
  // receives those of o+2 and o+1
  auto step = [&](int o, Ahead<TR, NPT, HMAX>& cur, Ahead<TR, NPT, HMAX>& nxt) {
    if (PF == 1) issue(o + 2, nxt);
    // keep the scheduler from moving these loads behind the wait for the current set
    __builtin_amdgcn_sched_barrier(0);
    update(o + 1, o + 1 < oe, cur.raw, Pn, Dn, Rn, Zn, In);
    // plane buffers of T + 2 nb positions and one spare slot that takes the halo writes of
    // lanes without a halo position (every lane consumes its halo loads, so that no load of
    // this set is left pending on some lanes only)
    TR* buf = lds + (o & 1) * (T + 2 * nb + 1);
#pragma unroll
    for (int i = 0; i < NPT; ++i) buf[fl[i] + nb] = Pc[i];
#pragma unroll
    for (int j = 0; j < HMAX; ++j)
      buf[hpos[j] >= 0 ? (int)(hpos[j] - f0) + nb : T + 2 * nb] = p_of(cur.halo[j]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int li = fl[i] + nb;
      const TR pk = Pc[i];
      const bool am = ia[i] > 0, ap = ia[i] < na - 1, bm = ib[i] > 0, bp = ib[i] < nb - 1;
      const TR pam = am ? buf[li - nb] : TR(0), pap = ap ? buf[li + nb] : TR(0);
      const TR pbm = bm ? buf[li - 1] : TR(0), pbp = bp ? buf[li + 1] : TR(0);
      const TR pom = o > 0 ? Pm[i] : TR(0), pop = o < no - 1 ? Pn[i] : TR(0);
      // w = H p accumulated in FP64 and rounded once: for smooth p the stencil's terms nearly
      // cancel (|H p| << d |p| where the Laplacian dominates), and FP32 accumulation would leave
      // an error of the size of d |p| eps_32 in w; products of FP32 values are exact in FP64
      double wd = (double)Dc[i] * (double)pk;
      if (ROLE == 0) {
        wd = fmad((double)Om[i], (double)pom, wd);
        wd = fmad((double)cur.oc[i], (double)pop, wd);
        wd = fmad(-(double)c_a, (double)pam + (double)pap, wd);
        wd = fmad(-(double)c_b, (double)pbm + (double)pbp, wd);
      } else if (ROLE == 1) {
        wd = fmad((double)cur.ob[i], (double)pam, wd);
        wd = fmad((double)cur.oc[i], (double)pap, wd);
        wd = fmad(-(double)c_o, (double)pom + (double)pop, wd);
        wd = fmad(-(double)c_b, (double)pbm + (double)pbp, wd);
      } else {
        wd = fmad((double)cur.ob[i], (double)pbm, wd);
        wd = fmad((double)cur.oc[i], (double)pbp, wd);
        wd = fmad(-(double)c_o, (double)pom + (double)pop, wd);
        wd = fmad(-(double)c_a, (double)pam + (double)pap, wd);
      }
      const TR w = (TR)wd;
      bst<TR>(rWo, off_at(own[i], node(o, i)), w);
      if (own[i]) {
        // FP64 products and sums (r.w/d as z.w, w.w/d and r.r/d with the stored 1/d); r and z
        // are this iteration's stored residual and its Jacobi step
        const double r = (double)Rc[i], ww = (double)w, z = (double)Zc[i], id = (double)Ic[i];
        acc[0] = fmad((double)pk, ww, acc[0]);
        acc[1] = fmad(z, ww, acc[1]);
        acc[2] = fmad(ww * ww, id, acc[2]);
        acc[3] = fmad(r, ww, acc[3]);
        acc[4] = fmad(ww, ww, acc[4]);
        acc[5] = fmad(r, z, acc[5]);
        acc[6] = fmad(r, r, acc[6]);
      }
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      Pm[i] = Pc[i];
      Pc[i] = Pn[i];
      Dc[i] = Dn[i];
      Rc[i] = Rn[i];
      Zc[i] = Zn[i];
      Ic[i] = In[i];
      if (ROLE == 0) Om[i] = cur.oc[i] + TR(0);  // own register, as for d above
    }
  };

  // Completes every load of begin_unit (an empty asm that reads the registers).  The march loop
  // then starts with exactly the loads of set S0 in flight, as after each of its own iterations;
  // otherwise the wait counts at the loop head would have to allow for the unit's first loads on
  // every iteration.
  auto settle = [&]() {
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      __asm__ volatile("" ::"v"(A0[i].d), "v"(A0[i].r), "v"(A0[i].w), "v"(A0[i].p), "v"(A0[i].x));
      __asm__ volatile("" ::"v"(M0[i].d), "v"(M0[i].r), "v"(M0[i].w), "v"(M0[i].p));
      __asm__ volatile("" ::"v"(S0.raw[i].d), "v"(S0.raw[i].r), "v"(S0.raw[i].w),
                       "v"(S0.raw[i].p), "v"(S0.raw[i].x));
      __asm__ volatile("" ::"v"(S0.oc[i]), "v"(S0.ob[i]), "v"(Om[i]));
    }
#pragma unroll
    for (int j = 0; j < HMAX; ++j)
      __asm__ volatile("" ::"v"(S0.halo[j].d), "v"(S0.halo[j].r), "v"(S0.halo[j].w),
                       "v"(S0.halo[j].p));
  };

  for (; u < uhi; u += gl) {
    if (u != ulo + lb) begin_unit(u);
    settle();
#pragma unroll
    for (int i = 0; i < NPT; ++i) Pm[i] = o0 > 0 ? p_of(M0[i]) : TR(0);
    update(o0, true, A0, Pc, Dc, Rc, Zc, Ic);
    if (PF == 1) {
      for (int o = o0; o < oe; o += 2) {
        step(o, S0, S1);
        if (o + 1 < oe) step(o + 1, S1, S0);
      }
    } else {  // oe - o0 <= 3 (the planner's guarantee for PF = 3)
      step(o0, S0, S0);
      if (o0 + 1 < oe) step(o0 + 1, S1, S1);
      if (o0 + 2 < oe) step(o0 + 2, S2, S2);
    }
    __syncthreads();  // the next unit reuses the LDS buffers
  }
  store_partials_cm<7, BLK>(acc, a.part, vb.id);
}

template <typename TR, int ROLE, int BLK, int NPT, int HMAX, int PF>
__global__ __launch_bounds__(BLK) void k_pcg_step(PcgArgs a, MarchGeo m) {
  pcg_step_body<TR, ROLE, BLK, NPT, HMAX, PF>(a, m, hw_block());
}

// One launch over several volumes (their PE axes may differ: the march role is per volume).
template <typename TR, int BLK, int NPT, int HMAX, int PF>
__global__ __launch_bounds__(BLK) void k_pcg_step_batch(const PcgArgs* __restrict__ tab,
                                                        const MarchGeo* __restrict__ geo,
                                                        const uint32_t* __restrict__ starts,
                                                        int n) {
  VBlock vb;
  const int p = batch_volume(starts, n, vb);
  const MarchGeo m = geo[p];
  if (m.role == 0)
    pcg_step_body<TR, 0, BLK, NPT, HMAX, PF>(tab[p], m, vb);
  else if (m.role == 1)
    pcg_step_body<TR, 1, BLK, NPT, HMAX, PF>(tab[p], m, vb);
  else
    pcg_step_body<TR, 2, BLK, NPT, HMAX, PF>(tab[p], m, vb);
}

// 256-thread workgroups, one wavefront per tile up to the grid cap (measured at 144x169x111 FP32:
// 10.3 us against 11.1 us with 1024-thread workgroups, 10.6 us with runs of 2, 11.4 us with 8).
Launch plan_hvp(const Geom& g, DType real) {
  (void)real;
  return plan_tiles(g, kRun, 256);
}

// PCG launch shape: one plane position per thread; 256-thread workgroups, 512 when the
// contiguous axis is longer than 256 nodes, so that its two halo rows fit in at most two slots
// per thread.  XL is the shortest march that keeps every unit resident at once (at most 16
// wavefronts per CU over 256 CUs): the halo planes cost less than a second wave of workgroups
// (measured on 144x168x111 and 200x200x132).  Batched launches use the same shapes (so a batched
// pair computes exactly what it computes alone) with two halo slots for every pair, unless the
// batch asks for a longer minimum march (batch_march_min), which regroups the block sums.
// Marches chosen by the autotuner (rgp_autotune), per volume geometry and field type.
namespace {
struct TuneKey {
  int32_t mp, nx, ny, pe, real;
  bool operator<(const TuneKey& o) const {
    return std::tie(mp, nx, ny, pe, real) < std::tie(o.mp, o.nx, o.ny, o.pe, o.real);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned_xl;
TuneKey tune_key(const Geom& g, DType real) { return TuneKey{g.mp, g.nx, g.ny, g.pe, (int)real}; }
}  // namespace

void set_tuned_march(const Geom& g, DType real, int xl) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (xl > 0)
    g_tuned_xl[tune_key(g, real)] = xl;
  else
    g_tuned_xl.erase(tune_key(g, real));
}

int tuned_march(const Geom& g, DType real) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const auto it = g_tuned_xl.find(tune_key(g, real));
  return it == g_tuned_xl.end() ? 0 : it->second;
}

PcgPlan plan_pcg_xl(const Geom& g, DType real, int xl_force) {
  PcgPlan L{};
  const int nb = march_geo(g, 1, 1).nb;
  L.block = 2 * nb <= 512 ? 256 : 512;
  L.npt = 1;
  L.hmax = (2 * nb <= (int)L.block && !batch_plans()) ? 1 : 2;
  const int T = (int)L.block;
  MarchGeo m = march_geo(g, T, 64);
  const int xl_t = xl_force > 0 ? xl_force : tuned_march(g, real);
  if (xl_t > 0) {
    m = march_geo(g, T, xl_t);
  } else {
    const int64_t max_units = 4096 / ((int64_t)L.block / kWave);
    for (int xl : kMarchLengths) {
      const MarchGeo c = march_geo(g, T, xl);
      if (c.units <= max_units) {
        m = c;
        break;
      }
    }
  }
  // a batched launch may ask for longer marches than the solo plan (never for a forced length)
  const int xl_b = batch_plans() && xl_force <= 0 ? batch_march_min() : 0;
  if (xl_b > m.XL) m = march_geo(g, T, xl_b < m.no ? xl_b : m.no);
  L.m = m;
  int64_t grid = m.units < kMaxGrid ? m.units : kMaxGrid;
  grid = (grid + 7) / 8 * 8;  // whole XCD rounds
  if (grid > kMaxGrid) grid = kMaxGrid;
  L.grid = (unsigned)grid;
  L.lds = 2 * (size_t)(T + 2 * nb + 1) * (real == DType::F64 ? 8 : 4);
  L.fused = 1;
  return L;
}

PcgPlan plan_pcg(const Geom& g, DType real) { return plan_pcg_xl(g, real, 0); }

hipError_t launch_hvp(const HvpArgs& a, DType real, hipStream_t s) {
  if (active_recorder())
    return record_other([a, real](hipStream_t s2) { return launch_hvp(a, real, s2); });
  const Launch L = plan_hvp(a.g, real);
  if (real == DType::F64)
    RGP_LAUNCH(kKindHvp, a.g, (k_hvp<double, kRun, 256>), L.grid, 256, 0, s, a);
  else
    RGP_LAUNCH(kKindHvp, a.g, (k_hvp<float, kRun, 256>), L.grid, 256, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sum_final(const double* part, unsigned nprod, double* out, hipStream_t s) {
  if (active_recorder())
    return record_other([part, nprod, out](hipStream_t s2) {
      return launch_sum_final(part, nprod, out, s2);
    });
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kReduceBlock), 0, s, part, nprod, out);
  return hipGetLastError();
}

template <typename TR, int BLK, int NPT, int HMAX, int PF>
static void launch_step_pf(const PcgArgs& a, const PcgPlan& L, hipStream_t s) {
  const int role = L.m.role;
  if (role == 0)
    RGP_LAUNCH_T(kKindPcgStep, a.sc.iter, a.g, (k_pcg_step<TR, 0, BLK, NPT, HMAX, PF>), L.grid,
                 BLK, L.lds, s, a, L.m);
  else if (role == 1)
    RGP_LAUNCH_T(kKindPcgStep, a.sc.iter, a.g, (k_pcg_step<TR, 1, BLK, NPT, HMAX, PF>), L.grid,
                 BLK, L.lds, s, a, L.m);
  else
    RGP_LAUNCH_T(kKindPcgStep, a.sc.iter, a.g, (k_pcg_step<TR, 2, BLK, NPT, HMAX, PF>), L.grid,
                 BLK, L.lds, s, a, L.m);
}
// units of at most 3 planes load all of them up front
template <typename TR, int BLK, int NPT, int HMAX>
static void launch_step_cfg(const PcgArgs& a, const PcgPlan& L, hipStream_t s) {
  if (L.m.XL <= 3)
    launch_step_pf<TR, BLK, NPT, HMAX, 3>(a, L, s);
  else
    launch_step_pf<TR, BLK, NPT, HMAX, 1>(a, L, s);
}

hipError_t launch_pcg_step(const PcgArgs& a, DType real, hipStream_t s) {
  return launch_pcg_step_plan(a, real, plan_pcg(a.g, real), s);
}

hipError_t launch_pcg_step_plan(const PcgArgs& a, DType real, const PcgPlan& L, hipStream_t s) {
  if (active_recorder()) {
    const hipError_t e = record_launch(RecKind::kPcgStep, a, L.grid, L.block, L.lds, (int)real, L.npt, L.hmax,
                  [a, real](hipStream_t s2) { return launch_pcg_step(a, real, s2); }, &L.m);
    if (e != hipSuccess) return e;
    return note_volume(a.g.ncell, a.g.nnode, a.sc.iter);
  }
  if (2 * L.m.nb > L.hmax * (int)L.block) return hipErrorInvalidValue;
  if (real != DType::F64 && real != DType::F32) return hipErrorInvalidValue;
  const bool f64 = real == DType::F64;
  if (L.block == 512) {
    if (f64)
      launch_step_cfg<double, 512, 1, 2>(a, L, s);
    else
      launch_step_cfg<float, 512, 1, 2>(a, L, s);
  } else if (L.hmax == 1) {
    if (f64)
      launch_step_cfg<double, 256, 1, 1>(a, L, s);
    else
      launch_step_cfg<float, 256, 1, 1>(a, L, s);
  } else {
    if (f64)
      launch_step_cfg<double, 256, 1, 2>(a, L, s);
    else
      launch_step_cfg<float, 256, 1, 2>(a, L, s);
  }
  return hipGetLastError();
}

hipError_t launch_pcg_scalars(const PcgScalarArgs& a, hipStream_t s) {
  if (active_recorder())
    return record_launch(RecKind::kPcgScalars, a, 1, kReduceBlock, 0, 0, 0, 0,
                         [a](hipStream_t s2) { return launch_pcg_scalars(a, s2); });
  hipLaunchKernelGGL(k_pcg_scalars, dim3(1), dim3(kReduceBlock), 0, s, a);
  return hipGetLastError();
}

// ---- shared launches over several volumes -----------------------------------------------------

hipError_t launch_pcg_scalars_batch(const void* tab, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_scalars_batch, dim3(n), dim3(kReduceBlock), 0, s,
                     static_cast<const PcgScalarArgs*>(tab));
  return hipGetLastError();
}

hipError_t launch_pcg_step_batch(const void* tab, const MarchGeo* geo, const uint32_t* starts,
                                 int n, unsigned grid, size_t lds, DType real, int max_xl,
                                 int64_t cells, int64_t nodes, int tag, hipStream_t s) {
  const PcgArgs* t = static_cast<const PcgArgs*>(tab);
  const bool whole = max_xl <= 3;
#define RGP_PCG_B(TR, PF)                                                                     \
  RGP_LAUNCH_TN(kKindPcgStep, tag, cells, nodes, (k_pcg_step_batch<TR, 256, 1, 2, PF>), grid, \
                256, lds, s, t, geo, starts, n)
  if (real == DType::F64) {
    if (whole)
      RGP_PCG_B(double, 3);
    else
      RGP_PCG_B(double, 1);
  } else if (real == DType::F32) {
    if (whole)
      RGP_PCG_B(float, 3);
    else
      RGP_PCG_B(float, 1);
  } else {
    return hipErrorInvalidValue;
  }
#undef RGP_PCG_B
  return hipGetLastError();
}

}  // namespace rgp
