// Objective, gradient and Gauss-Newton linearisation; Armijo trial evaluations; step application;
// Jacobian-modulation correction.  gfx950, one thread per run of S consecutive nodes of a column.
//
// Per cell j of a column (Eq. 1-6 of the paper, staggered discretisation of Sec. 2.1):
//   A b_j = (b_j + b_{j+1}) / 2,   D b_j = (b_{j+1} - b_j) / h_pe,   t_j = A b_j / h_pe
//   I+(xi+) , I-(xi-) with xi+- = j +- t_j   (1D linear image model, zero outside the column)
//   r_j = I+(xi+) (1 + D b_j) - I-(xi-) (1 - D b_j)
//   c1 = I+'(xi+)(1 + D b) + I-'(xi-)(1 - D b),  c2 = I+(xi+) + I-(xi-)
//   u0 = dr_j/db_j = c1/2 - c2/h,  u1 = dr_j/db_{j+1} = c1/2 + c2/h.
// The Gauss-Newton Hessian vol Jr^T Jr + alpha vol L + (beta vol/2) D^T diag(phi'') D couples a
// node to its two PE neighbours through per-cell 2x2 blocks, so it is stored as a tridiagonal
// along every column (diag, off) plus the constant cross-axis Laplacian couplings.
#include "rgp_internal.hpp"
#include "rgp_launch.hpp"
#include "rgp_solver.hpp"
#include "batch.hpp"

namespace rgp {

template <typename TI, typename TR>
__device__ __forceinline__ void interp_at(const TI* __restrict__ I, int64_t cb, int64_t cps,
                                          int mp, int j, TR t, TR inv_hp, TR& val, TR& slope) {
  TR ft = floor(t);
  ft = fmin(fmax(ft, TR(-mp - 2)), TR(mp + 2));
  const TR w = t - ft;
  const int k0 = j + static_cast<int>(ft);
  TR v0 = TR(0), v1 = TR(0);
  if (k0 >= 0 && k0 < mp) v0 = to_real(I[cb + (int64_t)k0 * cps], TR());
  if (k0 + 1 >= 0 && k0 + 1 < mp) v1 = to_real(I[cb + (int64_t)(k0 + 1) * cps], TR());
  val = (TR(1) - w) * v0 + w * v1;
  slope = (v1 - v0) * inv_hp;
}

// Residual-related quantities of one cell.
template <typename TR>
struct CellOut {
  TR r, u0, u1, db;
};

template <typename TI, typename TR>
__device__ __forceinline__ CellOut<TR> eval_cell(const TI* __restrict__ Ip, const TI* __restrict__ Im,
                                                 int64_t cb, int64_t cps, int mp, int j, TR b0,
                                                 TR b1, TR inv_hp) {
  const TR ab = (b0 + b1) * TR(0.5);
  const TR db = (b1 - b0) * inv_hp;
  const TR t = ab * inv_hp;
  TR vp, sp, vm, sm;
  interp_at(Ip, cb, cps, mp, j, t, inv_hp, vp, sp);
  interp_at(Im, cb, cps, mp, j, -t, inv_hp, vm, sm);
  const TR ap = TR(1) + db, am = TR(1) - db;
  CellOut<TR> o;
  o.r = vp * ap - vm * am;
  const TR c1 = sp * ap + sm * am;
  const TR c2 = vp + vm;
  o.u0 = c1 * TR(0.5) - c2 * inv_hp;
  o.u1 = c1 * TR(0.5) + c2 * inv_hp;
  o.db = db;
  return o;
}

// t clamped to [-lim, lim] (one median-of-three).
__device__ __forceinline__ float clamp_abs(float t, float lim) {
  return __builtin_amdgcn_fmed3f(t, -lim, lim);
}
__device__ __forceinline__ double clamp_abs(double t, double lim) { return fmin(fmax(t, -lim), lim); }

// 1/q: the hardware reciprocal in FP32 (1 ulp), a division in FP64.
__device__ __forceinline__ float recip(float q) { return __builtin_amdgcn_rcpf(q); }
__device__ __forceinline__ double recip(double q) { return 1.0 / q; }

// phi(z) = z^4/(1-z^2), phi', phi'' (Eq. 3); valid for |z| < 1.
template <typename TR>
__device__ __forceinline__ void phi3(TR z, TR& f, TR& f1, TR& f2) {
  const TR z2 = z * z;
  const TR iq = recip(TR(1) - z2);
  const TR iq2 = iq * iq;
  f = z2 * z2 * iq;
  f1 = TR(2) * z2 * z * (TR(2) - z2) * iq2;
  f2 = TR(2) * z2 * (TR(6) - TR(3) * z2 + z2 * z2) * iq2 * iq;
}

// --------------------------------------------------------------------------------------------
// loss_grad: block sums of D, S, P (and |grad J|^2); optionally grad J and the GN tridiagonal
// (diag, off).  With STEP it first forms b = b_in + gamma q (gamma and the acceptance from the
// line search) and writes it to b_out, a different buffer since neighbours read b_in.
// Per tile every lane first issues all loads of its run (b, and q with STEP, at nodes k0-1 ..
// k0+S, the x neighbours, and on the first / last lane of the wavefront the y neighbours, which
// the other lanes take from the adjacent lane), then the image taps of its S+1 cells, then
// computes.  Every load and store is unconditional: unneeded ones use kNullOff, and a missing
// output array is a descriptor of size 0.
// --------------------------------------------------------------------------------------------
template <typename TI, typename TR, int S, int BLK, bool STEP>
__device__ __forceinline__ void loss_grad_body(const LossGradArgs& a, VBlock vb) {
  const Geom g = a.g;
  State* st = a.st;
  const int mp = g.mp;
  const int64_t ntiles = (int64_t)g.by_nct.d * ((mp + 1 + S - 1) / S);
  const int lane = threadIdx.x & (kWave - 1);

  if (a.level_start && vb.id == 0 && threadIdx.x == 0) {
    // a non-finite input image (found by the input scan) stops every level before its first step
    st->gn_stop = st->status == RGP_ENONFINITE ? 1 : 0;
    st->accepted = 0;
  }
  TR coef = TR(0);
  if (STEP) {
    if (load_flag(&st->gn_stop)) {  // the solve stopped on this level: carry b over unchanged
      const TR* __restrict__ bin = static_cast<const TR*>(a.b_in);
      TR* __restrict__ bout = static_cast<TR*>(a.b_out);
      const int64_t stride = (int64_t)vb.n * blockDim.x;
      for (int64_t i = (int64_t)vb.id * blockDim.x + threadIdx.x; i < g.nnode; i += stride)
        bout[i] = bin[i];
      return;
    }
    coef = st->accepted ? (TR)st->gamma : TR(0);
  }

  constexpr uint32_t kSr = sizeof(TR), kSi = sizeof(TI);
  const uint32_t nbytes = (uint32_t)(g.nnode * (int64_t)kSr);
  const uint32_t cbytes = (uint32_t)(g.ncell * (int64_t)kSi);
  const BRes rIp = bres(a.Ip, cbytes), rIm = bres(a.Im, cbytes);
  const BRes rB = bres(a.b_in, nbytes), rQ = bres(STEP ? a.q : nullptr, STEP ? nbytes : 0u);
  const BRes rBo = bres(a.b_out, STEP && a.b_out ? nbytes : 0u);
  const BRes rG = bres(a.grad, a.grad ? nbytes : 0u);
  const BRes rD = bres(a.diag, a.diag ? nbytes : 0u), rO = bres(a.off, a.diag ? nbytes : 0u);
  const uint32_t nps = (uint32_t)g.nps, nxs = (uint32_t)g.nxs, nys = (uint32_t)g.nys;
  const uint32_t cps = (uint32_t)g.cps;
  const bool prox = a.prox_c != nullptr;
  const BRes rC = bres(a.prox_c, prox ? nbytes : 0u);
  const double rho = prox ? st->admm_rho : 0.0;
  const TR prv = (TR)(rho * g.vol), prw = (TR)(prox ? rho / a.alpha : 0.0);

  const TR inv_hp = TR(1) / (TR)g.hp;
  const TR wp2 = TR(1) / ((TR)g.hp * (TR)g.hp);
  const TR wx2 = TR(1) / ((TR)g.hx * (TR)g.hx);
  const TR wy2 = TR(1) / ((TR)g.hy * (TR)g.hy);
  const TR vol = (TR)g.vol;
  const TR avol = (TR)(a.alpha * g.vol);
  const TR bh = (TR)(0.5 * a.beta * g.vol);
  const TR hih = TR(0.5) * inv_hp, bhi = bh * inv_hp, bhw = bh * wp2, avw = avol * wp2;
  const TR lim = TR(mp + 2);

  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // r^2, S terms, phi, violations, g^2

  for (WaveIter it = wave_iter(ntiles, vb); it.t < it.end; it.t += it.stride) {
    ColTile c = col_tile(g, it.t, S);
    if (prox) c.hasxm = c.hasxp = c.hasym = c.hasyp = false;  // F_rho: PE smoothness only
    const int k0 = __builtin_amdgcn_readfirstlane(c.k0);  // uniform: one tile per wavefront
    auto noff = [&](int k) -> uint32_t { return (c.nb + (uint32_t)k * nps) * kSr; };

    // 1. b (and q) at nodes k0-1 .. k0+S clamped into the column, the x neighbours and the
    //    wavefront-edge y neighbours of nodes k0 .. k0+S-1 (node k clamped to mp)
    TR bv[S + 2], qv[S + 2], xm[S], xp[S], ym[S], yp[S], qxm[S], qxp[S], qym[S], qyp[S];
#pragma unroll
    for (int i = 0; i < S + 2; ++i) {
      const int k = min(max(k0 - 1 + i, 0), mp);
      bv[i] = bld<TR>(rB, noff(k));
      if (STEP) qv[i] = bld<TR>(rQ, noff(k));
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t n = c.nb + (uint32_t)min(k0 + s, mp) * nps;
      const uint32_t oxm = c.hasxm ? (n - nxs) * kSr : kNullOff;
      const uint32_t oxp = c.hasxp ? (n + nxs) * kSr : kNullOff;
      const uint32_t oym = (lane == 0 && c.hasym) ? (n - nys) * kSr : kNullOff;
      const uint32_t oyp = (lane == kWave - 1 && c.hasyp) ? (n + nys) * kSr : kNullOff;
      xm[s] = bld<TR>(rB, oxm);
      xp[s] = bld<TR>(rB, oxp);
      ym[s] = bld<TR>(rB, oym);
      yp[s] = bld<TR>(rB, oyp);
      if (STEP) {
        qxm[s] = bld<TR>(rQ, oxm);
        qxp[s] = bld<TR>(rQ, oxp);
        qym[s] = bld<TR>(rQ, oym);
        qyp[s] = bld<TR>(rQ, oyp);
      }
    }
    if (STEP) {
#pragma unroll
      for (int i = 0; i < S + 2; ++i) bv[i] += coef * qv[i];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        xm[s] += coef * qxm[s];
        xp[s] += coef * qxp[s];
        ym[s] += coef * qym[s];
        yp[s] += coef * qyp[s];
      }
    }

    // 2. image taps of cells k0-1 .. k0+S-1 (cell index k0-1+i for i = 0..S): the linear image
    //    model is zero outside the column, which the out-of-range offset reproduces (a sample
    //    position beyond +-(mp+2) cells has both taps outside, so it is clamped there first)
    TR vp0[S + 1], vp1[S + 1], vm0[S + 1], vm1[S + 1], wp[S + 1], wm[S + 1];
#pragma unroll
    for (int i = 0; i <= S; ++i) {
      const int j = k0 - 1 + i;
      const TR t = clamp_abs((bv[i] + bv[i + 1]) * hih, lim);
      const TR fp = floor(t), fm = floor(-t);
      wp[i] = t - fp;
      wm[i] = -t - fm;
      const int kp = j + (int)fp, km = j + (int)fm;
      const uint32_t rp = c.cb + (uint32_t)kp * cps, rm = c.cb + (uint32_t)km * cps;
      vp0[i] = bld_img<TI, TR>(rIp, (uint32_t)kp < (uint32_t)mp ? rp * kSi : kNullOff);
      vp1[i] = bld_img<TI, TR>(rIp, (uint32_t)(kp + 1) < (uint32_t)mp ? (rp + cps) * kSi : kNullOff);
      vm0[i] = bld_img<TI, TR>(rIm, (uint32_t)km < (uint32_t)mp ? rm * kSi : kNullOff);
      vm1[i] = bld_img<TI, TR>(rIm, (uint32_t)(km + 1) < (uint32_t)mp ? (rm + cps) * kSi : kNullOff);
    }

    // 3. per cell i (between nodes k0-1+i and k0+i): residual r, its derivatives u0, u1 with
    //    respect to the lower and upper node, phi; then the cell's gradient and Hessian
    //    contributions to its upper node (gU, dU), to its lower node (gD, dD) and the coupling
    //    of the two nodes (oc)
    TR gU[S + 1], dU[S + 1], gD[S + 1], dD[S + 1], oc[S + 1];
    TR tr2 = TR(0), tf = TR(0), tviol = TR(0);
#pragma unroll
    for (int i = 0; i <= S; ++i) {
      const TR db = (bv[i + 1] - bv[i]) * inv_hp;
      const TR ep = vp1[i] - vp0[i], em = vm1[i] - vm0[i];
      const TR valp = fma(wp[i], ep, vp0[i]), valm = fma(wm[i], em, vm0[i]);
      const TR ap = TR(1) + db, am = TR(1) - db;
      const TR r = valp * ap - valm * am;
      const TR c1h = (ep * ap + em * am) * hih;   // (slope+ (1+Db) + slope- (1-Db)) / 2
      const TR c2h = (valp + valm) * inv_hp;
      const TR u0 = c1h - c2h, u1 = c1h + c2h;
      TR f = TR(0), f1 = TR(0), f2 = TR(0);
      const bool viol = !(fabs(db) < TR(1));
      if (!viol) phi3(db, f, f1, f2);
      const TR vr = vol * r, pf1 = bhi * f1, pf2 = bhw * f2;
      gU[i] = fma(vr, u1, pf1);
      dU[i] = fma(vol * u1, u1, pf2);
      gD[i] = fma(vr, u0, -pf1);
      dD[i] = fma(vol * u0, u0, pf2);
      oc[i] = fma(vol * u0, u1, -pf2) - avw;
      // cells of the column only (cell index 0 .. mp-1), nodes of the run only (i >= 1)
      const int j = k0 - 1 + i;
      if (i >= 1 && j < mp && c.colok) {
        tr2 = fma(r, r, tr2);
        tf += f;
        tviol += viol ? TR(1) : TR(0);
      }
    }

    // 4. per node k = k0 + s: cells k-1 (index s, its upper node) and k (index s+1, its lower
    //    node), the Laplacian (Neumann) and the forward differences of S.  The cross-axis terms
    //    take the column's weights, 0 for a missing neighbour: adding a zero term leaves every
    //    sum exactly as skipping it would, without a select per node and term.
    const TR wxm = c.hasxm ? wx2 : TR(0), wxp = c.hasxp ? wx2 : TR(0);
    const TR wym = c.hasym ? wy2 : TR(0), wyp = c.hasyp ? wy2 : TR(0);
    TR tst = TR(0), tg2 = TR(0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int k = k0 + s;
      const bool nodeok = k <= mp, lo = k > 0, up = k < mp;
      const TR bk = bv[s + 1];
      const TR bym = from_lower_lane(bk, ym[s]), byp = from_upper_lane(bk, yp[s]);
      const TR dpm = bk - bv[s], dpp = bv[s + 2] - bk;
      const TR dxm = bk - xm[s], dxp = xp[s] - bk, dym = bk - bym, dyp = byp - bk;
      TR lap = TR(0), ldg = TR(0), st = TR(0);
      if (lo) { lap = fma(dpm, wp2, lap); ldg += wp2; }
      if (up) { lap = fma(-dpp, wp2, lap); ldg += wp2; st = fma(dpp * dpp, wp2, st); }
      lap = fma(dxm, wxm, lap);
      ldg += wxm;
      lap = fma(-dxp, wxp, lap);
      ldg += wxp;
      st = fma(dxp * dxp, wxp, st);
      lap = fma(dym, wym, lap);
      ldg += wym;
      lap = fma(-dyp, wyp, lap);
      ldg += wyp;
      st = fma(dyp * dyp, wyp, st);
      TR gk = (lo ? gU[s] : TR(0)) + (up ? gD[s + 1] : TR(0)) + avol * lap;
      TR dk = (lo ? dU[s] : TR(0)) + (up ? dD[s + 1] : TR(0)) + avol * ldg;
      if (prox) {   // (rho vol / 2)|b - c|^2: gradient rho vol e, diagonal rho vol
        const TR e = bk - bld<TR>(rC, noff(min(k, mp)));
        gk = fma(prv, e, gk);
        dk += prv;
        st = fma(prw * e, e, st);
      }
      const bool out = nodeok && c.colok;
      if (out) {
        tst += st;
        tg2 = fma(gk, gk, tg2);
      }
      const uint32_t o = out ? noff(k) : kNullOff;
      bst<TR>(rG, o, gk);
      bst<TR>(rD, o, dk);
      bst<TR>(rO, o, up ? oc[s + 1] : TR(0));
      bst<TR>(rBo, o, bk);
    }
    // the tile's sums (at most S+1 terms each) join the FP64 block sums
    acc[0] += (double)tr2;
    acc[1] += (double)tst;
    acc[2] += (double)tf;
    acc[3] += (double)tviol;
    acc[4] += (double)tg2;
  }
  store_partials<5, BLK>(acc, a.part, vb.id);
}

template <typename TI, typename TR, int S, int BLK, bool STEP>
__global__ __launch_bounds__(BLK) void k_loss_grad(LossGradArgs a) {
  loss_grad_body<TI, TR, S, BLK, STEP>(a, hw_block());
}

// One launch over several volumes: tab[p] drives the workgroups starts[p] .. starts[p+1]-1.
template <typename TI, typename TR, int BLK>
__global__ __launch_bounds__(BLK) void k_loss_grad_batch(const LossGradArgs* __restrict__ tab,
                                                         const uint32_t* __restrict__ starts,
                                                         int n) {
  VBlock vb;
  const int p = batch_volume(starts, n, vb);
  const LossGradArgs& a = tab[p];
  if (a.run == 4) {
    if (a.step)
      loss_grad_body<TI, TR, 4, BLK, true>(a, vb);
    else
      loss_grad_body<TI, TR, 4, BLK, false>(a, vb);
  } else {
    if (a.step)
      loss_grad_body<TI, TR, 2, BLK, true>(a, vb);
    else
      loss_grad_body<TI, TR, 2, BLK, false>(a, vb);
  }
}

// J, D, S, P from loss_grad's block sums (standalone entry point; one block).
__global__ __launch_bounds__(kReduceBlock) void k_loss_final(LossFinalArgs a) { finalize_loss(a, true); }

// --------------------------------------------------------------------------------------------
// Armijo trials: block sums of D and P at b + gamma_c q for NC step sizes gamma_c = 2^-(first+c)
// in one pass.  S(b + gamma q) = S + gamma vol sum(dB dQ)/h^2 + gamma^2 (vol/2) sum(dQ^2)/h^2 is
// exact, so only D and P are evaluated per candidate; the pass with first == 0 also forms grad.q
// and the two S sums.  A single-block decide kernel then takes the first (largest) gamma that
// satisfies the Armijo condition, which is exactly what halving from gamma = 1 selects.
// --------------------------------------------------------------------------------------------
template <typename TI, typename TR, int S, int NC, int BLK, bool PASS0>
__device__ __forceinline__ void trial_body(const TrialArgs& a, VBlock vb) {
  const State* st = a.st;
  if (load_flag(&st->gn_stop) || st->accepted) return;
  const Geom g = a.g;
  const int mp = g.mp;
  const int64_t ntiles = (int64_t)g.by_nct.d * ((mp + 1 + S - 1) / S);
  const int lane = threadIdx.x & (kWave - 1);

  constexpr uint32_t kSr = sizeof(TR), kSi = sizeof(TI);
  const uint32_t nbytes = (uint32_t)(g.nnode * (int64_t)kSr);
  const uint32_t cbytes = (uint32_t)(g.ncell * (int64_t)kSi);
  const BRes rIp = bres(a.Ip, cbytes), rIm = bres(a.Im, cbytes);
  const BRes rB = bres(a.b, nbytes), rQ = bres(a.q, nbytes), rG = bres(a.grad, nbytes);
  const uint32_t nps = (uint32_t)g.nps, nxs = (uint32_t)g.nxs, nys = (uint32_t)g.nys;
  const uint32_t cps = (uint32_t)g.cps;
  const bool prox = a.prox_c != nullptr;
  const BRes rC = bres(a.prox_c, prox ? nbytes : 0u);
  const TR prw = (TR)(prox ? st->admm_rho / a.alpha : 0.0);

  const TR inv_hp = TR(1) / (TR)g.hp;
  const TR hih = TR(0.5) * inv_hp;
  const TR wp2 = TR(1) / ((TR)g.hp * (TR)g.hp);
  const TR wx2 = TR(1) / ((TR)g.hx * (TR)g.hx);
  const TR wy2 = TR(1) / ((TR)g.hy * (TR)g.hy);
  const TR lim = TR(mp + 2);
  TR gam[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) gam[c] = (TR)ldexp(1.0, -(a.first + c));

  constexpr int K = 3 + 3 * NC;
  double v[K];
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = 0.0;

  for (WaveIter it = wave_iter(ntiles, vb); it.t < it.end; it.t += it.stride) {
    ColTile c = col_tile(g, it.t, S);
    if (prox) c.hasxm = c.hasxp = c.hasym = c.hasyp = false;  // F_rho: PE smoothness only
    const int k0 = __builtin_amdgcn_readfirstlane(c.k0);  // uniform: one tile per wavefront
    auto noff = [&](int k) -> uint32_t { return (c.nb + (uint32_t)k * nps) * kSr; };
    // b, q at nodes k0 .. k0+S (clamped to mp); first pass: grad and the upper x and y neighbours
    // (y on the last lane of the wavefront; the others take it from the next lane)
    TR bb[S + 1], qq[S + 1], gk[S], bxp[S], qxp[S], byp[S], qyp[S];
#pragma unroll
    for (int i = 0; i <= S; ++i) {
      const uint32_t o = noff(min(k0 + i, mp));
      bb[i] = bld<TR>(rB, o);
      qq[i] = bld<TR>(rQ, o);
    }
    if (PASS0) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const uint32_t n = c.nb + (uint32_t)min(k0 + s, mp) * nps;
        const uint32_t oxp = c.hasxp ? (n + nxs) * kSr : kNullOff;
        const uint32_t oyp = (lane == kWave - 1 && c.hasyp) ? (n + nys) * kSr : kNullOff;
        gk[s] = bld<TR>(rG, n * kSr);
        bxp[s] = bld<TR>(rB, oxp);
        qxp[s] = bld<TR>(rQ, oxp);
        byp[s] = bld<TR>(rB, oyp);
        qyp[s] = bld<TR>(rQ, oyp);
      }
    }
    // image taps of cells k0 .. k0+S-1 for every candidate step
    TR vp0[S][NC], vp1[S][NC], vm0[S][NC], vm1[S][NC], wp[S][NC], wm[S][NC];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int k = k0 + s;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const TR b0 = fma(gam[cc], qq[s], bb[s]), b1 = fma(gam[cc], qq[s + 1], bb[s + 1]);
        const TR t = clamp_abs((b0 + b1) * hih, lim);
        const TR fp = floor(t), fm = floor(-t);
        wp[s][cc] = t - fp;
        wm[s][cc] = -t - fm;
        const int kp = k + (int)fp, km = k + (int)fm;
        const uint32_t rp = c.cb + (uint32_t)kp * cps, rm = c.cb + (uint32_t)km * cps;
        vp0[s][cc] = bld_img<TI, TR>(rIp, (uint32_t)kp < (uint32_t)mp ? rp * kSi : kNullOff);
        vp1[s][cc] =
            bld_img<TI, TR>(rIp, (uint32_t)(kp + 1) < (uint32_t)mp ? (rp + cps) * kSi : kNullOff);
        vm0[s][cc] = bld_img<TI, TR>(rIm, (uint32_t)km < (uint32_t)mp ? rm * kSi : kNullOff);
        vm1[s][cc] =
            bld_img<TI, TR>(rIm, (uint32_t)(km + 1) < (uint32_t)mp ? (rm + cps) * kSi : kNullOff);
      }
    }
    // tile sums in the working precision (at most S terms each), then into the FP64 block sums
    TR tgq = TR(0), tsbq = TR(0), tsqq = TR(0);
    TR tr2[NC], tph[NC], tvi[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) tr2[cc] = tph[cc] = tvi[cc] = TR(0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int k = k0 + s;
      const bool nodeok = k <= mp && c.colok;
      if (PASS0) {
        const TR bk = bb[s], qk = qq[s];
        const TR by = from_upper_lane(bk, byp[s]), qy = from_upper_lane(qk, qyp[s]);
        TR sbq = TR(0), sqq = TR(0);
        if (k < mp) {
          const TR db = bb[s + 1] - bk, dq = qq[s + 1] - qk;
          sbq = fma(db * dq, wp2, sbq);
          sqq = fma(dq * dq, wp2, sqq);
        }
        {  // cross-axis terms with weight 0 for a missing neighbour (an exact no-op)
          const TR wxp = c.hasxp ? wx2 : TR(0), wyp = c.hasyp ? wy2 : TR(0);
          const TR dbx = bxp[s] - bk, dqx = qxp[s] - qk;
          sbq = fma(dbx * dqx, wxp, sbq);
          sqq = fma(dqx * dqx, wxp, sqq);
          const TR dby = by - bk, dqy = qy - qk;
          sbq = fma(dby * dqy, wyp, sbq);
          sqq = fma(dqy * dqy, wyp, sqq);
        }
        if (prox) {   // the proximal term as part of S: (rho / alpha)(e q, q^2) with e = b - c
          const TR e = bk - bld<TR>(rC, noff(min(k, mp)));
          sbq = fma(prw * e, qk, sbq);
          sqq = fma(prw * qk, qk, sqq);
        }
        if (nodeok) {
          tgq = fma(gk[s], qk, tgq);
          tsbq += sbq;
          tsqq += sqq;
        }
      }
      if (nodeok && k < mp) {
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          const TR b0 = fma(gam[cc], qq[s], bb[s]), b1 = fma(gam[cc], qq[s + 1], bb[s + 1]);
          const TR db = (b1 - b0) * inv_hp;
          const TR valp = fma(wp[s][cc], vp1[s][cc] - vp0[s][cc], vp0[s][cc]);
          const TR valm = fma(wm[s][cc], vm1[s][cc] - vm0[s][cc], vm0[s][cc]);
          const TR r = valp * (TR(1) + db) - valm * (TR(1) - db);
          tr2[cc] = fma(r, r, tr2[cc]);
          if (fabs(db) < TR(1)) {
            const TR z2 = db * db;
            tph[cc] += z2 * z2 * recip(TR(1) - z2);
          } else {
            tvi[cc] += TR(1);
          }
        }
      }
    }
    if (PASS0) {
      v[0] += (double)tgq;
      v[1] += (double)tsbq;
      v[2] += (double)tsqq;
    }
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      v[3 + 3 * cc] += (double)tr2[cc];
      v[4 + 3 * cc] += (double)tph[cc];
      v[5 + 3 * cc] += (double)tvi[cc];
    }
  }
  // column-major (sum k of block b at k * kMaxGrid + b): the single-block decision kernel then
  // reads each sum of consecutive blocks from consecutive addresses
  store_partials_cm<K, BLK>(v, a.part, vb.id);
}

template <typename TI, typename TR, int S, int NC, int BLK, bool PASS0>
__global__ __launch_bounds__(BLK) void k_trial(TrialArgs a) {
  trial_body<TI, TR, S, NC, BLK, PASS0>(a, hw_block());
}

// Shared launches: every volume of one launch is in the same pass, so `first` is uniform.
template <typename TI, typename TR, int S, int NC, int BLK>
__global__ __launch_bounds__(BLK) void k_trial_batch(const TrialArgs* __restrict__ tab,
                                                     const uint32_t* __restrict__ starts, int n) {
  VBlock vb;
  const int p = batch_volume(starts, n, vb);
  if constexpr (NC == 1) {
    if (tab[p].first == 0) {
      trial_body<TI, TR, S, NC, BLK, true>(tab[p], vb);
      return;
    }
  }
  trial_body<TI, TR, S, NC, BLK, false>(tab[p], vb);
}

// Armijo decision on the pass just evaluated (one block per volume).
// This thread's share of K column-major block sums (sum k of block b at k * kMaxGrid + b) over
// nprod blocks: blocks threadIdx.x, + blockDim.x, ..., loaded kB blocks per sum at a time, all
// independent (fewer for many sums, so that the loads stay in registers); fixed summation order.
template <int K>
__device__ __forceinline__ void trial_sums_share(double (&out)[K], const double* part,
                                                 unsigned nprod) {
  constexpr int kB = K <= 8 ? 4 : (K <= 16 ? 2 : 1);
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  for (unsigned b0 = 0; b0 < nprod; b0 += kB * blockDim.x) {
    double v[K][kB];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int j = 0; j < kB; ++j) {
        const unsigned b = b0 + j * blockDim.x + threadIdx.x;
        v[k][j] = b < nprod ? part[(size_t)k * kMaxGrid + b] : 0.0;
      }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int j = 0; j < kB; ++j) out[k] += v[k][j];
  }
}

// The single-candidate pass (gamma = 1) is decided at every Gauss-Newton step that runs, so its
// block sums are loaded together with the state (one memory round trip); a later pass is usually
// skipped (a step was accepted), so its larger set of sums is loaded only once the state says it
// ran.
template <int NC>
__device__ __forceinline__ void decide_body(const DecideArgs& a) {
  const State* st = a.st;
  double t[3 + 3 * NC];
  // vector loads, so that they are counted with the block sums below (written by earlier kernels)
  const int stop = load_flag(&st->gn_stop), acc = load_flag(&st->accepted);
  if (NC == 1) {
    trial_sums_share<3 + 3 * NC>(t, a.part_prev, a.nprod_prev);
    // keeps the loads above the test below (they are not needed on its early-out path, and
    // would otherwise be sunk past it into a second memory round trip)
    __asm__ volatile("" ::"v"(t[0]));
  }
  if (stop || acc) return;
  const State s = *st;
  if (NC != 1) trial_sums_share<3 + 3 * NC>(t, a.part_prev, a.nprod_prev);
  decide_pass<NC>(a, s, t);
}
template <int NC>
__global__ __launch_bounds__(kReduceBlock) void k_decide(DecideArgs a) { decide_body<NC>(a); }
template <int NC>
__global__ __launch_bounds__(kReduceBlock) void k_decide_batch(const DecideArgs* __restrict__ tab) {
  decide_body<NC>(tab[blockIdx.x]);
}

// b <- b + gamma q (in place, pointwise) with the accepted line-search step.
template <typename TR>
__device__ __forceinline__ void apply_step_body(const ApplyArgs& a, VBlock vb) {
  const State* st = a.st;
  if (!st->accepted) return;
  const TR gam = (TR)st->gamma;
  TR* __restrict__ b = static_cast<TR*>(a.b);
  const TR* __restrict__ q = static_cast<const TR*>(a.q);
  const int64_t i = (int64_t)vb.id * kBlock + threadIdx.x;
  if (i < a.n) b[i] = b[i] + gam * q[i];
}
template <typename TR>
__global__ __launch_bounds__(kBlock) void k_apply_step(ApplyArgs a) {
  apply_step_body<TR>(a, hw_block());
}
template <typename TR>
__global__ __launch_bounds__(kBlock) void k_apply_step_batch(const ApplyArgs* __restrict__ tab,
                                                             const uint32_t* __restrict__ starts,
                                                             int n) {
  VBlock vb;
  const int p = batch_volume(starts, n, vb);
  apply_step_body<TR>(tab[p], vb);
}

// Corrected images T[I+, b, v] and T[I-, b, -v] at the cell centres (Sec. 2.4.7).
template <typename TI, typename TR, int S>
__global__ __launch_bounds__(1024) void k_correct(CorrectArgs a) {
  const Geom g = a.g;
  const TI* __restrict__ Ip = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ Im = static_cast<const TI*>(a.Im);
  const TR* __restrict__ b = static_cast<const TR*>(a.b);
  TI* __restrict__ Tp = static_cast<TI*>(a.Tp);
  TI* __restrict__ Tm = static_cast<TI*>(a.Tm);
  const int mp = g.mp;
  const int64_t nct = (g.ncol + kWave - 1) / kWave;
  const int64_t ntiles = nct * ((mp + S - 1) / S);
  const int lane = threadIdx.x & (kWave - 1);
  const TR inv_hp = TR(1) / (TR)g.hp;
  for (WaveIter it = wave_iter(ntiles, hw_block()); it.t < it.end; it.t += it.stride) {
    const int64_t col = (it.t % nct) * kWave + lane;
    const int k0 = (int)(it.t / nct) * S;
    if (col >= g.ncol) continue;
    const int64_t nb = node_base(g, col);
    const int64_t cb = cell_base(g, col);
    TR bb[S + 1];
#pragma unroll
    for (int i = 0; i < S + 1; ++i) {
      int k = k0 + i;
      k = k > mp ? mp : k;
      bb[i] = b[nb + (int64_t)k * g.nps];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = k0 + s;
      if (j >= mp) break;
      const TR ab = (bb[s] + bb[s + 1]) * TR(0.5);
      const TR db = (bb[s + 1] - bb[s]) * inv_hp;
      const TR t = ab * inv_hp;
      TR vp, sp, vm, sm;
      interp_at(Ip, cb, g.cps, mp, j, t, inv_hp, vp, sp);
      interp_at(Im, cb, g.cps, mp, j, -t, inv_hp, vm, sm);
      const int64_t c = cb + (int64_t)j * g.cps;
      if (Tp) Tp[c] = from_real<TI>(vp * (TR(1) + db));
      if (Tm) Tm[c] = from_real<TI>(vm * (TR(1) - db));
    }
  }
}

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------

namespace {
// PE nodes per thread: short runs give more wavefronts and shorter dependent chains (measured on
// 144x168x111 and its coarser levels: loss_grad 4 on volumes above 1 M nodes, 2 below; the trial
// passes 2 everywhere; the correction 4).
constexpr int kRunTrial = 2;
constexpr int kRunCorrect = 4;
inline int loss_run(const Geom& g) { return g.nnode > (int64_t(1) << 20) ? 4 : 2; }
}

Launch plan_tiles(const Geom& g, int S, int block) {
  Launch L;
  L.S = S;
  L.block = (unsigned)block;
  const int64_t nct = (g.ncol + kWave - 1) / kWave;
  L.ntiles = nct * ((g.mp + 1 + S - 1) / S);
  const int64_t wpb = block / kWave;
  int64_t grid = (L.ntiles + wpb - 1) / wpb;
  if (grid > kMaxGrid) grid = kMaxGrid;
  grid = (grid + 7) / 8 * 8;  // whole XCD rounds (see wave_iter); spare blocks add zero sums
  if (grid > kMaxGrid) grid = kMaxGrid;
  L.grid = (unsigned)(grid < 1 ? 1 : grid);
  return L;
}

// 256-thread blocks; the grid holds one wavefront per tile up to kMaxGrid blocks (full
// occupancy matters more than anything else for these latency-heavy gathers and stencils).
static int pick_block(const Geom& g, DType real, int S) {
  (void)g;
  (void)real;
  (void)S;
  return 256;
}

// --------------------------------------------------------------------------------------------
// dJ/dI+ and dJ/dI- (only D depends on the images, Eq. 2): per column the residual r_j, weighted
// by vol (1 + D b_j) for I+ and -vol (1 - D b_j) for I-, is spread back onto the two samples that
// interpolate the image at xi+-_j (the adjoint of the linear image model, zero outside).  With
// |D b| < 1 the positions increase strictly along the column, so one thread walks its column once
// and emits every sample's total in order while holding at most two open samples: no atomics and
// every output written once.  (With |D b| >= 1 somewhere the output is unspecified.)
// --------------------------------------------------------------------------------------------
template <typename TR>
struct Spread {
  int kc, kw;     // open samples kc, kc + 1; samples below kw are written
  TR a0, a1;
};

template <typename TI, typename TR>
__global__ __launch_bounds__(kBlock) void k_image_grad(ImageGradArgs a) {
  const Geom g = a.g;
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= g.ncol) return;
  const TI* __restrict__ Ip = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ Im = static_cast<const TI*>(a.Im);
  const TR* __restrict__ b = static_cast<const TR*>(a.b);
  TR* __restrict__ gp = static_cast<TR*>(a.gIp);
  TR* __restrict__ gm = static_cast<TR*>(a.gIm);
  const int mp = g.mp;
  const int64_t cb = cell_base(g, col), nb = node_base(g, col);
  const int64_t cps = g.cps, nps = g.nps;
  const TR inv_hp = TR(1) / (TR)g.hp;
  const TR vol = (TR)g.vol;
  constexpr int kNone = -(1 << 30);

  auto emit = [&](TR* out, int& kw, int k, TR v) {
    if (k < kw || k >= mp) return;  // outside the column (or out of order)
    for (; kw < k; ++kw) out[cb + (int64_t)kw * cps] = TR(0);
    out[cb + (int64_t)k * cps] = v;
    kw = k + 1;
  };
  auto push = [&](Spread<TR>& e, TR* out, int k0, TR w, TR u) {
    if (k0 != e.kc) {
      if (e.kc != kNone) {
        emit(out, e.kw, e.kc, e.a0);
        if (k0 == e.kc + 1) {
          e.a0 = e.a1;
        } else {
          emit(out, e.kw, e.kc + 1, e.a1);
          e.a0 = TR(0);
        }
        e.a1 = TR(0);
      }
      e.kc = k0;
    }
    e.a0 += (TR(1) - w) * u;
    e.a1 += w * u;
  };
  Spread<TR> sp{kNone, 0, TR(0), TR(0)}, sm{kNone, 0, TR(0), TR(0)};
  TR b0 = b[nb];
  for (int j = 0; j < mp; ++j) {
    const TR b1 = b[nb + (int64_t)(j + 1) * nps];
    const TR ab = (b0 + b1) * TR(0.5);
    const TR db = (b1 - b0) * inv_hp;
    const TR t = ab * inv_hp;
    TR vp, slp, vm, slm;
    interp_at(Ip, cb, cps, mp, j, t, inv_hp, vp, slp);
    interp_at(Im, cb, cps, mp, j, -t, inv_hp, vm, slm);
    const TR r = vp * (TR(1) + db) - vm * (TR(1) - db);
    // the same interval as interp_at: k0 = j + floor(+-t), w = +-t - floor(+-t)
    TR fp = fmin(fmax(floor(t), TR(-mp - 2)), TR(mp + 2));
    TR fm = fmin(fmax(floor(-t), TR(-mp - 2)), TR(mp + 2));
    push(sp, gp, j + (int)fp, t - fp, vol * r * (TR(1) + db));
    push(sm, gm, j + (int)fm, -t - fm, -vol * r * (TR(1) - db));
    b0 = b1;
  }
  for (Spread<TR>* e : {&sp, &sm}) {
    TR* out = e == &sp ? gp : gm;
    if (e->kc != kNone) {
      emit(out, e->kw, e->kc, e->a0);
      emit(out, e->kw, e->kc + 1, e->a1);
    }
    for (; e->kw < mp; ++e->kw) out[cb + (int64_t)e->kw * cps] = TR(0);
  }
}

// loss_grad holds ~140 VGPRs (3 wavefronts per SIMD): a grid of one resident round (3 blocks of
// 4 wavefronts on each of the 256 CUs) leaves no tail round, and the consumers of its block sums
// (the PCG scalar phase of iteration 0) read 768 instead of 2048 of them.
Launch plan_loss_grad(const Geom& g, DType real) {
  Launch L = plan_tiles(g, loss_run(g), pick_block(g, real, loss_run(g)));
  if (L.grid > 768u) L.grid = 768u;
  return L;
}
// The first trial pass holds ~65 VGPRs (7 wavefronts per SIMD): one resident round is 7 blocks of
// 4 wavefronts per CU.
Launch plan_trial(const Geom& g, DType real, int nc) {
  Launch L = plan_tiles(g, kRunTrial, nc == 1 ? pick_block(g, real, kRunTrial) : 256);
  if (L.grid > 1792u) L.grid = 1792u;
  return L;
}


hipError_t launch_loss_grad(const LossGradArgs& a0, DType img, DType real, hipStream_t s) {
  const Launch L = plan_loss_grad(a0.g, real);
  LossGradArgs a = a0;
  a.run = L.S;
  // timing tag 1: the launch also applies the previous step (reads q, writes b + gamma q)
  const int tag = a.step ? 1 : 0;
  if (active_recorder()) {
    const hipError_t e = record_launch(RecKind::kLossGrad, a, L.grid, L.block, 0, (int)img, (int)real, 0,
                  [a, img, real](hipStream_t s2) { return launch_loss_grad(a, img, real, s2); });
    if (e != hipSuccess) return e;
    return note_volume(a.g.ncell, a.g.nnode, tag);
  }
#define RGP_LG(RUN, STEP)                                                                    \
  RGP_DISPATCH_TYPES(img, real, RGP_LAUNCH_T(kKindLossGrad, tag, a.g,                        \
                                             (k_loss_grad<TI, TR, RUN, 256, STEP>), L.grid,  \
                                             256, 0, s, a))
  if (L.S == 4) {
    if (a.step)
      RGP_LG(4, true);
    else
      RGP_LG(4, false);
  } else {
    if (a.step)
      RGP_LG(2, true);
    else
      RGP_LG(2, false);
  }
#undef RGP_LG
  return hipGetLastError();
}

hipError_t launch_loss_final(const LossFinalArgs& a, hipStream_t s) {
  if (active_recorder())
    return record_other([a](hipStream_t s2) { return launch_loss_final(a, s2); });
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kReduceBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_trial(const TrialArgs& a, DType img, DType real, hipStream_t s) {
  const Launch L = plan_trial(a.g, real, a.nc);
  if (active_recorder()) {
    const hipError_t e = record_launch(RecKind::kTrial, a, L.grid, L.block, 0, (int)img, (int)real, a.nc,
                  [a, img, real](hipStream_t s2) { return launch_trial(a, img, real, s2); });
    if (e != hipSuccess) return e;
    return note_volume(a.g.ncell, a.g.nnode, a.nc);
  }
#define RGP_TRIAL_P(NC, B, P)                                                              \
  RGP_DISPATCH_TYPES(img, real, RGP_LAUNCH_T(kKindTrial, NC, a.g,                          \
                                             (k_trial<TI, TR, kRunTrial, NC, B, P>), L.grid, B, \
                                             0, s, a))
  // only the first pass (one candidate, first == 0) forms grad.q and the S cross sums
  if (a.first == 0 && a.nc != 1) return hipErrorInvalidValue;
  switch (a.nc) {
    case 1:
      if (a.first == 0) {
        if (L.block == 1024) RGP_TRIAL_P(1, 1024, true);
        else RGP_TRIAL_P(1, 256, true);
      } else {
        RGP_TRIAL_P(1, 256, false);
      }
      break;
    case 2: RGP_TRIAL_P(2, 256, false); break;
    case 3: RGP_TRIAL_P(3, 256, false); break;
    case 4: RGP_TRIAL_P(4, 256, false); break;
    case 5: RGP_TRIAL_P(5, 256, false); break;
    case 6: RGP_TRIAL_P(6, 256, false); break;
    case 7: RGP_TRIAL_P(7, 256, false); break;
    case 8: RGP_TRIAL_P(8, 256, false); break;
    case 9: RGP_TRIAL_P(9, 256, false); break;
    default: return hipErrorInvalidValue;
  }
#undef RGP_TRIAL_P
  return hipGetLastError();
}

hipError_t launch_decide(const DecideArgs& a, hipStream_t s) {
  if (active_recorder())
    return record_launch(RecKind::kDecide, a, 1, kReduceBlock, 0, a.prev_nc, 0, 0,
                         [a](hipStream_t s2) { return launch_decide(a, s2); });
#define RGP_DECIDE(NC) hipLaunchKernelGGL(k_decide<NC>, dim3(1), dim3(kReduceBlock), 0, s, a)
  switch (a.prev_nc) {
    case 1: RGP_DECIDE(1); break;
    case 2: RGP_DECIDE(2); break;
    case 3: RGP_DECIDE(3); break;
    case 4: RGP_DECIDE(4); break;
    case 5: RGP_DECIDE(5); break;
    case 6: RGP_DECIDE(6); break;
    case 7: RGP_DECIDE(7); break;
    case 8: RGP_DECIDE(8); break;
    case 9: RGP_DECIDE(9); break;
    default: return hipErrorInvalidValue;
  }
#undef RGP_DECIDE
  return hipGetLastError();
}

hipError_t launch_apply_step(const ApplyArgs& a, DType real, hipStream_t s) {
  const unsigned nb = (unsigned)((a.n + kBlock - 1) / kBlock);
  if (active_recorder())
    return record_launch(RecKind::kApply, a, nb, kBlock, 0, (int)real, 0, 0,
                         [a, real](hipStream_t s2) { return launch_apply_step(a, real, s2); });
  if (real == DType::F64)
    hipLaunchKernelGGL(k_apply_step<double>, dim3(nb), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_apply_step<float>, dim3(nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_correct(const CorrectArgs& a, DType img, DType real, hipStream_t s) {
  if (active_recorder())
    return record_other([a, img, real](hipStream_t s2) { return launch_correct(a, img, real, s2); });
  Launch L = plan_tiles(a.g, kRunCorrect, 1024);
  RGP_DISPATCH_TYPES(img, real, hipLaunchKernelGGL((k_correct<TI, TR, kRunCorrect>), dim3(L.grid),
                                                   dim3(1024), 0, s, a));
  return hipGetLastError();
}

hipError_t launch_image_grad(const ImageGradArgs& a, DType img, DType real, hipStream_t s) {
  if (active_recorder())
    return record_other([a, img, real](hipStream_t s2) { return launch_image_grad(a, img, real, s2); });
  const unsigned nb = (unsigned)((a.g.ncol + kBlock - 1) / kBlock);
  RGP_DISPATCH_TYPES(img, real, hipLaunchKernelGGL((k_image_grad<TI, TR>), dim3(nb),
                                                   dim3(kBlock), 0, s, a));
  return hipGetLastError();
}

// ---- shared launches over several volumes -----------------------------------------------------

hipError_t launch_loss_grad_batch(const void* tab, const uint32_t* starts, int n, unsigned grid,
                                  DType img, DType real, int64_t cells, int64_t nodes, int tag,
                                  hipStream_t s) {
  const LossGradArgs* t = static_cast<const LossGradArgs*>(tab);
  RGP_DISPATCH_TYPES(img, real, RGP_LAUNCH_TN(kKindLossGrad, tag, cells, nodes,
                                              (k_loss_grad_batch<TI, TR, 256>), grid, 256, 0, s,
                                              t, starts, n));
  return hipGetLastError();
}

hipError_t launch_trial_batch(const void* tab, const uint32_t* starts, int n, unsigned grid,
                              int nc, DType img, DType real, int64_t cells, int64_t nodes,
                              hipStream_t s) {
  const TrialArgs* t = static_cast<const TrialArgs*>(tab);
#define RGP_TRIAL_B(NC)                                                                      \
  RGP_DISPATCH_TYPES(img, real, RGP_LAUNCH_TN(kKindTrial, NC, cells, nodes,                  \
                                              (k_trial_batch<TI, TR, kRunTrial, NC, 256>), grid, \
                                              256, 0, s, t, starts, n))
  switch (nc) {
    case 1: RGP_TRIAL_B(1); break;
    case 2: RGP_TRIAL_B(2); break;
    case 3: RGP_TRIAL_B(3); break;
    case 4: RGP_TRIAL_B(4); break;
    case 5: RGP_TRIAL_B(5); break;
    case 6: RGP_TRIAL_B(6); break;
    case 7: RGP_TRIAL_B(7); break;
    case 8: RGP_TRIAL_B(8); break;
    case 9: RGP_TRIAL_B(9); break;
    default: return hipErrorInvalidValue;
  }
#undef RGP_TRIAL_B
  return hipGetLastError();
}

hipError_t launch_decide_batch(const void* tab, int n, int nc, hipStream_t s) {
  const DecideArgs* t = static_cast<const DecideArgs*>(tab);
#define RGP_DECIDE_B(NC) hipLaunchKernelGGL(k_decide_batch<NC>, dim3(n), dim3(kReduceBlock), 0, s, t)
  switch (nc) {
    case 1: RGP_DECIDE_B(1); break;
    case 2: RGP_DECIDE_B(2); break;
    case 3: RGP_DECIDE_B(3); break;
    case 4: RGP_DECIDE_B(4); break;
    case 5: RGP_DECIDE_B(5); break;
    case 6: RGP_DECIDE_B(6); break;
    case 7: RGP_DECIDE_B(7); break;
    case 8: RGP_DECIDE_B(8); break;
    case 9: RGP_DECIDE_B(9); break;
    default: return hipErrorInvalidValue;
  }
#undef RGP_DECIDE_B
  return hipGetLastError();
}

hipError_t launch_apply_step_batch(const void* tab, const uint32_t* starts, int n, unsigned grid,
                                   DType real, hipStream_t s) {
  const ApplyArgs* t = static_cast<const ApplyArgs*>(tab);
  if (real == DType::F64)
    hipLaunchKernelGGL(k_apply_step_batch<double>, dim3(grid), dim3(kBlock), 0, s, t, starts, n);
  else
    hipLaunchKernelGGL(k_apply_step_batch<float>, dim3(grid), dim3(kBlock), 0, s, t, starts, n);
  return hipGetLastError();
}

}  // namespace rgp
