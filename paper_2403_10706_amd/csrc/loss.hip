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

// phi(z) = z^4/(1-z^2), phi', phi'' (Eq. 3); valid for |z| < 1.
template <typename TR>
__device__ __forceinline__ void phi3(TR z, TR& f, TR& f1, TR& f2) {
  const TR z2 = z * z;
  const TR q = TR(1) - z2;
  const TR iq = TR(1) / q;
  f = z2 * z2 * iq;
  f1 = TR(2) * z2 * z * (TR(2) - z2) * iq * iq;
  f2 = TR(2) * z2 * (TR(6) - TR(3) * z2 + z2 * z2) * iq * iq * iq;
}

__device__ __forceinline__ void write_record(double* rec, const State& s) {
  rec[0] = s.J;
  rec[1] = s.D;
  rec[2] = s.S;
  rec[3] = s.P;
  rec[4] = sqrt(s.gnorm2);
  rec[5] = s.gq;
  rec[6] = (double)s.pcg_iters;
  rec[7] = s.relres;
  rec[8] = s.accepted ? s.gamma : 0.0;
  rec[9] = (double)s.trials;
  rec[10] = (double)s.accepted;
  rec[11] = 0.0;
}

// --------------------------------------------------------------------------------------------
// loss_grad: J, D, S, P; optionally grad J and the GN tridiagonal (diag, off).  With step != 0
// the kernel first forms b = b_in + gamma q (gamma from the line search state) and writes it to
// b_out (a different buffer: neighbours read b_in concurrently).
// --------------------------------------------------------------------------------------------
template <typename TI, typename TR, int S>
__global__ __launch_bounds__(kBlock) void k_loss_grad(LossGradArgs a) {
  const Geom g = a.g;
  const TI* __restrict__ Ip = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ Im = static_cast<const TI*>(a.Im);
  const TR* __restrict__ bin = static_cast<const TR*>(a.b_in);
  const TR* __restrict__ q = static_cast<const TR*>(a.q);
  TR* __restrict__ bout = static_cast<TR*>(a.b_out);
  TR* __restrict__ grad = static_cast<TR*>(a.grad);
  TR* __restrict__ diag = static_cast<TR*>(a.diag);
  TR* __restrict__ off = static_cast<TR*>(a.off);
  State* st = a.st;

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
  const int64_t cb = ix * g.cxs + iy * g.cys;

  // Step application (Gauss-Newton update of the previous iteration).
  TR coef = TR(0);
  if (a.step) {
    if (st->gn_stop) {  // solve stopped at this level: carry b over unchanged
      for (int s = 0; s < S; ++s) {
        const int k = k0 + s;
        if (colok && k <= mp) bout[nb + (int64_t)k * g.nps] = bin[nb + (int64_t)k * g.nps];
      }
      return;
    }
    coef = st->accepted ? (TR)st->gamma : TR(0);
  }

  auto ldb = [&](int64_t n) -> TR {
    TR v = bin[n];
    if (a.step) v += coef * q[n];
    return v;
  };

  const TR inv_hp = TR(1) / (TR)g.hp;
  const TR wp2 = TR(1) / ((TR)g.hp * (TR)g.hp);
  const TR wx2 = TR(1) / ((TR)g.hx * (TR)g.hx);
  const TR wy2 = TR(1) / ((TR)g.hy * (TR)g.hy);
  const TR vol = (TR)g.vol;
  const TR avol = (TR)(a.alpha * g.vol);
  const TR bh = (TR)(0.5 * a.beta * g.vol);

  // b at nodes k0-1 .. k0+S (index i <-> node k0-1+i), clamped into the column.
  TR bb[S + 2];
#pragma unroll
  for (int i = 0; i < S + 2; ++i) {
    int k = k0 - 1 + i;
    k = k < 0 ? 0 : (k > mp ? mp : k);
    bb[i] = ldb(nb + (int64_t)k * g.nps);
  }

  double accD = 0.0, accS = 0.0, accP = 0.0, accV = 0.0, accG = 0.0;

  // Right-hand contributions of cell k0-1 to node k0.
  TR gR = TR(0), dR = TR(0);
  {
    const int j = k0 - 1;
    if (j >= 0 && j < mp) {
      const CellOut<TR> c = eval_cell(Ip, Im, cb, g.cps, mp, j, bb[0], bb[1], inv_hp);
      TR f, f1, f2;
      if (fabs(c.db) < TR(1)) {
        phi3(c.db, f, f1, f2);
      } else {
        f = f1 = f2 = TR(0);
      }
      gR = vol * c.r * c.u1 + bh * f1 * inv_hp;
      dR = vol * c.u1 * c.u1 + bh * f2 * wp2;
    }
  }

#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int k = k0 + s;
    const bool nodeok = k <= mp;
    const TR bk = bb[s + 1];
    // y neighbours through lane shuffles; the first/last lane of the wave loads from memory.
    TR bym = __shfl_up(bk, 1, kWave);
    TR byp = __shfl_down(bk, 1, kWave);
    const bool hasym = iy > 0, hasyp = iy < g.ny - 1;
    const bool hasxm = ix > 0, hasxp = ix < g.nx - 1;
    const int kc = nodeok ? k : mp;
    const int64_t n = nb + (int64_t)kc * g.nps;
    if (lane == 0 && hasym) bym = ldb(n - g.nys);
    if (lane == kWave - 1 && hasyp) byp = ldb(n + g.nys);
    const TR bxm = hasxm ? ldb(n - g.nxs) : bk;
    const TR bxp = hasxp ? ldb(n + g.nxs) : bk;

    // Own cell k (left contributions to node k).
    TR gL = TR(0), dL = TR(0), oc = TR(0);
    TR nR = TR(0), ndR = TR(0);
    if (nodeok && k < mp) {
      const CellOut<TR> c = eval_cell(Ip, Im, cb, g.cps, mp, k, bk, bb[s + 2], inv_hp);
      TR f, f1, f2;
      if (fabs(c.db) < TR(1)) {
        phi3(c.db, f, f1, f2);
      } else {
        f = f1 = f2 = TR(0);
        accV += colok ? 1.0 : 0.0;
      }
      gL = vol * c.r * c.u0 - bh * f1 * inv_hp;
      dL = vol * c.u0 * c.u0 + bh * f2 * wp2;
      oc = vol * c.u0 * c.u1 - bh * f2 * wp2 - avol * wp2;
      nR = vol * c.r * c.u1 + bh * f1 * inv_hp;
      ndR = vol * c.u1 * c.u1 + bh * f2 * wp2;
      if (colok) {
        accD += (double)c.r * (double)c.r;
        accP += (double)f;
      }
    }
    if (nodeok) {
      // Laplacian (Neumann) at node k and the forward differences of S.
      TR lap = TR(0), ldg = TR(0);
      double sterm = 0.0;
      if (k > 0) {
        lap += (bk - bb[s]) * wp2;
        ldg += wp2;
      }
      if (k < mp) {
        const TR d = bb[s + 2] - bk;
        lap -= d * wp2;
        ldg += wp2;
        sterm += (double)(d * d * wp2);
      }
      if (hasxm) { lap += (bk - bxm) * wx2; ldg += wx2; }
      if (hasxp) {
        const TR d = bxp - bk;
        lap -= d * wx2;
        ldg += wx2;
        sterm += (double)(d * d * wx2);
      }
      if (hasym) { lap += (bk - bym) * wy2; ldg += wy2; }
      if (hasyp) {
        const TR d = byp - bk;
        lap -= d * wy2;
        ldg += wy2;
        sterm += (double)(d * d * wy2);
      }
      const TR gk = gR + gL + avol * lap;
      if (colok) {
        accS += sterm;
        accG += (double)gk * (double)gk;
        if (grad) grad[n] = gk;
        if (diag) {
          diag[n] = dR + dL + avol * ldg;
          off[n] = (k < mp) ? oc : TR(0);
        }
        if (bout) bout[n] = bk;
      }
    }
    gR = nR;
    dR = ndR;
  }

  double v[5] = {accD, accS, accP, accV, accG};
  if (publish_partials<5>(v, a.partials, a.counter, bid, nblocks)) {
    double t[5];
    reduce_partials<5>(t, a.partials, nblocks);
    if (threadIdx.x == 0) {
      const double D = 0.5 * g.vol * t[0];
      const double Sv = 0.5 * g.vol * t[1];
      const double P = t[3] > 0.0 ? inf_d() : 0.5 * g.vol * t[2];
      const double J = D + a.alpha * Sv + a.beta * P;
      st->J = J;
      st->D = D;
      st->S = Sv;
      st->P = P;
      st->gnorm2 = t[4];
      st->accepted = 0;
      st->gamma = 0.0;
      st->trials = 0;
      st->gq = 0.0;
      st->pcg_status = kPcgRunning;
      st->pcg_iters = 0;
      st->relres = 0.0;
      if (a.gn_mode) {
        st->gn_stop = (t[3] > 0.0) ? 1 : 0;
        if (st->gn_stop && a.record) write_record(a.record, *st);
      }
      if (a.jdsp) {
        a.jdsp[0] = J;
        a.jdsp[1] = D;
        a.jdsp[2] = Sv;
        a.jdsp[3] = P;
      }
      *a.counter = 0u;
    }
  }
}

// --------------------------------------------------------------------------------------------
// Armijo trials: J(b + gamma_c q) for NC step sizes gamma_c = 2^-(first + c), c = 0..NC-1, in
// one pass.  S(b + gamma q) = S + gamma vol sum(dB dQ)/h^2 + gamma^2 (vol/2) sum(dQ^2)/h^2 is
// exact, so only D and P are evaluated per candidate; the pass with first == 0 also forms grad.q
// and the two S sums.  The first (largest) gamma satisfying the Armijo condition is taken,
// which is exactly what halving from gamma = 1 selects.
// --------------------------------------------------------------------------------------------
template <typename TI, typename TR, int S, int NC>
__global__ __launch_bounds__(kBlock) void k_trial(TrialArgs a) {
  State* st = a.st;
  if (st->gn_stop) return;
  if (a.first > 0 && st->accepted) return;
  const Geom g = a.g;
  const TI* __restrict__ Ip = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ Im = static_cast<const TI*>(a.Im);
  const TR* __restrict__ b = static_cast<const TR*>(a.b);
  const TR* __restrict__ q = static_cast<const TR*>(a.q);
  const TR* __restrict__ gr = static_cast<const TR*>(a.grad);

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
  const int64_t cb = ix * g.cxs + iy * g.cys;
  const bool pass0 = a.first == 0;

  const TR inv_hp = TR(1) / (TR)g.hp;
  const TR wp2 = TR(1) / ((TR)g.hp * (TR)g.hp);
  const TR wx2 = TR(1) / ((TR)g.hx * (TR)g.hx);
  const TR wy2 = TR(1) / ((TR)g.hy * (TR)g.hy);

  TR bb[S + 1], qq[S + 1];
#pragma unroll
  for (int i = 0; i < S + 1; ++i) {
    int k = k0 + i;
    k = k > mp ? mp : k;
    bb[i] = b[nb + (int64_t)k * g.nps];
    qq[i] = q[nb + (int64_t)k * g.nps];
  }
  TR gam[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) gam[c] = (TR)ldexp(1.0, -(a.first + c));

  constexpr int K = 3 * NC + 3;
  double v[K];
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = 0.0;

#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int k = k0 + s;
    const bool nodeok = k <= mp;
    if (pass0) {
      const TR bk = bb[s], qk = qq[s];
      TR byp = __shfl_down(bk, 1, kWave);
      TR qyp = __shfl_down(qk, 1, kWave);
      const int kc = nodeok ? k : mp;
      const int64_t n = nb + (int64_t)kc * g.nps;
      const bool hasyp = iy < g.ny - 1, hasxp = ix < g.nx - 1;
      if (lane == kWave - 1 && hasyp) {
        byp = b[n + g.nys];
        qyp = q[n + g.nys];
      }
      if (nodeok && colok) {
        double sbq = 0.0, sqq = 0.0;
        if (k < mp) {
          const TR db = bb[s + 1] - bk, dq = qq[s + 1] - qk;
          sbq += (double)(db * dq * wp2);
          sqq += (double)(dq * dq * wp2);
        }
        if (hasxp) {
          const TR db = b[n + g.nxs] - bk, dq = q[n + g.nxs] - qk;
          sbq += (double)(db * dq * wx2);
          sqq += (double)(dq * dq * wx2);
        }
        if (hasyp) {
          const TR db = byp - bk, dq = qyp - qk;
          sbq += (double)(db * dq * wy2);
          sqq += (double)(dq * dq * wy2);
        }
        v[3 * NC + 0] += (double)gr[n] * (double)qk;
        v[3 * NC + 1] += sbq;
        v[3 * NC + 2] += sqq;
      }
    }
    if (nodeok && k < mp && colok) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const TR b0 = bb[s] + gam[c] * qq[s];
        const TR b1 = bb[s + 1] + gam[c] * qq[s + 1];
        const TR ab = (b0 + b1) * TR(0.5);
        const TR db = (b1 - b0) * inv_hp;
        const TR t = ab * inv_hp;
        TR vp, sp, vm, sm;
        interp_at(Ip, cb, g.cps, mp, k, t, inv_hp, vp, sp);
        interp_at(Im, cb, g.cps, mp, k, -t, inv_hp, vm, sm);
        const TR r = vp * (TR(1) + db) - vm * (TR(1) - db);
        v[3 * c + 0] += (double)r * (double)r;
        if (fabs(db) < TR(1)) {
          const TR z2 = db * db;
          v[3 * c + 1] += (double)(z2 * z2 / (TR(1) - z2));
        } else {
          v[3 * c + 2] += 1.0;
        }
      }
    }
  }

  if (publish_partials<K>(v, a.partials, a.counter, bid, nblocks)) {
    double t[K];
    reduce_partials<K>(t, a.partials, nblocks);
    if (threadIdx.x == 0) {
      if (pass0) {
        st->gq = t[3 * NC + 0];
        st->sbq = t[3 * NC + 1];
        st->sqq = t[3 * NC + 2];
      }
      const double gq = st->gq, sbq = st->sbq, sqq = st->sqq;
      int acc = -1;
      double gacc = 0.0;
      for (int c = 0; c < NC; ++c) {
        const double gm = ldexp(1.0, -(a.first + c));
        const double D = 0.5 * g.vol * t[3 * c + 0];
        const double P = t[3 * c + 2] > 0.0 ? inf_d() : 0.5 * g.vol * t[3 * c + 1];
        const double Sg = st->S + gm * g.vol * sbq + 0.5 * gm * gm * g.vol * sqq;
        const double J = D + a.alpha * Sg + a.beta * P;
        if (J <= st->J + a.armijo_c * gm * gq) {
          acc = c;
          gacc = gm;
          break;
        }
      }
      if (acc >= 0) {
        st->accepted = 1;
        st->gamma = gacc;
        st->trials = a.first + acc + 1;
        if (a.record) write_record(a.record, *st);
      } else if (a.last_pass) {
        st->accepted = 0;
        st->gamma = 0.0;
        st->gn_stop = 1;
        st->trials = a.first + NC;
        if (a.record) write_record(a.record, *st);
      }
      *a.counter = 0u;
    }
  }
}

// b <- b + gamma q (in place, pointwise) with the accepted line-search step.
template <typename TR>
__global__ __launch_bounds__(kBlock) void k_apply_step(ApplyArgs a) {
  const State* st = a.st;
  if (st->gn_stop || !st->accepted) return;
  const TR gam = (TR)st->gamma;
  TR* __restrict__ b = static_cast<TR*>(a.b);
  const TR* __restrict__ q = static_cast<const TR*>(a.q);
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < a.n) b[i] = b[i] + gam * q[i];
}

// Corrected images T[I+, b, v] and T[I-, b, -v] at the cell centres (Sec. 2.4.7).
template <typename TI, typename TR, int S>
__global__ __launch_bounds__(kBlock) void k_correct(CorrectArgs a) {
  const Geom g = a.g;
  const TI* __restrict__ Ip = static_cast<const TI*>(a.Ip);
  const TI* __restrict__ Im = static_cast<const TI*>(a.Im);
  const TR* __restrict__ b = static_cast<const TR*>(a.b);
  TI* __restrict__ Tp = static_cast<TI*>(a.Tp);
  TI* __restrict__ Tm = static_cast<TI*>(a.Tm);
  const unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t nct = (g.ncol + kWave - 1) / kWave;
  const int64_t coltile = bid % nct;
  const int64_t petile = bid / nct;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int64_t col = coltile * kWave + lane;
  if (col >= g.ncol) return;
  const int64_t ix = col / g.ny, iy = col - (col / g.ny) * g.ny;
  const int k0 = (int)((petile * kWaves + wv) * S);
  const int mp = g.mp;
  if (k0 >= mp) return;
  const int64_t nb = ix * g.nxs + iy * g.nys;
  const int64_t cb = ix * g.cxs + iy * g.cys;
  const TR inv_hp = TR(1) / (TR)g.hp;
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

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------

namespace {
constexpr int kRun = 8;  // nodes per thread along the PE axis

unsigned col_run_blocks(const Geom& g, int run) {
  const int64_t nct = (g.ncol + kWave - 1) / kWave;
  const int64_t npt = (g.mp + 1 + kWaves * run - 1) / (kWaves * run);
  return (unsigned)(nct * npt);
}
}  // namespace

unsigned loss_grad_blocks(const Geom& g) { return col_run_blocks(g, kRun); }
unsigned trial_blocks(const Geom& g) { return col_run_blocks(g, kRun); }

#define RGP_DISPATCH_TYPES(IMG, REAL, ...)                                              \
  do {                                                                                  \
    if ((REAL) == DType::F64 && (IMG) == DType::F64) {                                  \
      using TI = double; using TR = double; __VA_ARGS__;                                \
    } else if ((REAL) == DType::F32 && (IMG) == DType::F32) {                           \
      using TI = float; using TR = float; __VA_ARGS__;                                  \
    } else if ((REAL) == DType::F32 && (IMG) == DType::BF16) {                          \
      using TI = bf16_t; using TR = float; __VA_ARGS__;                                 \
    } else if ((REAL) == DType::F64 && (IMG) == DType::F32) {                           \
      using TI = float; using TR = double; __VA_ARGS__;                                 \
    } else if ((REAL) == DType::F64 && (IMG) == DType::BF16) {                          \
      using TI = bf16_t; using TR = double; __VA_ARGS__;                                \
    } else {                                                                            \
      return hipErrorInvalidValue;                                                      \
    }                                                                                   \
  } while (0)

hipError_t launch_loss_grad(const LossGradArgs& a, DType img, DType real, hipStream_t s) {
  const unsigned nb = loss_grad_blocks(a.g);
  RGP_DISPATCH_TYPES(img, real, hipLaunchKernelGGL((k_loss_grad<TI, TR, kRun>), dim3(nb),
                                                   dim3(kBlock), 0, s, a));
  return hipGetLastError();
}

hipError_t launch_trial(const TrialArgs& a, int ncand, DType img, DType real, hipStream_t s) {
  const unsigned nb = trial_blocks(a.g);
#define RGP_TRIAL(NC)                                                                     \
  RGP_DISPATCH_TYPES(img, real, hipLaunchKernelGGL((k_trial<TI, TR, kRun, NC>), dim3(nb),  \
                                                   dim3(kBlock), 0, s, a))
  switch (ncand) {
    case 1: RGP_TRIAL(1); break;
    case 2: RGP_TRIAL(2); break;
    case 3: RGP_TRIAL(3); break;
    case 4: RGP_TRIAL(4); break;
    case 5: RGP_TRIAL(5); break;
    default: return hipErrorInvalidValue;
  }
#undef RGP_TRIAL
  return hipGetLastError();
}

hipError_t launch_apply_step(const ApplyArgs& a, DType real, hipStream_t s) {
  const unsigned nb = (unsigned)((a.n + kBlock - 1) / kBlock);
  if (real == DType::F64)
    hipLaunchKernelGGL(k_apply_step<double>, dim3(nb), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_apply_step<float>, dim3(nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_correct(const CorrectArgs& a, DType img, DType real, hipStream_t s) {
  const unsigned nb = col_run_blocks(a.g, kRun);
  RGP_DISPATCH_TYPES(img, real, hipLaunchKernelGGL((k_correct<TI, TR, kRun>), dim3(nb),
                                                   dim3(kBlock), 0, s, a));
  return hipGetLastError();
}

}  // namespace rgp
