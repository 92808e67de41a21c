// Device-side scalar logic of the Gauss-Newton solve shared by several kernels: the reduction of
// loss_grad's block sums into J = D + alpha S + beta P, the Armijo decision, and stats records.
#pragma once

#include "rgp_internal.hpp"
#include "rgp_launch.hpp"

namespace rgp {

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

// Reduces loss_grad's block sums (every thread of the block calls this); returns true when the
// barrier is violated (J = +inf).  Thread 0 of the block writes the state when `write` is set.
__device__ __forceinline__ int load_flag(const int32_t* f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// J, D, S, P from the reduced block sums t of loss_grad; thread 0 of the calling block writes the
// state when `write` is set.  Returns true when the barrier is violated (J = +inf).
__device__ __forceinline__ bool finalize_loss_sums(const LossFinalArgs& a, const double (&t)[5],
                                                   bool write) {
  const bool viol = t[3] > 0.0;
  if (write && threadIdx.x == 0) {
    State* st = a.st;
    const double D = 0.5 * a.vol * t[0];
    const double S = 0.5 * a.vol * t[1];
    const double P = viol ? inf_d() : 0.5 * a.vol * t[2];
    const double J = D + a.alpha * S + a.beta * P;
    st->J = J;
    st->D = D;
    st->S = S;
    st->P = P;
    st->gnorm2 = t[4];
    st->accepted = 0;
    st->gamma = 0.0;
    st->trials = 0;
    st->gq = 0.0;
    st->pcg_iters = 0;
    st->relres = 0.0;
    if (a.gn_mode && viol) {
      __hip_atomic_store(&st->gn_stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (st->status == 0) st->status = RGP_EBARRIER;
      if (a.record) write_record(a.record, *st);
    }
    if (a.jdsp) {
      a.jdsp[0] = J;
      a.jdsp[1] = D;
      a.jdsp[2] = S;
      a.jdsp[3] = P;
    }
  }
  return viol;
}

// One block of kReduceBlock threads: reduces loss_grad's block sums and finalises them.
__device__ __forceinline__ bool finalize_loss(const LossFinalArgs& a, bool write) {
  double t[5];
  reduce_partials<5, kReduceBlock>(t, a.part, a.nprod);
  return finalize_loss_sums(a, t, write);
}

// Trial-pass block sums: [0] grad.q, [1] sum dB.dQ/h^2, [2] sum dQ^2/h^2 (first pass only),
// then per candidate c: [3+3c] sum r^2, [4+3c] sum phi, [5+3c] barrier violations.  At most
// kMaxTrialCand candidates per pass.
constexpr int kTrialSlots = 3 + 3 * kMaxTrialCand;

// Armijo decision over one pass (first index `first`, `nc` candidates): the largest gamma with
// J(b + gamma q) <= J(b) + c gamma grad.q.  Returns the candidate index or -1.
template <int NC>
__device__ __forceinline__ int armijo_pick(const double* t, int first, int nc, const State& st,
                                           double gq, double sbq, double sqq, double vol,
                                           double alpha, double beta, double c, double& gamma) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {  // unrolled: t stays in registers
    if (k >= nc) break;
    const double gm = ldexp(1.0, -(first + k));
    const double D = 0.5 * vol * t[3 + 3 * k];
    const double P = t[5 + 3 * k] > 0.0 ? inf_d() : 0.5 * vol * t[4 + 3 * k];
    const double S = st.S + gm * vol * sbq + 0.5 * gm * gm * vol * sqq;
    const double J = D + alpha * S + beta * P;
    if (J <= st.J + c * gm * gq) {
      gamma = gm;
      return k;
    }
  }
  return -1;
}

// Decision on one finished pass of NC candidates, taken by a single-block kernel from the state
// s and each thread's share t of the pass's 3 + 3 NC block sums (partials_share): the block adds
// the shares, then thread 0 updates the state.  Returns 1 when a step was accepted, 0 when the
// search continues, -1 when it failed (no trials left).
template <int NC>
__device__ __forceinline__ int decide_pass(const DecideArgs& a, const State& s,
                                           double (&t)[3 + 3 * NC]) {
  State* st = a.st;
  block_sum<3 + 3 * NC, kReduceBlock>(t);  // synchronises
  double gq = s.gq, sbq = s.sbq, sqq = s.sqq;
  if (a.prev_first == 0) {
    gq = t[0];
    sbq = t[1];
    sqq = t[2];
  }
  double gamma = 0.0;
  const int k = armijo_pick<NC>(t, a.prev_first, a.prev_nc, s, gq, sbq, sqq, a.vol, a.alpha,
                                a.beta, a.armijo_c, gamma);
  const bool last = a.prev_first + a.prev_nc >= a.total;
  const int res = k >= 0 ? 1 : (last ? -1 : 0);
  if (threadIdx.x == 0) {
    State n = s;
    n.gq = gq;
    n.sbq = sbq;
    n.sqq = sqq;
    if (res == 1) {
      n.accepted = 1;
      n.gamma = gamma;
      n.trials = a.prev_first + k + 1;
    } else if (res == -1) {
      n.accepted = 0;
      n.gamma = 0.0;
      n.gn_stop = 1;
      n.trials = a.total;
      if (n.status == 0) n.status = RGP_ELINESEARCH;
    }
    *st = n;
    if (res != 0 && a.record) write_record(a.record, n);
  }
  return res;
}

}  // namespace rgp
