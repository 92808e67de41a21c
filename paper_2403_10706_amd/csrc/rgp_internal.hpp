// Internal device-side definitions shared by the HIP kernels of librgp (gfx950).
//
// Layout conventions (caller arrays, C-contiguous [m0][m1][m2]):
//   * images are cell-centred, m0*m1*m2 values;
//   * the field map and every vector of the Gauss-Newton solve lives on the e_pe-staggered grid
//     (cell centres across the phase-encoding axis, nodes along it: m[pe]+1 of them), as in the
//     discretisation of Sec. 2.1 of the paper.
// A "column" is one line along the phase-encoding (PE) axis.  The two other axes are called x
// (the slower one) and y (the faster one); columns are enumerated col = ix*ny + iy so that
// consecutive lanes of a wavefront touch consecutive addresses whenever the PE axis is not the
// contiguous one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rgp {

constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kBlock = 256;       // threads per workgroup (4 wavefronts)
constexpr int kWaves = kBlock / kWave;

// bfloat16 image storage: upper 16 bits of an IEEE binary32.
struct bf16_t {
  uint16_t bits;
};

__device__ __forceinline__ float to_real(bf16_t v, float) {
  return __uint_as_float(static_cast<uint32_t>(v.bits) << 16);
}
__device__ __forceinline__ double to_real(bf16_t v, double) {
  return static_cast<double>(__uint_as_float(static_cast<uint32_t>(v.bits) << 16));
}
__device__ __forceinline__ float to_real(float v, float) { return v; }
__device__ __forceinline__ double to_real(float v, double) { return static_cast<double>(v); }
__device__ __forceinline__ float to_real(double v, float) { return static_cast<float>(v); }
__device__ __forceinline__ double to_real(double v, double) { return v; }

// Geometry of one volume on one pyramid level.
struct Geom {
  int32_t mp;       // cells along the PE axis (nodes: mp + 1)
  int32_t nx, ny;   // cells along the two cross axes (x slower than y in memory)
  int32_t pe;       // PE axis in caller order
  int64_t ncol;     // nx * ny columns
  int64_t cxs, cys, cps;  // cell (image) strides of x, y and PE
  int64_t nxs, nys, nps;  // node (field) strides of x, y and PE
  int64_t ncell, nnode;
  double hx, hy, hp, vol;
};

__host__ __device__ inline int64_t cell_base(const Geom& g, int64_t col) {
  const int64_t ix = col / g.ny, iy = col - (col / g.ny) * g.ny;
  return ix * g.cxs + iy * g.cys;
}
__host__ __device__ inline int64_t node_base(const Geom& g, int64_t col) {
  const int64_t ix = col / g.ny, iy = col - (col / g.ny) * g.ny;
  return ix * g.nxs + iy * g.nys;
}

// Per-pair device scalars of the solver.  All reductions are accumulated in FP64 in a fixed
// order, so results are bitwise reproducible run to run.
struct State {
  // objective at the current iterate
  double J, D, S, P, gnorm2;
  // line search
  double gq, sbq, sqq;      // grad.q, sum dB.dQ / h^2, sum dQ.dQ / h^2 (S is quadratic in gamma)
  double gamma;
  int32_t accepted, trials, gn_stop, ls_done;
  // PCG (Chronopoulos-Gear recurrences for r^T z and r^T r)
  double alpha, beta, rz, rr, bnorm2, relres;
  int32_t pcg_status, pcg_iters;
  // OT
  double ot_shift;
  int64_t ot_guarded;
  double pad[4];
};

enum PcgStatus : int32_t { kPcgRunning = 0, kPcgFinish = 1, kPcgDone = 2 };

// Stats record written once per Gauss-Newton step.
constexpr int kStatFields = 12;

// ----------------------------------------------------------------------------------------
// Reductions: wavefront shuffles, then LDS across the 4 wavefronts, then per-block partials in
// global memory; the last block to arrive reduces the partials in block order.
// ----------------------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*sh)[kWaves]) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) sh[k][wv] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += sh[k][w];
    v[k] = s;
  }
  __syncthreads();
}

// Writes this block's K partial sums and returns true in the last block to arrive (all threads of
// that block see true).  The last block then calls reduce_partials and must reset the counter.
template <int K>
__device__ bool publish_partials(double (&v)[K], double* partials, unsigned* counter,
                                 unsigned block_id, unsigned nblocks) {
  __shared__ double sh[K > 0 ? K : 1][kWaves];
  __shared__ int is_last;
  block_sum<K>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) partials[(size_t)block_id * K + k] = v[k];
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    is_last = (prev == nblocks - 1u);
  }
  __syncthreads();
  const bool last = is_last != 0;
  if (last) __threadfence();
  return last;
}

// Fixed-order reduction of the partials (called by every thread of the last block).
template <int K>
__device__ void reduce_partials(double (&out)[K], const double* partials, unsigned nblocks) {
  __shared__ double sh[K > 0 ? K : 1][kWaves];
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  for (unsigned b = threadIdx.x; b < nblocks; b += kBlock) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] += partials[(size_t)b * K + k];
  }
  block_sum<K>(out, sh);
}

// Block id remapped so that each XCD (blocks are dealt round-robin to the 8 XCDs) works on a
// contiguous range of tiles, which keeps stencil neighbours in the same L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned bid, unsigned nblocks) {
  constexpr unsigned kXcd = 8;
  const unsigned per = nblocks / kXcd;
  const unsigned full = per * kXcd;
  if (bid >= full) return bid;
  return (bid % kXcd) * per + bid / kXcd;
}

__device__ __forceinline__ double inf_d() { return __longlong_as_double(0x7ff0000000000000LL); }

}  // namespace rgp
