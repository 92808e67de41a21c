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

#include "rgp.h"

namespace rgp {

constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kBlock = 256;       // threads per workgroup of the small kernels
constexpr int kReduceBlock = 512;   // threads of the single-block reducing kernels

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

// Division by a loop-invariant divisor d >= 1 with one high multiply, an add and a shift
// (Granlund and Montgomery, "Division by invariant integers using multiplication", 1994):
// for 0 <= n < 2^31, n / d = (umulhi(n, mul) + n) >> shr with shr = ceil(log2 d) and
// mul = floor(2^32 (2^shr - d) / d) + 1.
struct FastDiv {
  uint32_t d, mul, shr;
};
inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
  return FastDiv{d, (uint32_t)m, l};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (__umulhi(n, f.mul) + n) >> f.shr;
}

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
  FastDiv by_ny;    // column -> (x, y) index
  FastDiv by_nct;   // column-kernel tile -> (run along PE, chunk of 64 columns)
};

__host__ __device__ inline int64_t cell_base(const Geom& g, int64_t col) {
  const int64_t ix = col / g.ny, iy = col - (col / g.ny) * g.ny;
  return ix * g.cxs + iy * g.cys;
}
__host__ __device__ inline int64_t node_base(const Geom& g, int64_t col) {
  const int64_t ix = col / g.ny, iy = col - (col / g.ny) * g.ny;
  return ix * g.nxs + iy * g.nys;
}

// Per-pair device scalars of the solver (written by one designated block of a kernel and read by
// later kernels only, so kernel boundaries order every access).
struct State {
  // objective at the current iterate
  double J, D, S, P, gnorm2;
  // line search
  double gq, sbq, sqq;      // grad.q, sum dB.dQ / h^2, sum dQ.dQ / h^2 (S is quadratic in gamma)
  double gamma;
  // status: the first failure of the solve (an rgp_status code, 0 while none): RGP_ENONFINITE
  // (an input image holds a NaN or an infinity; every level then stops before its first step),
  // RGP_EBARRIER (a level started from a field outside the barrier), RGP_ELINESEARCH (no Armijo
  // trial was accepted in some step); the last two stop only the level they happen on
  int32_t accepted, trials, gn_stop, status;
  // PCG summary of the current GN step
  double relres;
  int32_t pcg_iters, pad1;
  // OT
  double ot_shift;
  // ADMM: the current augmentation parameter rho and the factor the last adaptation applies to
  // the scaled multiplier u
  double admm_rho, admm_ufac;
  double pad[2];
};

// PCG recurrence scalars, double-buffered by iteration parity: kernel i reads slot (i-1)&1 and its
// block 0 writes slot i&1.
struct PcgSlot {
  double rz, rr, bnorm2, relres;
  double alpha, beta;   // coefficients the next main kernel applies
  int32_t status, iters;
};

// Running: apply the update and take the next HVP; Finish: apply the last update x += a p only;
// Done: nothing left to do.
enum PcgStatus : int32_t { kPcgRunning = 0, kPcgFinish = 1, kPcgDone = 2 };

// Stats record written once per Gauss-Newton step.
constexpr int kStatFields = 12;

// Partial sums: every reducing kernel writes kPartStride doubles per block (plain stores); a later
// single-block kernel reduces them in block order.  Grids are capped at kMaxGrid blocks.
constexpr int kPartStride = 32;
constexpr int kMaxGrid = 2048;

// Column-run tiling: a tile is 64 consecutive columns x S consecutive PE nodes, owned by one
// wavefront.  Tiles are split into 8 contiguous ranges, one per XCD (blocks are dealt to the XCDs
// round-robin), and the wavefronts of an XCD stride through its range.
struct WaveIter {
  int64_t t, end, stride;
};

// A workgroup's place in the grid of its volume: the hardware block in a plain launch, or its
// place within one volume's share of a batched launch (each share is a whole number of XCD rounds,
// so id % 8 is still the hardware XCD).
struct VBlock {
  unsigned id, n;
};
__device__ __forceinline__ VBlock hw_block() { return VBlock{blockIdx.x, gridDim.x}; }

// Volume of the calling workgroup in a batched launch over n volumes whose shares start at
// starts[0..n] (starts[n] = grid): the largest p with starts[p] <= blockIdx.x.
__device__ __forceinline__ int batch_volume(const uint32_t* __restrict__ starts, int n,
                                            VBlock& vb) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= blockIdx.x)
      lo = mid;
    else
      hi = mid - 1;
  }
  vb.id = blockIdx.x - starts[lo];
  vb.n = starts[lo + 1] - starts[lo];
  return lo;
}

__device__ __forceinline__ WaveIter wave_iter(int64_t ntiles, VBlock vb) {
  const unsigned G = vb.n, wpb = blockDim.x / 64u, w = threadIdx.x / 64u;
  unsigned nxcd = 1, xcd = 0, lb = vb.id, gl = G;
  if (G >= 8u && G % 8u == 0u) {
    nxcd = 8u;
    xcd = vb.id % 8u;
    lb = vb.id / 8u;
    gl = G / 8u;
  }
  WaveIter it;
  const int64_t lo = ntiles * xcd / nxcd, hi = ntiles * (xcd + 1) / nxcd;
  it.t = lo + (int64_t)lb * wpb + w;
  it.end = hi;
  it.stride = (int64_t)gl * wpb;
  return it;
}

// ----------------------------------------------------------------------------------------
// Reductions: DPP moves within a wavefront, then LDS across the wavefronts of the block.  A producer kernel
// stores its block sums with plain stores; a consumer kernel reduces all blocks in block order.
// No atomics and no fences: visibility comes from the kernel boundary, and the fixed order makes
// every result bitwise reproducible.
// ----------------------------------------------------------------------------------------

// Cross-lane moves of a double within the 16-lane rows of a wavefront (DPP, no LDS traffic).
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Row broadcast (DPP, GFX9): every lane of the rows in ROWMASK gets lane 15 of the previous row
// (CTRL 0x142) or lane 31 (CTRL 0x143); the other rows get 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_bcast(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sums over the 64 lanes of a wavefront (all lanes active) of K values at once, each stage applied
// to all K so the K dependency chains interleave: pairs of lanes, then quads (quad permutations),
// halves of a row (lane i with 7 - i) and rows (lane i with 15 - i) by DPP, which leaves every lane
// of a 16-lane row with the row total; then row 1 += row 0 and row 3 += row 2, and rows 2, 3 +=
// rows 0 + 1 (row broadcasts), so lane 63 holds (r3 + r2) + (r1 + r0), read out to all lanes.  The
// order is fixed, so the result is bitwise the same in every wavefront that sums the same values.
template <int K>
__device__ __forceinline__ void wave_sums(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_row<0xB1>(v[k]);   // quad_perm [1,0,3,2]
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_row<0x4E>(v[k]);   // quad_perm [2,3,0,1]
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_row<0x141>(v[k]);  // row_half_mirror
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_row<0x140>(v[k]);  // row_mirror
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_bcast<0x142, 0xA>(v[k]);  // row_bcast:15 -> rows 1, 3
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_bcast<0x143, 0xC>(v[k]);  // row_bcast:31 -> rows 2, 3
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = read_lane(v[k], 63);
}

// Block sums in a fixed order (BLK = blockDim.x, every lane active): each wavefront reduces its
// K values across its lanes (wave_sums), its first lane publishes them in LDS, and every thread
// adds the BLK/64 wavefront totals in wavefront order.
template <int K, int BLK>
__device__ __forceinline__ void block_sum(double (&v)[K]) {
  constexpr int NW = BLK / kWave;
  __shared__ double sh[NW][K > 0 ? K : 1];
  const int w = threadIdx.x / kWave;
  wave_sums<K>(v);
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[w][k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = sh[0][k];
#pragma unroll
    for (int j = 1; j < NW; ++j) s += sh[j][k];
    v[k] = s;
  }
  __syncthreads();  // the buffer may be reused by the next call
}

// Block sums of v stored at part[blk * kPartStride + k] (blk: the block's VBlock id).
template <int K, int BLK>
__device__ __forceinline__ void store_partials(double (&v)[K], double* part, unsigned blk) {
  block_sum<K, BLK>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) part[(size_t)blk * kPartStride + k] = v[k];
  }
}

// This thread's share of the row-major block sums part[b * kPartStride + k] (k < K) of nprod
// producer blocks, loaded in independent batches; block_sum completes the reduction.
template <int K>
__device__ __forceinline__ void load_partials_rm(double (&out)[K], const double* part,
                                                 unsigned nprod) {
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  for (unsigned b0 = 0; b0 < nprod; b0 += 4u * blockDim.x) {
    double v[4][K];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const unsigned b = b0 + j * blockDim.x + threadIdx.x;
#pragma unroll
      for (int k = 0; k < K; ++k) v[j][k] = b < nprod ? part[(size_t)b * kPartStride + k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) out[k] += v[j][k];
  }
}

// This thread's share of the sums over nprod producer blocks (blocks threadIdx.x, + blockDim.x,
// ...).  The loads are issued in batches of 4 (2 for K > 8) blocks per thread, all independent,
// so that one batch costs one memory round trip; the summation order is fixed.
template <int K>
__device__ __forceinline__ void partials_share(double (&out)[K], const double* part,
                                               unsigned nprod) {
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  constexpr int kB = K <= 8 ? 4 : 2;
  for (unsigned b0 = 0; b0 < nprod; b0 += kB * blockDim.x) {
    double v[kB][K];
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const unsigned b = b0 + j * blockDim.x + threadIdx.x;
#pragma unroll
      for (int k = 0; k < K; ++k) v[j][k] = b < nprod ? part[(size_t)b * kPartStride + k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kB; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) out[k] += v[j][k];
  }
}

// Every thread of the calling block obtains the sums over nprod producer blocks.
template <int K, int BLK>
__device__ __forceinline__ void reduce_partials(double (&out)[K], const double* part,
                                                unsigned nprod) {
  partials_share<K>(out, part, nprod);
  block_sum<K, BLK>(out);
}

// ----------------------------------------------------------------------------------------
// Buffer-resource memory access: one 128-bit descriptor per array (in scalar registers) and one
// 32-bit byte offset per lane shared by every array indexed at the same node, which keeps the
// per-lane address state of kernels that stream many arrays small.  Accesses outside the
// descriptor's range read 0 and are dropped on store.
// ----------------------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t BRes;

// A byte offset outside the range of every descriptor made here (they cover at most 2^31 bytes):
// a load there reads 0 and a store there is dropped.  Kernels use it to issue a fixed sequence of
// memory operations and mask the ones a lane or a step does not need, so that the compiler can
// count the operations in flight and wait for exactly the ones an instruction depends on.
constexpr uint32_t kNullOff = 0x80000000u;

__device__ __forceinline__ BRes bres(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bld(BRes r, uint32_t off);
template <>
__device__ __forceinline__ float bld<float>(BRes r, uint32_t off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ double bld<double>(BRes r, uint32_t off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
  return __hiloint2double((int)v[1], (int)v[0]);
}
template <typename T>
__device__ __forceinline__ void bst(BRes r, uint32_t off, T v);
template <>
__device__ __forceinline__ void bst<float>(BRes r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ void bst<double>(BRes r, uint32_t off, double v) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  u32x2 w;
  w[0] = (unsigned)u;
  w[1] = (unsigned)(u >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)off, 0, 0);
}

// ----------------------------------------------------------------------------------------
// Plane march over the node grid.  The field array is viewed as (o, a, b) with b contiguous, the
// (a, b) plane contiguous and o the outermost axis, whichever of x, y and PE they are:
//   PE axis 0: o = PE, a = x, b = y;   PE axis 1: o = x, a = PE, b = y;   PE axis 2: o = x, a = y,
//   b = PE.
// A work unit is a flat run of T consecutive plane positions (so any plane shape tiles without
// waste) times XL consecutive planes; a workgroup marches through its unit plane by plane.
// ----------------------------------------------------------------------------------------
struct MarchGeo {
  int32_t no, na, nb;    // extents of o, a, b
  int32_t role;          // which of o (0), a (1), b (2) is the PE axis
  int64_t P;             // plane size na * nb (also the o stride)
  int32_t T, XL;         // unit: T plane positions x XL planes
  int32_t ntile, noc;    // units per plane, units along o
  int64_t units;
};

__host__ __device__ inline MarchGeo march_geo(const Geom& g, int T, int XL) {
  MarchGeo m{};
  if (g.pe == 0) {
    m.no = g.mp + 1; m.na = g.nx; m.nb = g.ny; m.role = 0;
  } else if (g.pe == 1) {
    m.no = g.nx; m.na = g.mp + 1; m.nb = g.ny; m.role = 1;
  } else {
    m.no = g.nx; m.na = g.ny; m.nb = g.mp + 1; m.role = 2;
  }
  m.P = (int64_t)m.na * m.nb;
  m.T = T;
  m.XL = XL;
  m.ntile = (int32_t)((m.P + T - 1) / T);
  m.noc = (m.no + XL - 1) / XL;
  m.units = (int64_t)m.ntile * m.noc;
  return m;
}

// Column-major variant for consumers that reduce in every block: sum k of block b is stored at
// part[k * kMaxGrid + b], so the consumer's loads of one sum over all blocks are coalesced.
template <int K, int BLK>
__device__ __forceinline__ void store_partials_cm(double (&v)[K], double* part, unsigned blk) {
  block_sum<K, BLK>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) part[(size_t)k * kMaxGrid + blk] = v[k];
  }
}

// Per-thread partial sums of the first `kuse` column-major sums over nprod blocks (loads only,
// in batches of 4 independent loads per sum; block_sum completes the reduction in a fixed order).
template <int K>
__device__ __forceinline__ void load_partials_cm(double (&out)[K], const double* part,
                                                 unsigned nprod, int kuse) {
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = 0.0;
  for (unsigned b0 = 0; b0 < nprod; b0 += 4u * blockDim.x) {
    double v[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const unsigned b = b0 + j * blockDim.x + threadIdx.x;
        v[k][j] = (k < kuse && b < nprod) ? part[(size_t)k * kMaxGrid + b] : 0.0;
      }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) out[k] += v[k][j];
  }
}

// Image sample at a byte offset of an image descriptor (kNullOff or outside the image: 0).
template <typename TI, typename TR>
__device__ __forceinline__ TR bld_img(BRes r, uint32_t off);
template <>
__device__ __forceinline__ float bld_img<float, float>(BRes r, uint32_t off) {
  return bld<float>(r, off);
}
template <>
__device__ __forceinline__ double bld_img<float, double>(BRes r, uint32_t off) {
  return (double)bld<float>(r, off);
}
template <>
__device__ __forceinline__ float bld_img<double, float>(BRes r, uint32_t off) {
  return (float)bld<double>(r, off);
}
template <>
__device__ __forceinline__ double bld_img<double, double>(BRes r, uint32_t off) {
  return bld<double>(r, off);
}
template <>
__device__ __forceinline__ float bld_img<bf16_t, float>(BRes r, uint32_t off) {
  const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
  return __uint_as_float((uint32_t)h << 16);
}
template <>
__device__ __forceinline__ double bld_img<bf16_t, double>(BRes r, uint32_t off) {
  const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
  return (double)__uint_as_float((uint32_t)h << 16);
}

// Value of the next lower (wave_shr) or higher (wave_shl) lane of the wavefront; lane 0
// (respectively 63), which has no such lane, gets `edge` (DPP wavefront shifts).
template <int CTRL>
__device__ __forceinline__ float dpp_wave(float v, float edge) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_wave(double v, double edge) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(edge), __double2loint(v), CTRL, 0xF,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(edge), __double2hiint(v), CTRL, 0xF,
                                             0xF, false);
  return __hiloint2double(hi, lo);
}
template <typename T>
__device__ __forceinline__ T from_lower_lane(T v, T edge) { return dpp_wave<0x138>(v, edge); }
template <typename T>
__device__ __forceinline__ T from_upper_lane(T v, T edge) { return dpp_wave<0x130>(v, edge); }

// One tile of a column kernel: 64 consecutive columns (one per lane) times a run of S nodes
// along PE starting at node k0.  32-bit node and cell offsets (element units) of the lane's
// column and its neighbour flags; lanes past the last column work on the last one (colok false).
struct ColTile {
  uint32_t nb, cb;      // node and cell index of the column's first node / cell
  int k0;
  bool colok, hasxm, hasxp, hasym, hasyp;
};
__device__ __forceinline__ ColTile col_tile(const Geom& g, int64_t tile, int S) {
  ColTile c;
  const uint32_t tt = (uint32_t)tile;
  const uint32_t kc = fdiv(tt, g.by_nct), cc = tt - kc * g.by_nct.d;
  const uint32_t ncol = (uint32_t)g.ncol;
  const uint32_t col = cc * kWave + (threadIdx.x & (kWave - 1));
  c.colok = col < ncol;
  const uint32_t colc = c.colok ? col : ncol - 1;
  const uint32_t ix = fdiv(colc, g.by_ny), iy = colc - ix * (uint32_t)g.ny;
  c.nb = ix * (uint32_t)g.nxs + iy * (uint32_t)g.nys;
  c.cb = ix * (uint32_t)g.cxs + iy * (uint32_t)g.cys;
  c.k0 = (int)kc * S;
  c.hasxm = ix > 0;
  c.hasxp = ix + 1 < (uint32_t)g.nx;
  c.hasym = iy > 0;
  c.hasyp = iy + 1 < (uint32_t)g.ny;
  return c;
}

__device__ __forceinline__ double inf_d() { return __longlong_as_double(0x7ff0000000000000LL); }

}  // namespace rgp
