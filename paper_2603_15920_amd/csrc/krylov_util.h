// Helpers shared by the Krylov solvers and the AMG V-cycle: the cell-slot matrix view, reduction
// tiles with deterministic per-segment sums, and the PCG control state.
#pragma once

#include "device.h"
#include "ops.h"

namespace difvm {

// ---------------------------------------------------------------------------------------------
// matrix helpers
// ---------------------------------------------------------------------------------------------
struct SellView {
  int nc;
  const uint8_t* __restrict__ nslot;
  const int32_t* __restrict__ slice_start;
  const int32_t* __restrict__ col;
  const double* __restrict__ val;
  const double* __restrict__ diag;
  const int16_t* __restrict__ off16;  // col - row in 16 bits (NULL when it does not fit)
  int uw;                             // uniform row width (0: rows of varying width)
};

inline SellView sview(const difvm_mesh* m, SellMatrix A) {
  return {m->d.nc, m->d.cell_nslot, m->d.slice_start, m->d.slot_col, A.val, A.diag, m->d.slot_off16, m->d.uw};
}

// (A x)_i for NC interleaved components; padding and boundary slots carry val = 0, col = i.  The
// row's slots in layout order (the slice's width; padding adds nothing), the first four with every
// load issued before any is used (walk_row).
template <int NC>
__device__ __forceinline__ void sell_row(const SellView& A, int i, const double* __restrict__ x, double (&acc)[NC]) {
  SlotRange R = slots_of(A, i);
  double di = A.diag[i];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = di * x[(size_t)i * NC + c];
  const bool off16 = A.off16 != nullptr;  // the same for every thread: a uniform branch
  walk_row<4>(R.width, [&](auto Wc, int k0) {
    constexpr int N = decltype(Wc)::value;
    double a[N], xj[N][NC];
    int j[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      int at = R.base + (k0 + k) * SLICE;
      a[k] = A.val[at];
      j[k] = off16 ? i + A.off16[at] : A.col[at];
    }
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) xj[k][c] = x[(size_t)j[k] * NC + c];
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += a[k] * xj[k][c];
  });
}

// ---------------------------------------------------------------------------------------------
// Reduction tiles: TILE = 1024 cells per block (4 per thread), listed per segment.  A segment is one
// independent mesh of a block-diagonal batch (a single mesh is one segment); its dot products are
// the fixed-order sums of its own tiles' partials, so a batch member computes exactly what it would
// alone.
// ---------------------------------------------------------------------------------------------
constexpr int CPT = TILE / BLOCK;  // cells per thread

struct Tiles {
  int ntile;
  const int32_t* __restrict__ lo;
  const int32_t* __restrict__ hi;
  const int32_t* __restrict__ seg;
  const int32_t* __restrict__ first;  // per segment
  const int32_t* __restrict__ count;  // per segment
};
inline Tiles tiles_of(const difvm_mesh* m) {
  const DMesh& d = m->d;
  return {d.ntile, d.tile_lo, d.tile_hi, d.tile_seg, d.seg_tile_first, d.seg_tile_n};
}

struct TileIdx {
  int t, s, lo, hi;
};
__device__ __forceinline__ TileIdx tile_idx(const Tiles& T) {
  int t = xcd_tile(blockIdx.x, gridDim.x);
  return {t, T.seg[t], T.lo[t], T.hi[t]};
}

// fixed-order sum of a segment's tile partials (NV arrays, value-major over all tiles, the segment's
// n tiles from tile f) by a block of NT threads; every thread ends with the totals (sum_seg).  Each
// thread adds the partials q = tid, tid + NT, ... in that order (seg_thread_sum); the loads of four
// such steps (all NV arrays) are issued together, past the end at the clamped index n - 1 and not
// added, so the chain is one load latency per 4 NT tiles.  A block reduction then gives the totals.
template <int NV, int NT = BLOCK>
__device__ __forceinline__ void seg_thread_sum(const double* __restrict__ part, int ntile, int f, int n,
                                               double (&out)[NV]) {
  constexpr int UN = 4;
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = 0.0;
  for (int q = threadIdx.x; q < n; q += UN * NT) {
    double v[UN][NV];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      int at = f + min(q + u * NT, n - 1);
#pragma unroll
      for (int k = 0; k < NV; ++k) v[u][k] = part[(size_t)k * ntile + at];
    }
#pragma unroll
    for (int u = 0; u < UN; ++u)
      if (q + u * NT < n)
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] += v[u][k];
  }
}
template <int NV, int NT = BLOCK>
__device__ __forceinline__ void sum_seg(const double* __restrict__ part, const Tiles& T, int s, double (&out)[NV]) {
  __shared__ double lds[NV][NT / 64];
  seg_thread_sum<NV, NT>(part, T.ntile, T.first[s], T.count[s], out);
  block_sum<NV, NT>(out, lds);
}

template <int NV, int NT = BLOCK>
__device__ __forceinline__ void put_partial(double (&v)[NV], double* __restrict__ part, int ntile, int t) {
  __shared__ double lds[NV][NT / 64];
  block_sum<NV, NT>(v, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) part[(size_t)k * ntile + t] = v[k];
}

// one read of a flag per block, shared through LDS, so every wave of the block takes the same branch
// even while the segment's first tile of the same launch may be writing it
__device__ __forceinline__ bool block_flag(const int* flag) {
  __shared__ int f;
  __syncthreads();  // a previous call's readers are done with f
  if (threadIdx.x == 0) f = *flag;
  __syncthreads();
  return f != 0;
}

// thread 0's copy of a flag the block has already loaded, shared through LDS (as block_flag), so
// that the flag's load can be in flight together with others
__device__ __forceinline__ bool block_share(int v) {
  __shared__ int f;
  __syncthreads();  // a previous call's readers are done with f
  if (threadIdx.x == 0) f = v;
  __syncthreads();
  return f != 0;
}

#define FOR_TILE_CELLS(I) \
  _Pragma("unroll") for (int c_ = 0; c_ < CPT; ++c_) if (int I = ti.lo + c_ * BLOCK + threadIdx.x; I < ti.hi)

// The same cells in rounds of BLOCK consecutive cells [BASE, BASE + BLOCK), every thread of the block
// in every round whether or not its cell I < ti.hi exists: for kernels that stage their stores
// through LDS (store_rows synchronises the block).  Each thread still visits its cells in the same
// order as FOR_TILE_CELLS.
#define FOR_TILE_ROUNDS(BASE, I) \
  _Pragma("unroll") for (int c_ = 0; c_ < CPT; ++c_) \
    if (const int BASE = ti.lo + c_ * BLOCK, I = BASE + (int)threadIdx.x; BASE < ti.hi)

// per-segment PCG state (device)
struct PcgCtl {
  double tol, bn, res;
  double rho[2];  // rho_k at index k & 1
  int maxit, done, iters, status;
};

}  // namespace difvm
