// Device helpers shared by the libdifvm kernels: XCD-aware block mapping, slot decoding, geometry
// record types per precision, deterministic block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace difvm {

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X.  Remapping the block index
// gives each XCD one contiguous run of tiles, so a slice's neighbours (RCM keeps them close in
// index) are gathered through the same L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  int x = b & 7, k = b >> 3, q = G >> 3, r = G & 7;
  return x * q + (x < r ? x : r) + k;
}

template <class T>
struct Geo;
template <>
struct Geo<double> {
  using v4 = double4;
};
template <>
struct Geo<float> {
  using v4 = float4;
};

// read-only view of the device mesh passed by value to kernels
template <class T>
struct MeshView {
  int nc, nfi, nfb;
  const int32_t* __restrict__ own;
  const int32_t* __restrict__ nbr;
  const typename Geo<T>::v4* __restrict__ geomS;  // (S, w)
  const typename Geo<T>::v4* __restrict__ geomK;  // (k, delta)
  const T* __restrict__ w;
  const int32_t* __restrict__ bown;
  const typename Geo<T>::v4* __restrict__ bgeom;  // (S_b, delta_b)
  const int8_t* __restrict__ bcode;               // [N_TABLES][nfb]
  const T* __restrict__ V;
  const int32_t* __restrict__ slice_start;
  const int32_t* __restrict__ slot_face;
  const int32_t* __restrict__ slot_col;
  const uint8_t* __restrict__ nslot;  // slots of each cell (255: use the slice width)
  int uw;                             // > 0: every cell has exactly uw slots (uniform rows)
};

template <class T>
MeshView<T> view(const DMesh& d);
template <>
inline MeshView<double> view<double>(const DMesh& d) {
  return {d.nc, d.nfi, d.nfb, d.own, d.nbr, d.geomS, d.geomK, d.w, d.bown, d.bgeom, d.bcode, d.V,
          d.slice_start, d.slot_face, d.slot_col, d.cell_nslot, d.uw};
}
template <>
inline MeshView<float> view<float>(const DMesh& d) {
  return {d.nc, d.nfi, d.nfb, d.own, d.nbr, d.geomS32, d.geomK32, d.w32, d.bown, d.bgeom32, d.bcode, d.V32,
          d.slice_start, d.slot_face, d.slot_col, d.cell_nslot, d.uw};
}

// slot range of cell i: slots base + k*SLICE for k < width (the slice's width: trailing pads
// possible).  With uniform rows (uw > 0: every cell has exactly uw slots, as in a tet mesh whose
// boundary faces all carry slots) every slice has width uw and the range follows from i alone, so the
// slot loads need not wait for a load of the slice table.
struct SlotRange {
  int base, width;
};
__device__ __forceinline__ SlotRange slots_of(const int32_t* slice_start, int uw, int i) {
  if (uw > 0) return {(i >> 6) * (SLICE * uw) + (i & (SLICE - 1)), uw};
  int s = i >> 6;
  int b = slice_start[s];
  return {b + (i & (SLICE - 1)), (slice_start[s + 1] - b) >> 6};
}
template <class V>
__device__ __forceinline__ SlotRange slots_of(const V& v, int i) {
  return slots_of(v.slice_start, v.uw, i);
}

// number of slots a row walker visits for cell i: the cell's own count, so that a cell's arithmetic
// never depends on the other cells of its slice (cells of one mesh packed beside another compute the
// same bits as alone); 255 marks a count too large for the byte, then the slice width is used
__device__ __forceinline__ int row_len(const uint8_t* __restrict__ nslot, int uw, int i, const SlotRange& R) {
  if (uw > 0) return uw;
  int n = nslot[i];
  return n == 255 ? R.width : n;
}
template <class V>
__device__ __forceinline__ int row_len(const V& v, int i, const SlotRange& R) {
  return row_len(v.nslot, v.uw, i, R);
}

// Walks a row of n slots in order: body(W, k0) handles slots k0 .. k0+W-1 with W a compile-time
// count; the first min(n, CH) slots go in one unrolled chunk (all their loads issued together), the
// rest one at a time.  CH bounds the registers a kernel allocates (its widest chunk sets them).
template <int CH, class F>
__device__ __forceinline__ void walk_row(int n, F&& body) {
  int k0 = 0;
  if (n >= CH) {
    body(std::integral_constant<int, CH>{}, 0);
    k0 = CH;
  } else if constexpr (CH > 3) {
    if (n == 3) {
      body(std::integral_constant<int, 3>{}, 0);
      k0 = 3;
    }
  }
  for (; k0 < n; ++k0) body(std::integral_constant<int, 1>{}, k0);
}

__device__ __forceinline__ bool slot_internal(int sf, int nfi) { return sf != SLOT_PAD && sf < nfi; }
__device__ __forceinline__ int slot_face_index(int sf, int nfi) { return slot_internal(sf, nfi) ? (sf < 0 ? -sf - 1 : sf) : 0; }

// Gauss-gradient face sum of cell i (the Gauss gradient times V_i): acc[c] = sum over the row's slots
// of sigma phi_f S_f, phi_f = w phi_i + (1 - w) phi_j on internal faces (w this cell's weight), the
// boundary table's fixed value or phi_i on boundary faces.  Slots in layout order, the first four
// (two for vectors) with all their loads issued before any is used (walk_row).
template <class T, int NC>
__device__ __forceinline__ void gauss_row_sum(const MeshView<T>& m, int table, const T* __restrict__ phi,
                                              const T* __restrict__ phib, int i, T (&acc)[NC][3]) {
  SlotRange R = slots_of(m, i);
  T pi[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    pi[c] = phi[(size_t)i * NC + c];
    acc[c][0] = acc[c][1] = acc[c][2] = T(0);
  }
  const int8_t* code = m.bcode + table * m.nfb;
  walk_row<(NC == 3 ? 2 : 4)>(row_len(m, i, R), [&](auto Wc, int k0) {
    constexpr int N = decltype(Wc)::value;
    int sf[N], j[N];
    typename Geo<T>::v4 g[N];
    T pj[N][NC];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      int at = R.base + (k0 + k) * SLICE;
      sf[k] = m.slot_face[at];
      j[k] = m.slot_col[at];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      g[k] = m.geomS[slot_face_index(sf[k], m.nfi)];
#pragma unroll
      for (int c = 0; c < NC; ++c) pj[k][c] = phi[(size_t)j[k] * NC + c];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if (sf[k] == SLOT_PAD) continue;
      if (sf[k] < m.nfi) {
        bool nb = sf[k] < 0;
        T wself = nb ? T(1) - g[k].w : g[k].w;  // weight of this cell in phi_f
        T sg = nb ? T(-1) : T(1);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T pf = sg * (wself * pi[c] + (T(1) - wself) * pj[k][c]);
          acc[c][0] += pf * g[k].x;
          acc[c][1] += pf * g[k].y;
          acc[c][2] += pf * g[k].z;
        }
      } else {
        int b = sf[k] - m.nfi;
        auto gb = m.bgeom[b];
        bool fixed = code[b] == BC_FIXED;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T pf = fixed ? phib[(size_t)b * NC + c] : pi[c];
          acc[c][0] += pf * gb.x;
          acc[c][1] += pf * gb.y;
          acc[c][2] += pf * gb.z;
        }
      }
    }
  });
}

// ---------------------------------------------------------------------------------------------
// Stores of cell-major rows ([n][NC]: vectors, gradients).  One thread per row storing its NC values
// writes at a stride of NC values, so each store instruction covers only part of every cache line it
// touches, and such partial-line writes reach HBM amplified (2.7x measured for 3-vectors).  A block
// whose threads own the consecutive rows [base, base + blockDim.x) stages its rows in LDS and writes
// them back as consecutive values: every store instruction covers whole lines.  Every thread of the
// block must call these (they synchronise twice); rows >= n are not written.  lds holds NC values
// per thread of the block.
// ---------------------------------------------------------------------------------------------
extern __shared__ unsigned char difvm_dyn_lds[];  // dynamic LDS of kernels launched with tuned block sizes
template <class T>
__device__ __forceinline__ T* dyn_lds() {
  return reinterpret_cast<T*>(difvm_dyn_lds);
}

template <int NC, class T>
__device__ __forceinline__ void store_rows(T* __restrict__ out, int base, int n, const T (&v)[NC], T* lds) {
  const int nb = blockDim.x;
  if (base + (int)threadIdx.x < n)
#pragma unroll
    for (int c = 0; c < NC; ++c) lds[NC * threadIdx.x + c] = v[c];
  __syncthreads();
  const int cnt = NC * min(nb, n - base);
  T* o = out + (size_t)NC * base;
  for (int q = threadIdx.x; q < cnt; q += nb) o[q] = lds[q];
  __syncthreads();  // the block may stage again
}

// the same, writing only the values of the components c with keep[c] != 0 (the others keep what they
// hold)
template <int NC, class T>
__device__ __forceinline__ void store_rows_if(T* __restrict__ out, int base, int n, const T (&v)[NC],
                                              const bool (&keep)[NC], T* lds) {
  const int nb = blockDim.x;
  if (base + (int)threadIdx.x < n)
#pragma unroll
    for (int c = 0; c < NC; ++c) lds[NC * threadIdx.x + c] = v[c];
  __syncthreads();
  const int cnt = NC * min(nb, n - base);
  T* o = out + (size_t)NC * base;
  for (int q = threadIdx.x; q < cnt; q += nb) {
    int c = q % NC;
    bool k = keep[0];
#pragma unroll
    for (int u = 1; u < NC; ++u) k = c == u ? keep[u] : k;
    if (k) o[q] = lds[q];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// deterministic reductions: wave64 butterfly, then the 4 waves of a 256-thread block in order
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block of NT threads: every thread ends with the block total (fixed summation order)
template <int NV, int NT = BLOCK>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[NT / 64]) {
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k][wid] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) s += lds[k][q];
    v[k] = s;
  }
}

}  // namespace difvm
