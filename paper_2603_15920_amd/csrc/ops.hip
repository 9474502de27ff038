// Finite-volume operator kernels of libdifvm: permutation, face interpolation, Gauss gradient,
// face-sum divergence, over-relaxed Laplacian, LDU products and assembly.
//
// Cell kernels walk the cell-slot layout: one thread per cell, one slot per non-empty face side of
// that cell (owner side, neighbour side, boundary), so every aggregation of the paper's message
// passing (eq. aggregate) is a gather in a fixed order: no atomics, bitwise deterministic, and
// independent of the launch shape.  Face kernels (one thread per face) write per-face outputs.
#include <cstring>
#include <type_traits>

#include "abi_util.h"
#include "device.h"
#include "ops.h"

namespace difvm {

// ---------------------------------------------------------------------------------------------
// permutation between user and internal order
// ---------------------------------------------------------------------------------------------
// map[i] (new -> old) for each of n destination rows; sign flips where flip[i] (fluxes)
template <class T>
__global__ void k_permute(int n, int ncomp, const int32_t* __restrict__ map, int map_offset, const uint8_t* __restrict__ flip,
                          int to_internal, const T* __restrict__ src, T* __restrict__ dst, int src_off, int dst_off) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int old = map ? map[i] + map_offset : i + map_offset;
  T sg = (flip && flip[i]) ? T(-1) : T(1);
  if (to_internal) {
    for (int c = 0; c < ncomp; ++c) dst[(size_t)(dst_off + i) * ncomp + c] = sg * src[(size_t)old * ncomp + c];
  } else {
    for (int c = 0; c < ncomp; ++c) dst[(size_t)old * ncomp + c] = sg * src[(size_t)(src_off + i) * ncomp + c];
  }
}

template <class T>
void permute_t(const difvm_mesh* m, int ncomp, int kind, int dir, const T* src, T* dst) {
  const DMesh& d = m->d;
  hipStream_t s = stream_of(m);
  int to = dir == DIFVM_TO_INTERNAL;
  if (kind == DIFVM_KIND_CELL) {
    if (d.nc) k_permute<T><<<grid_for(d.nc), BLOCK, 0, s>>>(d.nc, ncomp, d.cell_perm, 0, nullptr, to, src, dst, 0, 0);
  } else if (kind == DIFVM_KIND_BFACE) {
    if (d.nfb) k_permute<T><<<grid_for(d.nfb), BLOCK, 0, s>>>(d.nfb, ncomp, d.bface_perm, 0, nullptr, to, src, dst, 0, 0);
  } else {
    const uint8_t* fl = kind == DIFVM_KIND_FACE_FLUX ? d.face_flip : nullptr;
    if (d.nfi) k_permute<T><<<grid_for(d.nfi), BLOCK, 0, s>>>(d.nfi, ncomp, d.face_perm, 0, fl, to, src, dst, 0, 0);
    // boundary block: internal row nfi+b <- user row nfi + bface_perm[b]
    if (d.nfb) {
      if (to)
        k_permute<T><<<grid_for(d.nfb), BLOCK, 0, s>>>(d.nfb, ncomp, d.bface_perm, d.nfi, nullptr, 1, src, dst, 0, d.nfi);
      else
        k_permute<T><<<grid_for(d.nfb), BLOCK, 0, s>>>(d.nfb, ncomp, d.bface_perm, d.nfi, nullptr, 0, src, dst, d.nfi, 0);
    }
  }
  DIFVM_HIP(hipGetLastError());
}

void permute(const difvm_mesh* m, int dtype, int ncomp, int kind, int dir, const void* src, void* dst) {
  if (dtype == DIFVM_F64) permute_t<double>(m, ncomp, kind, dir, (const double*)src, (double*)dst);
  else permute_t<float>(m, ncomp, kind, dir, (const float*)src, (float*)dst);
}

// largest threads-per-block a tuned operator kernel may be launched with (the knobs of
// difvm_mesh_set_launch); one cell or face per thread, so the outputs do not depend on it
constexpr int OP_MAX_BLOCK = 512;
static int op_block(const difvm_mesh* m, int knob_f64, int dtype_is_f32) { return m->tune[knob_f64 + dtype_is_f32]; }

// ---------------------------------------------------------------------------------------------
// face interpolation (face kernel)
// ---------------------------------------------------------------------------------------------
template <class T, int NC>
__global__ __launch_bounds__(OP_MAX_BLOCK) void k_interp(MeshView<T> m, int table, const T* __restrict__ phi,
                                                  const T* __restrict__ phib, T* __restrict__ out) {
  const int base = xcd_tile(blockIdx.x, gridDim.x) * (int)blockDim.x;
  const int f = base + threadIdx.x;
  T res[NC];
  if (f < m.nfi) {
    T w = m.w[f];
    int O = m.own[f], N = m.nbr[f];
#pragma unroll
    for (int c = 0; c < NC; ++c) res[c] = w * phi[(size_t)O * NC + c] + (T(1) - w) * phi[(size_t)N * NC + c];
  } else if (f < m.nfi + m.nfb) {
    int b = f - m.nfi;
    int8_t code = m.bcode[table * m.nfb + b];
    int O = m.bown[b];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T v = T(0);
      if (code == BC_FIXED) v = phib[(size_t)b * NC + c];
      else if (code == BC_ZEROGRAD) v = phi[(size_t)O * NC + c];
      res[c] = v;
    }
  }
  if constexpr (NC == 1) {
    if (f < m.nfi + m.nfb) out[f] = res[0];
  } else {
    store_rows<NC>(out, base, m.nfi + m.nfb, res, dyn_lds<T>());
  }
}

// ---------------------------------------------------------------------------------------------
// Row walkers.  A cell's own slots are visited in layout order; the first four (two for the vector
// gradient, whose slots carry more values) go in one unrolled chunk with every slot's loads issued
// before any is used (indices clamped so each load is in bounds whatever the slot holds), the rest
// one at a time.  (Two-slot chunks in the Laplacian raise occupancy but were slower: the second
// chunk's loads wait for the first's.)
// ---------------------------------------------------------------------------------------------


// ---------------------------------------------------------------------------------------------
// Gauss gradient (cell kernel): G_i = (1/V_i) sum_slots sigma phi_f S_f
// ---------------------------------------------------------------------------------------------
template <class T, int NC>
__global__ __launch_bounds__(OP_MAX_BLOCK) void k_grad(MeshView<T> m, int table, const T* __restrict__ phi,
                                                const T* __restrict__ phib, T* __restrict__ out) {
  const int base = xcd_tile(blockIdx.x, gridDim.x) * (int)blockDim.x;
  const int i = base + threadIdx.x;
  T res[3 * NC];
  if (i < m.nc) {
    const T vi = m.V[i];  // in flight with the row's loads
    T acc[NC][3];
    gauss_row_sum<T, NC>(m, table, phi, phib, i, acc);
    T rv = T(1) / vi;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int e = 0; e < 3; ++e) res[3 * c + e] = acc[c][e] * rv;
  }
  store_rows<3 * NC>(out, base, m.nc, res, dyn_lds<T>());
}

// ---------------------------------------------------------------------------------------------
// face-sum divergence (cell kernel): D_i = sum_slots sigma F_f psi_f
// ---------------------------------------------------------------------------------------------
template <class T, int NC, int SCHEME>
__global__ __launch_bounds__(OP_MAX_BLOCK) void k_div(MeshView<T> m, int table, const T* __restrict__ flux,
                                               const T* __restrict__ psi, const T* __restrict__ psib, T* __restrict__ out) {
  const int base = xcd_tile(blockIdx.x, gridDim.x) * (int)blockDim.x;
  const int i = base + threadIdx.x;
  T acc[NC];
  if (i < m.nc) {
  SlotRange R = slots_of(m, i);
  T pi[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    pi[c] = SCHEME == DIFVM_SCHEME_ONE ? T(0) : psi[(size_t)i * NC + c];
    acc[c] = T(0);
  }
  const int8_t* code = m.bcode + table * m.nfb;
  walk_row<4>(row_len(m, i, R), [&](auto Wc, int k0) {
    constexpr int N = decltype(Wc)::value;
    {
      int sf[N], j[N];
      T F[N], wf[N], pj[N][NC];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        int at = R.base + (k0 + k) * SLICE;
        sf[k] = m.slot_face[at];
        j[k] = m.slot_col[at];
      }
#pragma unroll
      for (int k = 0; k < N; ++k) {
        // internal face, or the boundary face's own flux entry (pad slots read entry 0)
        int fi = slot_internal(sf[k], m.nfi) ? (sf[k] < 0 ? -sf[k] - 1 : sf[k]) : (sf[k] == SLOT_PAD ? 0 : sf[k]);
        F[k] = flux[fi];
        wf[k] = SCHEME == DIFVM_SCHEME_LINEAR ? m.w[slot_face_index(sf[k], m.nfi)] : T(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) pj[k][c] = SCHEME == DIFVM_SCHEME_ONE ? T(0) : psi[(size_t)j[k] * NC + c];
      }
#pragma unroll
      for (int k = 0; k < N; ++k) {
        if (sf[k] == SLOT_PAD) continue;
        if (sf[k] < m.nfi) {
          bool nb = sf[k] < 0;
          T Fs = nb ? -F[k] : F[k];  // flux out of this cell
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            T pf;
            if (SCHEME == DIFVM_SCHEME_ONE) {
              pf = T(1);
            } else if (SCHEME == DIFVM_SCHEME_UPWIND) {
              bool owner_up = F[k] >= T(0);  // the tie F = 0 belongs to the owner
              bool self_up = nb ? !owner_up : owner_up;
              pf = self_up ? pi[c] : pj[k][c];
            } else {
              T wself = nb ? T(1) - wf[k] : wf[k];
              pf = wself * pi[c] + (T(1) - wself) * pj[k][c];
            }
            acc[c] += Fs * pf;
          }
        } else {
          int b = sf[k] - m.nfi;
          bool fixed = code[b] == BC_FIXED;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            T pf = SCHEME == DIFVM_SCHEME_ONE ? T(1) : (fixed ? psib[(size_t)b * NC + c] : pi[c]);
            acc[c] += F[k] * pf;
          }
        }
      }
    }
  });
  }
  if constexpr (NC == 1) {
    if (i < m.nc) out[i] = acc[0];
  } else {
    store_rows<NC>(out, base, m.nc, acc, dyn_lds<T>());
  }
}

// ---------------------------------------------------------------------------------------------
// Laplacian with over-relaxed correction (cell kernel)
// ---------------------------------------------------------------------------------------------
template <class T, bool GAMMA>
__global__ __launch_bounds__(OP_MAX_BLOCK) void k_laplacian(MeshView<T> m, int table, const T* __restrict__ gamma,
                                                     const T* __restrict__ phi, const T* __restrict__ g,
                                                     const T* __restrict__ phib, T* __restrict__ out) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * (int)blockDim.x + threadIdx.x;
  if (i >= m.nc) return;
  SlotRange R = slots_of(m, i);
  T pi = phi[i];
  T gi0 = g[3 * (size_t)i], gi1 = g[3 * (size_t)i + 1], gi2 = g[3 * (size_t)i + 2];
  T acc = T(0);
  const int8_t* code = m.bcode + table * m.nfb;
  walk_row<4>(row_len(m, i, R), [&](auto Wc, int k0) {
    constexpr int N = decltype(Wc)::value;
    int sf[N], j[N];
    typename Geo<T>::v4 kd[N];
    T wf[N], pj[N], gj[N][3], gm[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      int at = R.base + (k0 + k) * SLICE;
      sf[k] = m.slot_face[at];
      j[k] = m.slot_col[at];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      int f = slot_face_index(sf[k], m.nfi);
      kd[k] = m.geomK[f];
      wf[k] = m.w[f];
      gm[k] = GAMMA ? gamma[f] : T(1);
      pj[k] = phi[j[k]];
#pragma unroll
      for (int e = 0; e < 3; ++e) gj[k][e] = g[3 * (size_t)j[k] + e];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if (sf[k] == SLOT_PAD) continue;
      if (sf[k] < m.nfi) {
        bool nb = sf[k] < 0;
        T wself = nb ? T(1) - wf[k] : wf[k];
        // seen from this cell: delta (phi_other - phi_self) + k_out . gbar, with k_out the
        // correction vector oriented out of this cell; the owner-side form of eq. nonortho_flux,
        // negated for the neighbour side
        T corr = kd[k].x * (wself * gi0 + (T(1) - wself) * gj[k][0]) +
                 kd[k].y * (wself * gi1 + (T(1) - wself) * gj[k][1]) +
                 kd[k].z * (wself * gi2 + (T(1) - wself) * gj[k][2]);
        T t = kd[k].w * (pj[k] - pi) + (nb ? -corr : corr);
        if (GAMMA) t *= gm[k];
        acc += t;
      } else {
        int b = sf[k] - m.nfi;
        if (code[b] == BC_FIXED) {
          T t = m.bgeom[b].w * (phib[b] - pi);
          if (GAMMA) t *= gamma[m.nfi + b];
          acc += t;
        }
      }
    }
  });
  out[i] = acc;
}

// ---------------------------------------------------------------------------------------------
// LDU product through the slots (owner slot: upper, neighbour slot: lower)
// ---------------------------------------------------------------------------------------------
template <class T, int NC>
__global__ __launch_bounds__(OP_MAX_BLOCK) void k_ldu_spmv(MeshView<T> m, const T* __restrict__ diag, const T* __restrict__ up,
                                                    const T* __restrict__ lo, const T* __restrict__ x, T* __restrict__ y) {
  const int base = xcd_tile(blockIdx.x, gridDim.x) * (int)blockDim.x;
  const int i = base + threadIdx.x;
  T acc[NC];
  if (i < m.nc) {
  SlotRange R = slots_of(m, i);
  T di = diag[i];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = di * x[(size_t)i * NC + c];
  walk_row<4>(row_len(m, i, R), [&](auto Wc, int k0) {
    constexpr int N = decltype(Wc)::value;
    {
      int sf[N], j[N];
      T a[N], xj[N][NC];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        int at = R.base + (k0 + k) * SLICE;
        sf[k] = m.slot_face[at];
        j[k] = m.slot_col[at];
      }
#pragma unroll
      for (int k = 0; k < N; ++k) {
        bool in = slot_internal(sf[k], m.nfi);
        int f = in ? (sf[k] < 0 ? -sf[k] - 1 : sf[k]) : 0;
        T v = (in && sf[k] < 0) ? lo[f] : up[f];
        a[k] = in ? v : T(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) xj[k][c] = x[(size_t)j[k] * NC + c];
      }
#pragma unroll
      for (int k = 0; k < N; ++k) {
        if (!slot_internal(sf[k], m.nfi)) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += a[k] * xj[k][c];
      }
    }
  });
  }
  if constexpr (NC == 1) {
    if (i < m.nc) y[i] = acc[0];
  } else {
    store_rows<NC>(y, base, m.nc, acc, dyn_lds<T>());
  }
}

// ---------------------------------------------------------------------------------------------
// Laplace assembly (cell kernel; each face's upper is written by its owner side)
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_assemble_laplace(MeshView<double> m, int table, const double* __restrict__ gamma,
                                                            const double* __restrict__ phib, double* __restrict__ diag,
                                                            double* __restrict__ upper, double* __restrict__ rhs) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= m.nc) return;
  SlotRange R = slots_of(m, i);
  double d = 0.0, r = 0.0;
  const int8_t* code = m.bcode + table * m.nfb;
#pragma unroll 4
  for (int k = 0; k < R.width; ++k) {
    int at = R.base + k * SLICE;
    int sf = m.slot_face[at];
    if (sf == SLOT_PAD) continue;
    if (sf < m.nfi) {
      bool nb = sf < 0;
      int f = nb ? -sf - 1 : sf;
      double a = m.geomK[f].w * (gamma ? gamma[f] : 1.0);
      d += a;
      if (!nb) upper[f] = -a;
    } else {
      int b = sf - m.nfi;
      if (code[b] == BC_FIXED) {
        double a = m.bgeom[b].w * (gamma ? gamma[m.nfi + b] : 1.0);
        d += a;
        if (phib) r += a * phib[b];
      }
    }
  }
  diag[i] = d;
  if (rhs) rhs[i] = r;
}

// ---------------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------------
template <class T>
void interp_t(const difvm_mesh* mm, int ncomp, int table, const T* phi, const T* phib, T* out) {
  const DMesh& d = mm->d;
  int n = d.nfi + d.nfb;
  if (!n) return;
  MeshView<T> v = view<T>(d);
  int nb = op_block(mm, DIFVM_TUNE_INTERP_F64, sizeof(T) == 4);
  if (ncomp == 1) k_interp<T, 1><<<grid_for(n, nb), nb, 0, stream_of(mm)>>>(v, table, phi, phib, out);
  else k_interp<T, 3><<<grid_for(n, nb), nb, 3 * nb * sizeof(T), stream_of(mm)>>>(v, table, phi, phib, out);
  DIFVM_HIP(hipGetLastError());
}

template <class T>
void grad_t(const difvm_mesh* mm, int ncomp, int table, const T* phi, const T* phib, T* out) {
  const DMesh& d = mm->d;
  MeshView<T> v = view<T>(d);
  int nb = op_block(mm, DIFVM_TUNE_GRAD_F64, sizeof(T) == 4);
  if (ncomp == 1) k_grad<T, 1><<<grid_for(d.nc, nb), nb, 3 * nb * sizeof(T), stream_of(mm)>>>(v, table, phi, phib, out);
  else k_grad<T, 3><<<grid_for(d.nc, nb), nb, 9 * nb * sizeof(T), stream_of(mm)>>>(v, table, phi, phib, out);
  DIFVM_HIP(hipGetLastError());
}

template <class T, int NC>
void div_nc(const difvm_mesh* mm, int scheme, int table, const T* flux, const T* psi, const T* psib, T* out) {
  const DMesh& d = mm->d;
  MeshView<T> v = view<T>(d);
  int nb = op_block(mm, DIFVM_TUNE_DIV_F64, sizeof(T) == 4);
  int G = grid_for(d.nc, nb);
  hipStream_t s = stream_of(mm);
  size_t lds = NC > 1 ? NC * nb * sizeof(T) : 0;
  if (scheme == DIFVM_SCHEME_ONE) k_div<T, NC, DIFVM_SCHEME_ONE><<<G, nb, lds, s>>>(v, table, flux, psi, psib, out);
  else if (scheme == DIFVM_SCHEME_UPWIND) k_div<T, NC, DIFVM_SCHEME_UPWIND><<<G, nb, lds, s>>>(v, table, flux, psi, psib, out);
  else k_div<T, NC, DIFVM_SCHEME_LINEAR><<<G, nb, lds, s>>>(v, table, flux, psi, psib, out);
  DIFVM_HIP(hipGetLastError());
}

template <class T>
void laplacian_t(const difvm_mesh* mm, int table, const T* gamma, const T* phi, const T* g, const T* phib, T* out) {
  const DMesh& d = mm->d;
  MeshView<T> v = view<T>(d);
  int nb = op_block(mm, DIFVM_TUNE_LAPLACIAN_F64, sizeof(T) == 4);
  int G = grid_for(d.nc, nb);
  if (gamma) k_laplacian<T, true><<<G, nb, 0, stream_of(mm)>>>(v, table, gamma, phi, g, phib, out);
  else k_laplacian<T, false><<<G, nb, 0, stream_of(mm)>>>(v, table, gamma, phi, g, phib, out);
  DIFVM_HIP(hipGetLastError());
}

template <class T>
void ldu_spmv_t(const difvm_mesh* mm, int ncomp, int transpose, const T* diag, const T* up, const T* lo, const T* x, T* y) {
  const DMesh& d = mm->d;
  MeshView<T> v = view<T>(d);
  if (!lo) lo = up;
  if (transpose) std::swap(up, lo);
  // the kernel reads entry 0 of up / lo on non-internal slots (value unused): with no internal faces
  // the caller may pass NULL, so point both at diag (nc >= 1 entries)
  if (d.nfi == 0) up = lo = diag;
  int nb = op_block(mm, DIFVM_TUNE_LDU_SPMV_F64, sizeof(T) == 4);
  int G = grid_for(d.nc, nb);
  if (ncomp == 1) k_ldu_spmv<T, 1><<<G, nb, 0, stream_of(mm)>>>(v, diag, up, lo, x, y);
  else k_ldu_spmv<T, 3><<<G, nb, 3 * nb * sizeof(T), stream_of(mm)>>>(v, diag, up, lo, x, y);
  DIFVM_HIP(hipGetLastError());
}

void op_interp(const difvm_mesh* m, int dtype, int ncomp, int bc, const void* phi, const void* phib, void* out) {
  if (dtype == DIFVM_F64) interp_t<double>(m, ncomp, bc, (const double*)phi, (const double*)phib, (double*)out);
  else interp_t<float>(m, ncomp, bc, (const float*)phi, (const float*)phib, (float*)out);
}
void op_grad(const difvm_mesh* m, int dtype, int ncomp, int bc, const void* phi, const void* phib, void* out) {
  if (dtype == DIFVM_F64) grad_t<double>(m, ncomp, bc, (const double*)phi, (const double*)phib, (double*)out);
  else grad_t<float>(m, ncomp, bc, (const float*)phi, (const float*)phib, (float*)out);
}
void op_div(const difvm_mesh* m, int dtype, int scheme, int ncomp, int bc, const void* flux, const void* psi,
            const void* psib, void* out) {
  if (dtype == DIFVM_F64) {
    if (ncomp == 1) div_nc<double, 1>(m, scheme, bc, (const double*)flux, (const double*)psi, (const double*)psib, (double*)out);
    else div_nc<double, 3>(m, scheme, bc, (const double*)flux, (const double*)psi, (const double*)psib, (double*)out);
  } else {
    if (ncomp == 1) div_nc<float, 1>(m, scheme, bc, (const float*)flux, (const float*)psi, (const float*)psib, (float*)out);
    else div_nc<float, 3>(m, scheme, bc, (const float*)flux, (const float*)psi, (const float*)psib, (float*)out);
  }
}
void op_laplacian(const difvm_mesh* m, int dtype, int bc, const void* gamma, const void* phi, const void* g,
                  const void* phib, void* out) {
  if (dtype == DIFVM_F64)
    laplacian_t<double>(m, bc, (const double*)gamma, (const double*)phi, (const double*)g, (const double*)phib, (double*)out);
  else
    laplacian_t<float>(m, bc, (const float*)gamma, (const float*)phi, (const float*)g, (const float*)phib, (float*)out);
}
void op_ldu_spmv(const difvm_mesh* m, int dtype, int ncomp, int transpose, const void* diag, const void* up,
                 const void* lo, const void* x, void* y) {
  if (dtype == DIFVM_F64)
    ldu_spmv_t<double>(m, ncomp, transpose, (const double*)diag, (const double*)up, (const double*)lo, (const double*)x, (double*)y);
  else
    ldu_spmv_t<float>(m, ncomp, transpose, (const float*)diag, (const float*)up, (const float*)lo, (const float*)x, (float*)y);
}
void op_assemble_laplace(const difvm_mesh* m, int bc, const double* gamma, const double* phib, double* diag,
                         double* upper, double* rhs) {
  const DMesh& d = m->d;
  k_assemble_laplace<<<grid_for(d.nc), BLOCK, 0, stream_of(m)>>>(view<double>(d), bc, gamma, phib, diag, upper, rhs);
  DIFVM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------------------
// halo exchange of a partition part.  One thread per value (row-major rows of ncomp), so a wave's
// stores to the send buffer and its loads from the receive buffer are contiguous; the pack's loads
// gather owned rows next to the cut, which RCM keeps within a few cache lines of each other.
// ---------------------------------------------------------------------------------------------
template <class T>
__global__ void k_halo_pack(int n_val, int ncomp, const int32_t* __restrict__ send, const T* __restrict__ x,
                            T* __restrict__ buf) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_val) return;
  int k = e / ncomp, c = e - k * ncomp;
  buf[e] = x[(size_t)send[k] * ncomp + c];
}

template <class T>
__global__ void k_halo_unpack(int n_val, const T* __restrict__ buf, T* __restrict__ xg) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n_val) xg[e] = buf[e];
}

void op_halo_pack(const difvm_mesh* m, int dtype, int ncomp, const void* x, void* buf) {
  int n = m->part_n_send * ncomp;
  if (!n) return;
  if (dtype == DIFVM_F64)
    k_halo_pack<double><<<grid_for(n), BLOCK, 0, stream_of(m)>>>(n, ncomp, m->part_send, (const double*)x, (double*)buf);
  else
    k_halo_pack<float><<<grid_for(n), BLOCK, 0, stream_of(m)>>>(n, ncomp, m->part_send, (const float*)x, (float*)buf);
  DIFVM_HIP(hipGetLastError());
}

void op_halo_unpack(const difvm_mesh* m, int dtype, int ncomp, const void* buf, void* x) {
  int n = m->part_n_ghost * ncomp;
  if (!n) return;
  size_t off = (size_t)m->part_n_owned * ncomp;
  if (dtype == DIFVM_F64)
    k_halo_unpack<double><<<grid_for(n), BLOCK, 0, stream_of(m)>>>(n, (const double*)buf, (double*)x + off);
  else
    k_halo_unpack<float><<<grid_for(n), BLOCK, 0, stream_of(m)>>>(n, (const float*)buf, (float*)x + off);
  DIFVM_HIP(hipGetLastError());
}

}  // namespace difvm
