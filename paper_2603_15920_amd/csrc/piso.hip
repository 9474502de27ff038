// PISO time step of libdifvm (paper Sec. "PISO as divergence-free constrained message passing",
// eqs. momentum_predictor, Ap_H, pressure_poisson, velocity_correction; Windkessel outlets eqs.
// windkessel_Q, windkessel_ode, windkessel_discrete).
//
// One step, all on the device:
//   S0  Windkessel: Q_j = sum of outlet fluxes (start of step), exact exponential update of p_c,
//       p_o = p_c + Rp Q imposed on the outlet faces
//   S1  grad U^n; momentum matrix (implicit Euler, implicit upwind of the lagged flux, implicit
//       orthogonal diffusion, explicit non-orthogonal correction, explicit deferred correction of a
//       higher-order convection scheme) written straight into cell-slot form
//   S2  predictor M U* = b - V grad p^n by BiCGStab (three components, one matrix)
//   S3  n_corr times: H = b - offdiag(U), HbyA = H / a_P, rAU = V / a_P; face flux of HbyA and the
//       pressure matrix (negated to SPD form) with its explicit non-orthogonal source; PCG; flux
//       and velocity correction.
// Readings where the paper is open: implicit predictor; H of the latest velocity in every corrector;
// Windkessel flow lagged to the start of the step; pressure reference by diagonal doubling when no
// pressure value is fixed; no transient term in the face-flux interpolation.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "abi_util.h"
#include "dc.h"
#include "device.h"
#include "ops.h"

namespace difvm {

// ---------------------------------------------------------------------------------------------
// momentum matrix (cell kernel): diag, per-slot coefficients (owner slot: upper, neighbour slot:
// lower), optional face LDU copies, and the right-hand side b (without the pressure gradient),
// including the deferred correction of convection scheme CONV (rO/rN: x_f - x_O, x_f - x_N)
// ---------------------------------------------------------------------------------------------
// theta: time scheme weight of the matrix part (1 backward Euler, 1/2 Crank-Nicolson, 0 forward
// Euler); the remaining 1 - theta of it is applied to U^n on the right-hand side
template <int NC, int CONV>
__global__ __launch_bounds__(BLOCK) void k_momentum(MeshView<double> m, int table, double nu_all,
                                                    const double* __restrict__ nu_cell, double dt, double theta,
                                                    const double* __restrict__ flux, const double* __restrict__ U,
                                                    const double* __restrict__ gU, const double* __restrict__ Ub,
                                                    const double4* __restrict__ rO, const double4* __restrict__ rN,
                                                    double* __restrict__ diag, double* __restrict__ upper,
                                                    double* __restrict__ lower, double* __restrict__ slot_val,
                                                    double* __restrict__ b) {
  const int base = xcd_tile(blockIdx.x, gridDim.x) * BLOCK;
  const int i = base + threadIdx.x;
  __shared__ double lds[NC * BLOCK];
  double bi[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) bi[c] = 0.0;
  if (i < m.nc) {
    SlotRange R = slots_of(m, i);
    double nu = nu_cell ? nu_cell[i] : nu_all;  // faces never join cells of different viscosity
    double Vdt = m.V[i] / dt;
    double d = Vdt;
    double ui[NC], gi[3 * NC];  // own values and gradient, kept in registers
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      ui[c] = U[NC * (size_t)i + c];
      bi[c] = Vdt * ui[c];
    }
#pragma unroll
    for (int e = 0; e < 3 * NC; ++e) gi[e] = gU[3 * NC * (size_t)i + e];
    const int8_t* codeU = m.bcode + table * m.nfb;
    // slots in layout order; the first two (four for scalars) with all their loads issued before any
    // is used (walk_row; every index in range whatever the slot holds)
    walk_row<(NC == 3 ? 2 : 4)>(row_len(m, i, R), [&](auto Wc, int k0) {
      constexpr int N = decltype(Wc)::value;
      int sf[N], j[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        int at = R.base + (k0 + k) * SLICE;
        sf[k] = m.slot_face[at];
        j[k] = m.slot_col[at];
      }
      double F[N], wf[N], uj[N][NC], gj[N][3 * NC];
      double4 kd[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        int f = slot_face_index(sf[k], m.nfi);                            // 0 for boundary and padding
        int fl = sf[k] == SLOT_PAD ? 0 : (sf[k] < m.nfi ? f : sf[k]);    // flux index (boundary: nfi + b)
        F[k] = flux[fl];
        kd[k] = m.geomK[f];
        wf[k] = m.w[f];
#pragma unroll
        for (int c = 0; c < NC; ++c) uj[k][c] = U[NC * (size_t)j[k] + c];
#pragma unroll
        for (int e = 0; e < 3 * NC; ++e) gj[k][e] = gU[3 * NC * (size_t)j[k] + e];
      }
#pragma unroll
      for (int k = 0; k < N; ++k) {
        int at = R.base + (k0 + k) * SLICE;
        if (sf[k] == SLOT_PAD) continue;
        double a = 0.0;
        if (sf[k] < m.nfi) {
          bool nb = sf[k] < 0;
          int f = nb ? -sf[k] - 1 : sf[k];
          double nd = nu * kd[k].w;
          double Fp = F[k] >= 0.0 ? F[k] : 0.0;  // max(F,0): the tie F = 0 belongs to the owner
          double Fm = F[k] < 0.0 ? F[k] : 0.0;   // min(F,0)
          double ad = nb ? -Fm + nd : Fp + nd;    // this face's part of the diagonal
          double ao = nb ? -Fp - nd : Fm - nd;    // coefficient of the other cell (lower / upper)
          d += theta * ad;
          a = theta * ao;
          if (!nb) {
            if (upper) upper[f] = a;
          } else {
            if (lower) lower[f] = a;
          }
          if (theta != 1.0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) bi[c] -= (1.0 - theta) * (ad * ui[c] + ao * uj[k][c]);
          }
          double wself = nb ? 1.0 - wf[k] : wf[k];
          double sg = nb ? -nu : nu;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            double corr = kd[k].x * (wself * gi[3 * c] + (1.0 - wself) * gj[k][3 * c]) +
                          kd[k].y * (wself * gi[3 * c + 1] + (1.0 - wself) * gj[k][3 * c + 1]) +
                          kd[k].z * (wself * gi[3 * c + 2] + (1.0 - wself) * gj[k][3 * c + 2]);
            bi[c] += sg * corr;
          }
          if constexpr (CONV != DIFVM_CONV_UPWIND) {
            double4 rs = nb ? rN[f] : rO[f], ro = nb ? rO[f] : rN[f];
            bool up = dc_self_up(F[k], nb);
            double sF = nb ? F[k] : -F[k];  // owner side: b -= F delta; neighbour side: b += F delta
#pragma unroll
            for (int c = 0; c < NC; ++c)
              bi[c] += sF * dc_delta<CONV>(up, wself, ui[c], uj[k][c], gi + 3 * c, gj[k] + 3 * c, rs, ro);
          }
        } else {
          int bf = sf[k] - m.nfi;
          int8_t code = codeU[bf];
          if (code == BC_FIXED) {
            double nd = nu * m.bgeom[bf].w;
            d += theta * nd;
#pragma unroll
            for (int c = 0; c < NC; ++c) bi[c] += (nd - F[k]) * Ub[NC * (size_t)bf + c];
            if (theta != 1.0) {
#pragma unroll
              for (int c = 0; c < NC; ++c) bi[c] -= (1.0 - theta) * nd * ui[c];
            }
          } else if (code == BC_ZEROGRAD) {
            d += theta * F[k];
            if (theta != 1.0) {
#pragma unroll
              for (int c = 0; c < NC; ++c) bi[c] -= (1.0 - theta) * F[k] * ui[c];
            }
          }
        }
        if (slot_val) slot_val[at] = a;
      }
    });
    diag[i] = d;
  }
  if constexpr (NC == 1) {
    if (i < m.nc) b[i] = bi[0];
  } else {
    store_rows<NC>(b, base, m.nc, bi, lds);
  }
}

// deferred-correction source alone: out_i = - sum_f sigma F_f (phi^HO - phi^U), internal faces
template <int NC, int CONV>
__global__ __launch_bounds__(BLOCK) void k_dc(MeshView<double> m, const double* __restrict__ flux,
                                              const double* __restrict__ phi, const double* __restrict__ g,
                                              const double4* __restrict__ rO, const double4* __restrict__ rN,
                                              double* __restrict__ out) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= m.nc) return;
  SlotRange R = slots_of(m, i);
  double pi_[NC], acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    pi_[c] = phi[NC * (size_t)i + c];
    acc[c] = 0.0;
  }
  const double* gi = g + 3 * NC * (size_t)i;
  int n = row_len(m, i, R);
  for (int k = 0; k < n; ++k) {
    int at = R.base + k * SLICE;
    int sf = m.slot_face[at];
    if (sf == SLOT_PAD || sf >= m.nfi) continue;
    bool nb = sf < 0;
    int f = nb ? -sf - 1 : sf;
    int j = m.slot_col[at];
    double F = flux[f];
    double w = m.w[f];
    double wself = nb ? 1.0 - w : w;
    double4 rs = nb ? rN[f] : rO[f], ro = nb ? rO[f] : rN[f];
    bool up = dc_self_up(F, nb);
    double sF = nb ? F : -F;
    const double* pj = phi + NC * (size_t)j;
    const double* gj = g + 3 * NC * (size_t)j;
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += sF * dc_delta<CONV>(up, wself, pi_[c], pj[c], gi + 3 * c, gj + 3 * c, rs, ro);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) out[NC * (size_t)i + c] = acc[c];
}

template <int NC>
static void launch_dc(const difvm_mesh* m, int conv, const double* flux, const double* phi, const double* g,
                      double* out) {
  const DMesh& d = m->d;
  MeshView<double> v = view<double>(d);
  dim3 G(grid_for(d.nc)), B(BLOCK);
  hipStream_t s = stream_of(m);
  if (conv == DIFVM_CONV_LINEAR)
    k_dc<NC, DIFVM_CONV_LINEAR><<<G, B, 0, s>>>(v, flux, phi, g, d.face_rO, d.face_rN, out);
  else if (conv == DIFVM_CONV_SOU)
    k_dc<NC, DIFVM_CONV_SOU><<<G, B, 0, s>>>(v, flux, phi, g, d.face_rO, d.face_rN, out);
  else
    k_dc<NC, DIFVM_CONV_QUICK><<<G, B, 0, s>>>(v, flux, phi, g, d.face_rO, d.face_rN, out);
  DIFVM_HIP(hipGetLastError());
}

void op_deferred_correction(const difvm_mesh* m, int conv, int ncomp, const double* flux, const double* phi,
                            const double* grad, double* out) {
  DIFVM_CHECK(conv >= DIFVM_CONV_UPWIND && conv <= DIFVM_CONV_QUICK, DIFVM_ERR_INVALID_ARG, "unknown convection scheme");
  if (conv == DIFVM_CONV_UPWIND) {
    DIFVM_HIP(hipMemsetAsync(out, 0, sizeof(double) * ncomp * (size_t)m->d.nc, stream_of(m)));
    return;
  }
  if (ncomp == 1) launch_dc<1>(m, conv, flux, phi, grad, out);
  else launch_dc<3>(m, conv, flux, phi, grad, out);
}

double time_theta(int scheme) {
  if (scheme == DIFVM_TIME_FORWARD_EULER) return 0.0;
  if (scheme == DIFVM_TIME_CRANK_NICOLSON) return 0.5;
  return 1.0;
}

template <int NC>
static void launch_momentum(const difvm_mesh* m, int conv, double theta, int table, double nu, const double* nu_cell,
                            double dt, const double* flux, const double* U, const double* gradU, const double* Ub,
                            double* diag, double* upper, double* lower, double* slot_val, double* b) {
  const DMesh& d = m->d;
  MeshView<double> v = view<double>(d);
  dim3 G(grid_for(d.nc)), B(BLOCK);
  hipStream_t s = stream_of(m);
  switch (conv) {
    case DIFVM_CONV_UPWIND:
      k_momentum<NC, DIFVM_CONV_UPWIND><<<G, B, 0, s>>>(v, table, nu, nu_cell, dt, theta, flux, U, gradU, Ub, d.face_rO,
                                                        d.face_rN, diag, upper, lower, slot_val, b);
      break;
    case DIFVM_CONV_LINEAR:
      k_momentum<NC, DIFVM_CONV_LINEAR><<<G, B, 0, s>>>(v, table, nu, nu_cell, dt, theta, flux, U, gradU, Ub, d.face_rO,
                                                        d.face_rN, diag, upper, lower, slot_val, b);
      break;
    case DIFVM_CONV_SOU:
      k_momentum<NC, DIFVM_CONV_SOU><<<G, B, 0, s>>>(v, table, nu, nu_cell, dt, theta, flux, U, gradU, Ub, d.face_rO,
                                                     d.face_rN, diag, upper, lower, slot_val, b);
      break;
    case DIFVM_CONV_QUICK:
      k_momentum<NC, DIFVM_CONV_QUICK><<<G, B, 0, s>>>(v, table, nu, nu_cell, dt, theta, flux, U, gradU, Ub, d.face_rO,
                                                       d.face_rN, diag, upper, lower, slot_val, b);
      break;
    default:
      throw Error{DIFVM_ERR_INVALID_ARG, "unknown convection scheme"};
  }
  DIFVM_HIP(hipGetLastError());
}

void op_assemble_momentum(const difvm_mesh* m, int conv, int time, double nu, const double* nu_cell, double dt,
                          const double* flux, const double* U, const double* gradU, const double* Ub, double* diag,
                          double* upper, double* lower, double* slot_val, double* b) {
  launch_momentum<3>(m, conv, time_theta(time), DIFVM_BC_U, nu, nu_cell, dt, flux, U, gradU, Ub, diag, upper, lower,
                     slot_val, b);
}

// ---------------------------------------------------------------------------------------------
// step kernels
// ---------------------------------------------------------------------------------------------
// S0: one block per Windkessel; outlet flow summed over its faces in face order
__global__ __launch_bounds__(BLOCK) void k_windkessel(int nfi, double dt, const int32_t* __restrict__ wk_start,
                                                      const int32_t* __restrict__ wk_faces, const double* __restrict__ phi,
                                                      const double* __restrict__ wk, double* __restrict__ pc,
                                                      double* __restrict__ pbv, double* __restrict__ wk_out) {
  int j = blockIdx.x;
  int s0 = wk_start[j], s1 = wk_start[j + 1];
  double v[1] = {0.0};
  // each thread adds the fluxes of faces q = s0 + tid, s0 + tid + BLOCK, ... in that order, the loads
  // of UN such faces issued together (an outlet has thousands of faces: one dependent index-then-flux
  // load pair per face would make the sum a long latency chain)
  constexpr int UN = 8;
  for (int q = s0 + threadIdx.x; q < s1; q += UN * BLOCK) {
    int f[UN];
    double fl[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) f[u] = wk_faces[min(q + u * BLOCK, s1 - 1)];
#pragma unroll
    for (int u = 0; u < UN; ++u) fl[u] = phi[nfi + f[u]];
#pragma unroll
    for (int u = 0; u < UN; ++u)
      if (q + u * BLOCK < s1) v[0] += fl[u];
  }
  __shared__ double lds[1][BLOCK / 64];
  block_sum<1>(v, lds);
  double Q = v[0];
  double Rp = wk[3 * j], C = wk[3 * j + 1], Rd = wk[3 * j + 2];
  double E = exp(-dt / (Rd * C));
  double pcn = pc[j] * E + Rd * Q * (1.0 - E);
  double po = pcn + Rp * Q;
  __syncthreads();
  if (threadIdx.x == 0) {
    pc[j] = pcn;
    wk_out[2 * j] = Q;
    wk_out[2 * j + 1] = po;
  }
  for (int q = s0 + threadIdx.x; q < s1; q += BLOCK) pbv[wk_faces[q]] = po;
}

// rhs = b - V grad p
// (one thread per value, so consecutive lanes read and write consecutive doubles)
__global__ __launch_bounds__(BLOCK) void k_pred_rhs(int nc, const double* __restrict__ V, const double* __restrict__ b,
                                                    const double* __restrict__ gp, double* __restrict__ rhs) {
  size_t e = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= 3 * (size_t)nc) return;
  rhs[e] = b[e] - V[e / 3] * gp[e];
}

// H = b - sum_slots a U_j; HbyA = H / d; rAU = V / d
__global__ __launch_bounds__(BLOCK) void k_hbya(int nc, const int32_t* __restrict__ slice_start, int uw,
                                                const int32_t* __restrict__ col, const double* __restrict__ val,
                                                const double* __restrict__ diag, const double* __restrict__ V,
                                                const double* __restrict__ b, const double* __restrict__ U,
                                                double* __restrict__ HbyA, double* __restrict__ rAU) {
  const int base = xcd_tile(blockIdx.x, gridDim.x) * BLOCK;
  const int i = base + threadIdx.x;
  __shared__ double lds[3 * BLOCK];
  double hd[3] = {0.0, 0.0, 0.0};
  if (i < nc) {
  SlotRange R = slots_of(slice_start, uw, i);
  double h[3] = {b[3 * (size_t)i], b[3 * (size_t)i + 1], b[3 * (size_t)i + 2]};
  const double d = diag[i], vi = V[i];  // in flight with the row's loads
  // slots in layout order, the first four with every load issued before any is used
  walk_row<4>(R.width, [&](auto Wc, int k0) {
    constexpr int N = decltype(Wc)::value;
    double a[N], uj[N][3];
    int j[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      int at = R.base + (k0 + k) * SLICE;
      a[k] = val[at];
      j[k] = col[at];
    }
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) uj[k][c] = U[3 * (size_t)j[k] + c];
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) h[c] -= a[k] * uj[k][c];
  });
#pragma unroll
  for (int c = 0; c < 3; ++c) hd[c] = h[c] / d;
  rAU[i] = vi / d;
  }
  store_rows<3>(HbyA, base, nc, hd, lds);
}

// pressure face quantities: phiH (face flux of HbyA), aF = rAU_f delta_f (fixed-p boundaries only on
// the boundary), ncorr = rAU_f k_f . grad(p_old)_f
__global__ __launch_bounds__(BLOCK) void k_pface(MeshView<double> m, const double* __restrict__ HbyA,
                                                 const double* __restrict__ rAU, const double* __restrict__ gp,
                                                 const double* __restrict__ Ub, double* __restrict__ phiH,
                                                 double* __restrict__ aF, double* __restrict__ ncorr) {
  int f = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (f < m.nfi) {
    int O = m.own[f], N = m.nbr[f];
    auto g = m.geomS[f];
    auto kd = m.geomK[f];
    double w = g.w, wn = 1.0 - w;
    const double* hO = HbyA + 3 * (size_t)O;
    const double* hN = HbyA + 3 * (size_t)N;
    phiH[f] = (w * hO[0] + wn * hN[0]) * g.x + (w * hO[1] + wn * hN[1]) * g.y + (w * hO[2] + wn * hN[2]) * g.z;
    double rf = w * rAU[O] + wn * rAU[N];
    aF[f] = rf * kd.w;
    const double* gO = gp + 3 * (size_t)O;
    const double* gN = gp + 3 * (size_t)N;
    double kg = kd.x * (w * gO[0] + wn * gN[0]) + kd.y * (w * gO[1] + wn * gN[1]) + kd.z * (w * gO[2] + wn * gN[2]);
    ncorr[f] = rf * kg;
  } else if (f < m.nfi + m.nfb) {
    int b = f - m.nfi;
    int O = m.bown[b];
    auto g = m.bgeom[b];
    int8_t cu = m.bcode[DIFVM_BC_U * m.nfb + b];
    int8_t cp = m.bcode[DIFVM_BC_P * m.nfb + b];
    double ph = 0.0;
    if (cu == BC_FIXED) ph = Ub[3 * (size_t)b] * g.x + Ub[3 * (size_t)b + 1] * g.y + Ub[3 * (size_t)b + 2] * g.z;
    else if (cu == BC_ZEROGRAD)
      ph = HbyA[3 * (size_t)O] * g.x + HbyA[3 * (size_t)O + 1] * g.y + HbyA[3 * (size_t)O + 2] * g.z;
    phiH[f] = ph;
    aF[f] = cp == BC_FIXED ? rAU[O] * g.w : 0.0;
  }
}

// pressure matrix (SPD form) and right-hand side (cell kernel)
__global__ __launch_bounds__(BLOCK) void k_passemble(MeshView<double> m, const double* __restrict__ phiH,
                                                     const double* __restrict__ aF, const double* __restrict__ ncorr,
                                                     const double* __restrict__ pbv, const int8_t* __restrict__ is_ref,
                                                     double pref, double* __restrict__ diag, double* __restrict__ val,
                                                     double* __restrict__ rhs) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= m.nc) return;
  SlotRange R = slots_of(m, i);
  const int8_t ref = is_ref[i];
  double d = 0.0, r = 0.0;
  const int8_t* codeP = m.bcode + DIFVM_BC_P * m.nfb;
  // slots in layout order, the first four with all their loads issued before any is used
  walk_row<4>(R.width, [&](auto Wc, int k0) {
    constexpr int N = decltype(Wc)::value;
    int sf[N];
#pragma unroll
    for (int k = 0; k < N; ++k) sf[k] = m.slot_face[R.base + (k0 + k) * SLICE];
    double af[N], ph[N], nc[N], pb[N];
    int8_t cp[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      // internal face f, or the boundary face's entries at nfi + b; padding reads entry 0
      const bool in = slot_internal(sf[k], m.nfi), bnd = sf[k] != SLOT_PAD && sf[k] >= m.nfi;
      const int fe = in ? (sf[k] < 0 ? -sf[k] - 1 : sf[k]) : (bnd ? sf[k] : 0);
      af[k] = aF[fe];
      ph[k] = phiH[fe];
      nc[k] = in ? ncorr[fe] : 0.0;
      cp[k] = bnd ? codeP[sf[k] - m.nfi] : int8_t(0);
      pb[k] = bnd ? pbv[sf[k] - m.nfi] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if (sf[k] == SLOT_PAD) continue;
      double a = 0.0;
      if (sf[k] < m.nfi) {
        bool nb = sf[k] < 0;
        d += af[k];
        a = -af[k];
        double t = -ph[k] + nc[k];
        r += nb ? -t : t;
      } else {
        r -= ph[k];
        if (cp[k] == BC_FIXED) {
          d += af[k];
          r += af[k] * pb[k];
        }
      }
      val[R.base + (k0 + k) * SLICE] = a;
    }
  });
  if (ref) {
    r += d * pref;
    d = d + d;
  }
  diag[i] = d;
  rhs[i] = r;
}

// flux correction with the same explicit correction as the right-hand side
__global__ __launch_bounds__(BLOCK) void k_flux(MeshView<double> m, const double* __restrict__ phiH,
                                                const double* __restrict__ aF, const double* __restrict__ ncorr,
                                                const double* __restrict__ p, const double* __restrict__ pbv,
                                                double* __restrict__ phi) {
  int f = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (f < m.nfi) {
    phi[f] = phiH[f] - (aF[f] * (p[m.nbr[f]] - p[m.own[f]]) + ncorr[f]);
  } else if (f < m.nfi + m.nfb) {
    int b = f - m.nfi;
    int8_t cp = m.bcode[DIFVM_BC_P * m.nfb + b];
    double v = 0.0;
    if (cp == BC_FIXED) v = phiH[f] - aF[f] * (pbv[b] - p[m.bown[b]]);
    else if (cp == BC_ZEROGRAD) v = phiH[f];
    phi[f] = v;
  }
}

// velocity correction U = HbyA - rAU grad p (Gauss gradient of the new pressure, fused)
__global__ __launch_bounds__(BLOCK) void k_ucorr(MeshView<double> m, const double* __restrict__ p,
                                                 const double* __restrict__ pbv, const double* __restrict__ HbyA,
                                                 const double* __restrict__ rAU, double* __restrict__ U) {
  const int base = xcd_tile(blockIdx.x, gridDim.x) * BLOCK;
  const int i = base + threadIdx.x;
  __shared__ double lds[3 * BLOCK];
  double un[3] = {0.0, 0.0, 0.0};
  if (i < m.nc) {
    // own values first, in flight with the row's loads
    const double ra = rAU[i], vi = m.V[i];
    double hi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) hi[c] = HbyA[3 * (size_t)i + c];
    double acc[1][3];
    gauss_row_sum<double, 1>(m, DIFVM_BC_P, p, pbv, i, acc);
    double s = ra / vi;
#pragma unroll
    for (int c = 0; c < 3; ++c) un[c] = hi[c] - s * acc[0][c];
  }
  store_rows<3>(U, base, m.nc, un, lds);
}

// phi = interp(U).S with boundary values from the velocity table
__global__ __launch_bounds__(BLOCK) void k_initial_flux(MeshView<double> m, const double* __restrict__ U,
                                                        const double* __restrict__ Ub, double* __restrict__ phi) {
  int f = blockIdx.x * BLOCK + threadIdx.x;
  if (f < m.nfi) {
    auto g = m.geomS[f];
    const double* uo = U + 3 * (size_t)m.own[f];
    const double* un = U + 3 * (size_t)m.nbr[f];
    double w = g.w, wn = 1.0 - w;
    phi[f] = (w * uo[0] + wn * un[0]) * g.x + (w * uo[1] + wn * un[1]) * g.y + (w * uo[2] + wn * un[2]) * g.z;
  } else if (f < m.nfi + m.nfb) {
    int b = f - m.nfi;
    auto g = m.bgeom[b];
    int8_t cu = m.bcode[DIFVM_BC_U * m.nfb + b];
    const double* u = cu == BC_FIXED ? Ub + 3 * (size_t)b : U + 3 * (size_t)m.bown[b];
    phi[f] = cu == BC_EMPTY ? 0.0 : u[0] * g.x + u[1] * g.y + u[2] * g.z;
  }
}

}  // namespace difvm

#include "piso_internal.h"

namespace difvm {

static double* piso_alloc(difvm_piso* P, size_t n) {
  double* a = dalloc<double>(ctx_of(P->mesh), n);
  P->allocs.push_back(a);
  DIFVM_HIP(hipMemsetAsync(a, 0, sizeof(double) * (n ? n : 1), stream_of(P->mesh)));
  return a;
}

void piso_create(difvm_mesh* m, const difvm_piso_params* prm, difvm_piso** out) {
  DIFVM_CHECK(prm && prm->struct_size == sizeof(difvm_piso_params), DIFVM_ERR_INVALID_ARG, "difvm_piso_params mismatch");
  DIFVM_CHECK(prm->n_corr >= 1 && prm->n_corr <= 8, DIFVM_ERR_INVALID_ARG, "n_corr must be in 1..8");
  DIFVM_CHECK(prm->conv >= DIFVM_CONV_UPWIND && prm->conv <= DIFVM_CONV_QUICK, DIFVM_ERR_INVALID_ARG,
              "unknown convection scheme");
  DIFVM_CHECK(prm->time >= DIFVM_TIME_BACKWARD_EULER && prm->time <= DIFVM_TIME_CRANK_NICOLSON, DIFVM_ERR_INVALID_ARG,
              "unknown time scheme");
  DIFVM_CHECK(prm->precond == DIFVM_PRECOND_JACOBI || prm->precond == DIFVM_PRECOND_AMG, DIFVM_ERR_INVALID_ARG,
              "unknown pressure preconditioner");
  DIFVM_CHECK(prm->dt > 0 && prm->nu >= 0, DIFVM_ERR_INVALID_ARG, "dt must be > 0 and nu >= 0");
  const DMesh& d = m->d;
  const HostLayout& L = m->host;
  int min_seg = d.nc;
  for (int s = 0; s < d.nseg; ++s) min_seg = std::min(min_seg, L.seg_user_start[s + 1] - L.seg_user_start[s]);
  DIFVM_CHECK(prm->p_ref_cell >= 0 && prm->p_ref_cell < min_seg, DIFVM_ERR_INVALID_ARG,
              "p_ref_cell out of range (it indexes cells of each segment)");
  difvm_piso* P = new difvm_piso();
  try {
    P->mesh = m;
    P->prm = *prm;
    size_t nc = d.nc, nf = (size_t)d.nfi + d.nfb;
    // reference cell of each segment that fixes no pressure value: its p_ref_cell-th user cell
    std::vector<int8_t> ref(nc, 0);
    const std::vector<int32_t>& cp = L.cell_perm;  // internal -> user
    for (size_t i = 0; i < nc; ++i) {
      int s = L.cell_seg[i];
      if (!L.seg_has_fixed_p[s] && cp[i] == L.seg_user_start[s] + prm->p_ref_cell) ref[i] = 1;
    }
    P->is_ref = dalloc<int8_t>(ctx_of(m), nc);
    P->allocs.push_back(P->is_ref);
    upload(P->is_ref, ref, stream_of(m));
    P->seg_nu.assign(d.nseg, prm->nu);
    P->seg_stats.assign(d.nseg, difvm_step_stats{});
    P->nu_cell = piso_alloc(P, nc);
    std::vector<double> nu0(nc, prm->nu);  // kept until the synchronisation below
    upload(P->nu_cell, nu0, stream_of(m));
    P->U = piso_alloc(P, 3 * nc); P->p = piso_alloc(P, nc); P->phi = piso_alloc(P, nf);
    P->Ub = piso_alloc(P, 3 * (size_t)d.nfb); P->pb = piso_alloc(P, d.nfb); P->pbv = piso_alloc(P, d.nfb);
    int nwk = std::max(1, d.n_wk);
    P->wk = piso_alloc(P, 3 * nwk); P->pc = piso_alloc(P, nwk); P->wk_out = piso_alloc(P, 2 * nwk);
    P->wk_host.assign(3 * nwk, 1.0);
    P->gU = piso_alloc(P, 9 * nc); P->gp = piso_alloc(P, 3 * nc); P->dM = piso_alloc(P, nc);
    P->valM = piso_alloc(P, d.nslot); P->bM = piso_alloc(P, 3 * nc); P->rhs = piso_alloc(P, 3 * nc);
    P->HbyA = piso_alloc(P, 3 * nc); P->rAU = piso_alloc(P, nc); P->phiH = piso_alloc(P, nf); P->aF = piso_alloc(P, nf);
    P->ncorr = piso_alloc(P, std::max<size_t>(1, d.nfi));
    P->dK = piso_alloc(P, nc); P->valK = piso_alloc(P, d.nslot); P->rhsK = piso_alloc(P, nc);
    upload(P->wk, P->wk_host, stream_of(m));
    DIFVM_HIP(hipStreamSynchronize(stream_of(m)));  // the host vectors above are temporaries
  } catch (...) {
    for (void* a : P->allocs) dfree(ctx_of(m), a);
    delete P;
    throw;
  }
  m->refs++;
  *out = P;
}

void piso_graph_free(difvm_piso* P);

void piso_release(difvm_piso* P) {
  if (!P || --P->refs > 0) return;
  difvm_mesh* m = P->mesh;
  (void)hipStreamSynchronize(stream_of(m));
  piso_graph_free(P);
  amg_free(P->amg);
  for (void* a : P->allocs) dfree(ctx_of(m), a);
  delete P;
  mesh_release(m);
}

void piso_set_boundary(difvm_piso* P, const double* Ub_user, const double* pb_user) {
  difvm_mesh* m = P->mesh;
  if (Ub_user) permute(m, DIFVM_F64, 3, DIFVM_KIND_BFACE, DIFVM_TO_INTERNAL, Ub_user, P->Ub);
  if (pb_user) permute(m, DIFVM_F64, 1, DIFVM_KIND_BFACE, DIFVM_TO_INTERNAL, pb_user, P->pb);
  DIFVM_HIP(hipMemcpyAsync(P->pbv, P->pb, sizeof(double) * m->d.nfb, hipMemcpyDeviceToDevice, stream_of(m)));
}

void piso_set_viscosity(difvm_piso* P, int nseg, const double* nu_seg) {
  difvm_mesh* m = P->mesh;
  const DMesh& d = m->d;
  DIFVM_CHECK(nseg == d.nseg, DIFVM_ERR_INVALID_ARG, "one viscosity per segment expected");
  for (int s = 0; s < nseg; ++s) DIFVM_CHECK(nu_seg[s] >= 0, DIFVM_ERR_INVALID_ARG, "viscosity must be >= 0");
  P->seg_nu.assign(nu_seg, nu_seg + nseg);
  std::vector<double> cell(d.nc);
  for (int i = 0; i < d.nc; ++i) cell[i] = P->seg_nu[m->host.cell_seg[i]];
  upload(P->nu_cell, cell, stream_of(m));
  DIFVM_HIP(hipStreamSynchronize(stream_of(m)));
}

// Passive scalar over one step with the current face flux: the momentum predictor's discretisation
// with one component, diffusivity D in place of the viscosity and the given boundary table.
SolveResult piso_transport_scalar(difvm_piso* P, double D, int table, const double* cb_user, double* c_user) {
  DIFVM_CHECK(D >= 0, DIFVM_ERR_INVALID_ARG, "D must be >= 0");
  DIFVM_CHECK(table >= 0 && table < N_TABLES, DIFVM_ERR_INVALID_ARG, "unknown boundary table");
  difvm_mesh* m = P->mesh;
  const DMesh& d = m->d;
  DIFVM_CHECK(cb_user || d.nfb == 0, DIFVM_ERR_INVALID_ARG, "c_b is NULL");
  hipStream_t s = stream_of(m);
  if (!P->sc) {
    P->sc = piso_alloc(P, d.nc); P->scb = piso_alloc(P, d.nfb); P->sg = piso_alloc(P, 3 * (size_t)d.nc);
    P->sd = piso_alloc(P, d.nc); P->sval = piso_alloc(P, d.nslot); P->sb = piso_alloc(P, d.nc);
  }
  permute(m, DIFVM_F64, 1, DIFVM_KIND_CELL, DIFVM_TO_INTERNAL, c_user, P->sc);
  if (d.nfb) permute(m, DIFVM_F64, 1, DIFVM_KIND_BFACE, DIFVM_TO_INTERNAL, cb_user, P->scb);
  op_grad(m, DIFVM_F64, 1, table, P->sc, P->scb, P->sg);
  launch_momentum<1>(m, P->prm.conv, time_theta(P->prm.time), table, D, nullptr, P->prm.dt, P->phi, P->sc, P->sg, P->scb, P->sd, nullptr,
                     nullptr, P->sval, P->sb);
  SolveResult r = bicgstab(m, 1, SellMatrix{P->sd, P->sval}, P->sb, P->sc, P->prm.tol_u, P->prm.maxit_u, nullptr,
                           &P->hint_sc);
  permute(m, DIFVM_F64, 1, DIFVM_KIND_CELL, DIFVM_FROM_INTERNAL, P->sc, c_user);
  DIFVM_HIP(hipStreamSynchronize(s));
  return r;
}

void piso_segment_stats(const difvm_piso* P, int nseg, difvm_step_stats* out) {
  DIFVM_CHECK(nseg == P->mesh->d.nseg, DIFVM_ERR_INVALID_ARG, "n_seg differs from the mesh's segment count");
  for (int s = 0; s < nseg; ++s) out[s] = P->seg_stats[s];
}

void piso_set_windkessel(difvm_piso* P, int id, double Rp, double C, double Rd, double pc) {
  DIFVM_CHECK(id >= 0 && id < P->mesh->d.n_wk, DIFVM_ERR_INVALID_ARG, "Windkessel id out of range");
  DIFVM_CHECK(Rp >= 0 && C > 0 && Rd > 0, DIFVM_ERR_INVALID_ARG, "Windkessel needs Rp >= 0, C > 0, Rd > 0");
  P->wk_host[3 * id] = Rp;
  P->wk_host[3 * id + 1] = C;
  P->wk_host[3 * id + 2] = Rd;
  hipStream_t s = stream_of(P->mesh);
  DIFVM_HIP(hipMemcpyAsync(P->wk + 3 * id, &P->wk_host[3 * id], 3 * sizeof(double), hipMemcpyHostToDevice, s));
  DIFVM_HIP(hipMemcpyAsync(P->pc + id, &pc, sizeof(double), hipMemcpyHostToDevice, s));
  DIFVM_HIP(hipStreamSynchronize(s));  // the host scalars are on the stack
}

void piso_set_state(difvm_piso* P, const double* U, const double* p, const double* phi) {
  difvm_mesh* m = P->mesh;
  const DMesh& d = m->d;
  if (U) permute(m, DIFVM_F64, 3, DIFVM_KIND_CELL, DIFVM_TO_INTERNAL, U, P->U);
  if (p) permute(m, DIFVM_F64, 1, DIFVM_KIND_CELL, DIFVM_TO_INTERNAL, p, P->p);
  if (phi) {
    permute(m, DIFVM_F64, 1, DIFVM_KIND_FACE_FLUX, DIFVM_TO_INTERNAL, phi, P->phi);
  } else {
    int nf = d.nfi + d.nfb;
    k_initial_flux<<<grid_for(nf), BLOCK, 0, stream_of(m)>>>(view<double>(d), P->U, P->Ub, P->phi);
    DIFVM_HIP(hipGetLastError());
  }
}

void piso_get_state(difvm_piso* P, double* U, double* p, double* phi, double* pc_host) {
  difvm_mesh* m = P->mesh;
  if (U) permute(m, DIFVM_F64, 3, DIFVM_KIND_CELL, DIFVM_FROM_INTERNAL, P->U, U);
  if (p) permute(m, DIFVM_F64, 1, DIFVM_KIND_CELL, DIFVM_FROM_INTERNAL, P->p, p);
  if (phi) permute(m, DIFVM_F64, 1, DIFVM_KIND_FACE_FLUX, DIFVM_FROM_INTERNAL, P->phi, phi);
  if (pc_host && m->d.n_wk)
    DIFVM_HIP(hipMemcpyAsync(pc_host, P->pc, sizeof(double) * m->d.n_wk, hipMemcpyDeviceToHost, stream_of(m)));
  DIFVM_HIP(hipStreamSynchronize(stream_of(m)));
}

void piso_pressure_matrix(difvm_piso* P, const double* HbyA, const double* rAU, const double* gp, const double* pbv) {
  difvm_mesh* m = P->mesh;
  const DMesh& d = m->d;
  hipStream_t s = stream_of(m);
  MeshView<double> mv = view<double>(d);
  k_pface<<<grid_for(d.nfi + d.nfb), BLOCK, 0, s>>>(mv, HbyA, rAU, gp, P->Ub, P->phiH, P->aF, P->ncorr);
  k_passemble<<<grid_for(d.nc), BLOCK, 0, s>>>(mv, P->phiH, P->aF, P->ncorr, pbv, P->is_ref, P->prm.p_ref_value,
                                               P->dK, P->valK, P->rhsK);
  DIFVM_HIP(hipGetLastError());
}

// device-to-device copies are kernels, so a captured step or adjoint segment holds kernel nodes only
__global__ void k_dcopy(double* __restrict__ dst, const double* __restrict__ src, size_t n) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = src[q];
}
static void dcopy_k(double* dst, const double* src, size_t n, hipStream_t s) {
  if (!n) return;
  k_dcopy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dst, src, n);
  DIFVM_HIP(hipGetLastError());
}
void dcopy(double* dst, const double* src, size_t n, hipStream_t s) { dcopy_k(dst, src, n, s); }

static void set_seg_stats_u(difvm_piso* P, const SolveResult& ru) {
  for (size_t g = 0; g < P->seg_stats.size(); ++g) {
    difvm_step_stats& sg = P->seg_stats[g];
    sg = difvm_step_stats{};
    for (int c = 0; c < 3; ++c) {
      sg.it_u[c] = ru.seg[g].iters[c];
      sg.res_u[c] = ru.seg[g].res[c];
    }
    sg.status = ru.seg[g].status;
  }
}

static void set_seg_stats_p(difvm_piso* P, int corr, const SolveResult& rp) {
  for (size_t g = 0; g < P->seg_stats.size(); ++g) {
    difvm_step_stats& sg = P->seg_stats[g];
    sg.it_p[corr] = rp.seg[g].iters[0];
    sg.res_p[corr] = rp.seg[g].res[0];
    sg.status = std::max(sg.status, rp.seg[g].status);
  }
}

void piso_advance(difvm_piso* P, difvm_step_stats* stp, StepRecord* rec) { piso_advance_q(P, stp, rec, nullptr); }

void piso_advance_q(difvm_piso* P, difvm_step_stats* stp, StepRecord* rec, const StepQueue* qu) {
  difvm_mesh* m = P->mesh;
  const DMesh& d = m->d;
  hipStream_t s = stream_of(m);
  MeshView<double> mv = view<double>(d);
  const difvm_piso_params& prm = P->prm;
  int Gc = grid_for(d.nc), Gf = grid_for(d.nfi + d.nfb);
  size_t nc = d.nc;
  difvm_step_stats st{};
  // phases of the step timed with events while the context's phase profiling is on (eager steps only)
  PhaseScope ph(m, "step: momentum assembly");
  // S0
  if (rec) dcopy(rec->phi_in, P->phi, (size_t)d.nfi + d.nfb, s);
  if (rec && d.n_wk) dcopy(rec->pc_in, P->pc, d.n_wk, s);
  if (d.n_wk)
    k_windkessel<<<d.n_wk, BLOCK, 0, s>>>(d.nfi, prm.dt, d.wk_start, d.wk_faces, P->phi, P->wk, P->pc, P->pbv, P->wk_out);
  if (rec) {
    dcopy(rec->pbv, P->pbv, d.nfb, s);
    if (d.n_wk) dcopy(rec->wk_out, P->wk_out, 2 * (size_t)d.n_wk, s);
  }
  // S1
  op_grad(m, DIFVM_F64, 3, DIFVM_BC_U, P->U, P->Ub, P->gU);
  if (rec && rec->Un) dcopy(rec->Un, P->U, 3 * nc, s);
  op_assemble_momentum(m, prm.conv, prm.time, prm.nu, P->nu_cell, prm.dt, P->phi, P->U, P->gU, P->Ub, P->dM, nullptr, nullptr,
                       P->valM, P->bM);
  ph.next("step: momentum solve");
  // S2
  op_grad(m, DIFVM_F64, 1, DIFVM_BC_P, P->p, P->pbv, P->gp);
  k_pred_rhs<<<grid_for(3 * d.nc), BLOCK, 0, s>>>(d.nc, d.V, P->bM, P->gp, P->rhs);
  DIFVM_HIP(hipGetLastError());
  SolveResult ru = bicgstab(m, 3, SellMatrix{P->dM, P->valM}, P->rhs, P->U, prm.tol_u, prm.maxit_u, qu ? &qu->u : nullptr,
                            &P->hint_u);
  for (int c = 0; c < 3; ++c) { st.it_u[c] = ru.iters[c]; st.res_u[c] = ru.res[c]; }
  st.status = ru.status;
  if (!qu) set_seg_stats_u(P, ru);
  if (P->trace_U) dcopy(P->trace_U, P->U, 3 * nc, s);
  if (rec) {
    dcopy(rec->dM, P->dM, nc, s);
    dcopy(rec->valM, P->valM, d.nslot, s);
    dcopy(rec->Ustar, P->U, 3 * nc, s);
  }
  // S3
  for (int corr = 0; corr < prm.n_corr; ++corr) {
    ph.next("step: pressure assembly");
    if (rec) {
      dcopy(rec->Uin[corr], P->U, 3 * nc, s);
      dcopy(rec->pold[corr], P->p, nc, s);
    }
    k_hbya<<<Gc, BLOCK, 0, s>>>(d.nc, d.slice_start, d.uw, d.slot_col, P->valM, P->dM, d.V, P->bM, P->U, P->HbyA, P->rAU);
    // grad of the entering pressure: at the first corrector p and its boundary values are those of the
    // predictor, whose gradient P->gp still holds
    if (corr > 0) op_grad(m, DIFVM_F64, 1, DIFVM_BC_P, P->p, P->pbv, P->gp);
    if (rec) {
      dcopy(rec->HbyA[corr], P->HbyA, 3 * nc, s);
      dcopy(rec->gpo[corr], P->gp, 3 * nc, s);
      if (corr == 0) dcopy(rec->rAU, P->rAU, nc, s);
    }
    k_pface<<<Gf, BLOCK, 0, s>>>(mv, P->HbyA, P->rAU, P->gp, P->Ub, P->phiH, P->aF, P->ncorr);
    k_passemble<<<Gc, BLOCK, 0, s>>>(mv, P->phiH, P->aF, P->ncorr, P->pbv, P->is_ref, prm.p_ref_value, P->dK, P->valK,
                                     P->rhsK);
    DIFVM_HIP(hipGetLastError());
    ph.end();  // (the AMG setup, once, is not part of a phase)
    if (prm.precond == DIFVM_PRECOND_AMG && !P->amg) {
      DIFVM_CHECK(!ctx_of(m).capturing, DIFVM_ERR_INVALID_ARG, "AMG hierarchy must exist before a step is captured");
      P->amg = amg_create(m, SellMatrix{P->dK, P->valK}, AmgOptions{});
    }
    ph.next("step: pressure solve");
    SolveResult rp = pcg(m, SellMatrix{P->dK, P->valK}, P->rhsK, P->p, prm.tol_p, prm.maxit_p, qu ? &qu->p[corr] : nullptr,
                         P->amg, &P->hint_p[corr]);
    st.it_p[corr] = rp.iters[0];
    st.res_p[corr] = rp.res[0];
    st.status = std::max(st.status, rp.status);
    if (!qu) set_seg_stats_p(P, corr, rp);
    ph.next("step: correction");
    if (P->trace_p) dcopy(P->trace_p + (size_t)corr * nc, P->p, nc, s);
    k_flux<<<Gf, BLOCK, 0, s>>>(mv, P->phiH, P->aF, P->ncorr, P->p, P->pbv, P->phi);
    k_ucorr<<<Gc, BLOCK, 0, s>>>(mv, P->p, P->pbv, P->HbyA, P->rAU, P->U);
    DIFVM_HIP(hipGetLastError());
    ph.end();
    if (rec) {
      dcopy(rec->pnew[corr], P->p, nc, s);
      op_grad(m, DIFVM_F64, 1, DIFVM_BC_P, P->p, P->pbv, rec->gpn[corr]);
    }
  }
  if (stp) *stp = st;
}

// ---------------------------------------------------------------------------------------------
// Graph mode.  The step (Windkessel, assembly, BiCGStab, correctors) is captured once on a private
// stream with a fixed iteration budget per solve and replayed with one hipGraphLaunch per step; the
// host reads the solver states once per step.  Iterations past a solve's stop are predicated no-ops,
// so a replay computes what the eager step computes.  A replay in which some solve had not stopped
// within its budget is discarded: the state saved by the graph's first node is restored and the
// step is run eagerly, then the graph is recaptured with budgets from the new counts.
// ---------------------------------------------------------------------------------------------

static size_t state_words(const DMesh& d) { return 4 * (size_t)d.nc + d.nfi + d.nfb + std::max(1, d.n_wk); }

// save (to backup) or restore (from backup) U, p, phi, pc
static void backup_state(difvm_piso* P, bool save, hipStream_t s) {
  const DMesh& d = P->mesh->d;
  double* b = P->g.backup;
  size_t nc = d.nc, nf = (size_t)d.nfi + d.nfb, nw = std::max(1, d.n_wk);
  double* dev[4] = {P->U, P->p, P->phi, P->pc};
  size_t len[4] = {3 * nc, nc, nf, nw};
  for (int k = 0; k < 4; ++k) {
    if (save) dcopy_k(b, dev[k], len[k], s);
    else dcopy_k(dev[k], b, len[k], s);
    b += len[k];
  }
}

static void graph_drop(PisoGraph& G) {
  if (G.exec) (void)hipGraphExecDestroy(G.exec);
  if (G.graph) (void)hipGraphDestroy(G.graph);
  G.exec = nullptr;
  G.graph = nullptr;
}

void piso_graph_free(difvm_piso* P) {
  PisoGraph& G = P->g;
  graph_drop(G);
  if (G.cap) (void)hipStreamDestroy(G.cap);
  if (G.state_host) (void)hipHostFree(G.state_host);
  G.cap = nullptr;
  G.state_host = nullptr;
  // state_dev and backup are in P->allocs
}

static void graph_capture(difvm_piso* P) {
  PisoGraph& G = P->g;
  difvm_mesh* m = P->mesh;
  Ctx& c = ctx_of(m);
  StepQueue qu;
  char* st = static_cast<char*>(G.state_dev);
  qu.u = QueueOnly{G.budget_u, st};
  for (int k = 0; k < P->prm.n_corr; ++k) qu.p[k] = QueueOnly{G.budget_p[k], st + G.bytes_u + k * G.bytes_p};
  hipStream_t orig = c.stream;
  c.stream = G.cap;
  c.capturing = true;
  DIFVM_HIP(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
  try {
    backup_state(P, true, G.cap);
    piso_advance_q(P, nullptr, nullptr, &qu);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(G.cap, &g);
    if (g) (void)hipGraphDestroy(g);
    c.stream = orig;
    c.capturing = false;
    throw;
  }
  hipError_t e = hipStreamEndCapture(G.cap, &G.graph);
  c.stream = orig;
  c.capturing = false;
  DIFVM_HIP(e);
  DIFVM_HIP(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
  G.captures++;
}

// Budgets track the counts: a solve's budget is the largest count of its kind (BiCGStab components,
// or pressure correctors) over the last few steps, plus the margin and 1/64 of that count (long
// Jacobi solves drift by a few per cent from step to step).  A replay in which some solve ran out of
// budget is redone eagerly and widens the margin by one (up to extra); once the recent counts have
// fallen two or more below the budgets, the step is recaptured with tighter ones.  Idle iterations
// of a replay (past every solve's stop) are predicated no-ops but still launches, about 30 us each
// with the AMG V-cycle at 1M cells, so budgets close to the counts keep replays cheap.
static void push_counts(PisoGraph& G, const difvm_step_stats& st, int n_corr) {
  int mu = std::max(st.it_u[0], std::max(st.it_u[1], st.it_u[2]));
  int mp = 0;
  for (int k = 0; k < n_corr; ++k) mp = std::max(mp, st.it_p[k]);
  G.hist_u[G.hist_at] = mu;
  G.hist_p[G.hist_at] = mp;
  G.hist_at = (G.hist_at + 1) % PisoGraph::HIST;
  G.nhist = std::min(G.nhist + 1, PisoGraph::HIST);
}

static void wanted_budgets(const PisoGraph& G, int* bu, int* bp) {
  int mu = 0, mp = 0;
  for (int k = 0; k < G.nhist; ++k) {
    mu = std::max(mu, G.hist_u[k]);
    mp = std::max(mp, G.hist_p[k]);
  }
  *bu = mu + G.margin + mu / 64;
  *bp = mp + G.margin + mp / 64;
}

static void set_budgets(difvm_piso* P, bool grow_only) {
  PisoGraph& G = P->g;
  int bu, bp;
  wanted_budgets(G, &bu, &bp);
  G.budget_u = grow_only ? std::max(G.budget_u, bu) : bu;
  for (int k = 0; k < P->prm.n_corr; ++k) G.budget_p[k] = grow_only ? std::max(G.budget_p[k], bp) : bp;
}

static void graph_step(difvm_piso* P, difvm_step_stats* out) {
  PisoGraph& G = P->g;
  difvm_mesh* m = P->mesh;
  hipStream_t s = stream_of(m);
  difvm_step_stats st{};
  if (!G.exec) {
    // learn the iteration counts eagerly, then capture with budgets from them
    piso_advance(P, &st, nullptr);
    push_counts(G, st, P->prm.n_corr);
    set_budgets(P, false);
    graph_capture(P);
    *out = st;
    return;
  }
  DIFVM_HIP(hipGraphLaunch(G.exec, s));
  size_t bytes = G.bytes_u + (size_t)P->prm.n_corr * G.bytes_p;
  DIFVM_HIP(hipMemcpyAsync(G.state_host, G.state_dev, bytes, hipMemcpyDeviceToHost, s));
  DIFVM_HIP(hipStreamSynchronize(s));
  const char* hs = static_cast<const char*>(G.state_host);
  bool ok = true, c1 = true;
  SolveResult ru = bicgstab_result(m, 3, hs, &c1);
  ok = ok && c1;
  SolveResult rp[StepRecord::MAXC];
  for (int k = 0; k < P->prm.n_corr; ++k) {
    rp[k] = pcg_result(m, hs + G.bytes_u + k * G.bytes_p, &c1);
    ok = ok && c1;
  }
  if (!ok) {
    // some solve needed more than its budget: discard the replay, redo the step eagerly, widen the
    // margin and recapture
    backup_state(P, false, s);
    piso_advance(P, &st, nullptr);
    push_counts(G, st, P->prm.n_corr);
    G.margin = std::min(G.margin + 1, G.extra);
    set_budgets(P, true);
    graph_drop(G);
    graph_capture(P);
    G.redos++;
    *out = st;
    return;
  }
  G.replays++;  // kept replays only; a discarded one counts as a redo
  for (int c = 0; c < 3; ++c) {
    st.it_u[c] = ru.iters[c];
    st.res_u[c] = ru.res[c];
  }
  st.status = ru.status;
  set_seg_stats_u(P, ru);
  for (int k = 0; k < P->prm.n_corr; ++k) {
    st.it_p[k] = rp[k].iters[0];
    st.res_p[k] = rp[k].res[0];
    st.status = std::max(st.status, rp[k].status);
    set_seg_stats_p(P, k, rp[k]);
  }
  *out = st;
  // tighten the budgets once the recent counts sit two or more below them
  push_counts(G, st, P->prm.n_corr);
  int bu, bp;
  wanted_budgets(G, &bu, &bp);
  bool slack = G.budget_u - bu >= 2;
  for (int k = 0; k < P->prm.n_corr; ++k) slack = slack || G.budget_p[k] - bp >= 2;
  if (slack && G.nhist >= 4) {
    set_budgets(P, false);
    graph_drop(G);
    graph_capture(P);
  }
}

void piso_set_graph(difvm_piso* P, int enable, int extra) {
  DIFVM_CHECK(extra >= 0, DIFVM_ERR_INVALID_ARG, "extra_iters must be >= 0");
  PisoGraph& G = P->g;
  graph_drop(G);
  G.on = enable != 0;
  G.extra = extra;
  G.margin = std::min(1, extra);
  G.nhist = G.hist_at = 0;
  if (!G.on) return;
  difvm_mesh* m = P->mesh;
  const DMesh& d = m->d;
  if (!G.cap) DIFVM_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
  G.bytes_u = bicgstab_state_bytes(m);
  G.bytes_p = pcg_state_bytes(m);
  size_t bytes = G.bytes_u + (size_t)StepRecord::MAXC * G.bytes_p;
  if (!G.state_dev) {
    G.state_dev = piso_alloc(P, (bytes + 7) / 8);
    G.backup = piso_alloc(P, state_words(d));
    DIFVM_HIP(hipHostMalloc(&G.state_host, bytes, hipHostMallocDefault));
  }
}

// drops the pressure preconditioner's hierarchy (and a captured step that uses it): the next AMG
// solve builds one from its own matrix
void piso_rebuild_preconditioner(difvm_piso* P) {
  DIFVM_CHECK(P->prm.precond == DIFVM_PRECOND_AMG, DIFVM_ERR_INVALID_ARG, "the PISO object does not use AMG");
  graph_drop(P->g);
  amg_free(P->amg);
  P->amg = nullptr;
}

void piso_precond_info(const difvm_piso* P, int32_t* n_levels, int32_t* rows, int32_t cap, double* vcycle_bytes) {
  DIFVM_CHECK(P->prm.precond == DIFVM_PRECOND_AMG, DIFVM_ERR_INVALID_ARG, "the PISO object does not use AMG");
  *n_levels = 0;
  if (vcycle_bytes) *vcycle_bytes = 0.0;
  if (!P->amg) return;
  int r[64];
  int n = amg_levels(P->amg, r, 64);
  *n_levels = n;
  for (int l = 0; l < n && l < cap; ++l) rows[l] = r[l];
  if (vcycle_bytes) *vcycle_bytes = amg_vcycle_bytes(P->amg);
}

void piso_graph_info(const difvm_piso* P, long long* replays, long long* redos, long long* captures) {
  if (replays) *replays = P->g.replays;
  if (redos) *redos = P->g.redos;
  if (captures) *captures = P->g.captures;
}

// One eager step that also hands out the solution of each linear solve (user order, device arrays):
// the predictor's U* and the pressure solved by each corrector.  The internal-order copies live in
// buffers of the PISO object made at the first call.
int piso_step_trace(difvm_piso* P, double* Ustar_user, double* p_user, difvm_step_stats* stats) {
  difvm_mesh* m = P->mesh;
  const DMesh& d = m->d;
  size_t nc = d.nc;
  if (!P->trace_buf) P->trace_buf = piso_alloc(P, 3 * nc + (size_t)StepRecord::MAXC * nc);
  P->trace_U = P->trace_buf;
  P->trace_p = P->trace_buf + 3 * nc;
  difvm_step_stats st{};
  try {
    piso_advance(P, &st, nullptr);
  } catch (...) {
    P->trace_U = P->trace_p = nullptr;
    throw;
  }
  P->trace_U = P->trace_p = nullptr;
  permute(m, DIFVM_F64, 3, DIFVM_KIND_CELL, DIFVM_FROM_INTERNAL, P->trace_buf, Ustar_user);
  for (int c = 0; c < P->prm.n_corr; ++c)
    permute(m, DIFVM_F64, 1, DIFVM_KIND_CELL, DIFVM_FROM_INTERNAL, P->trace_buf + 3 * nc + (size_t)c * nc,
            p_user + (size_t)c * nc);
  DIFVM_HIP(hipStreamSynchronize(stream_of(m)));
  if (stats) *stats = st;
  return st.status;
}

int piso_step(difvm_piso* P, int nsteps, difvm_step_stats* stats) {
  int worst = 0;
  for (int step = 0; step < nsteps; ++step) {
    difvm_step_stats st{};
    if (P->g.on) graph_step(P, &st);
    else piso_advance(P, &st, nullptr);
    worst = std::max(worst, st.status);
    if (stats) stats[step] = st;
  }
  DIFVM_HIP(hipStreamSynchronize(stream_of(P->mesh)));
  return worst;
}

}  // namespace difvm
