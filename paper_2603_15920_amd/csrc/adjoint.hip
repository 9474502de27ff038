// Discrete adjoint of the PISO step and its checkpointed N-step window (paper Sec. "End-to-End
// Automatic Differentiation": reverse mode through the time loop, eq. vjp; checkpointing, eq.
// checkpointing; linear solves differentiated implicitly with the same solver, eq. implicit_diff;
// Windkessel parameters as leaves, Sec. "Windkessel RCR outlet condition").
//
// Given the lagged flux phi^n, one step is linear in (U^n, p^n, boundary pressures); it depends
// nonlinearly on phi^n only through the momentum coefficients (upwind branches, frozen in reverse:
// d max(F,0)/dF = 1 for F >= 0) and on the Windkessel parameters through the exponential update.
// The reverse step walks the forward operations backwards:
//   gather  (cell reads neighbours)      -> transpose is a scatter, written here as a gather of
//                                           per-face cotangents by each cell in slot order
//   solve   A x = b                      -> A^T lambda = xbar with the same Krylov solver
//                                           (momentum: owner/neighbour coefficients swapped;
//                                           pressure: symmetric), then bbar += lambda and
//                                           Abar = -lambda x^T on the sparsity pattern.
// No atomics: every cotangent array is written by the thread owning its row, cell or face.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "abi_util.h"
#include "dc.h"
#include "device.h"
#include "ops.h"
#include "piso_internal.h"

namespace difvm {

// ---------------------------------------------------------------------------------------------
// transposed operators
// ---------------------------------------------------------------------------------------------
// Adjoint of the Gauss gradient: gbar[nc][NC][3] -> phibar[nc][NC] (+=) and, on fixed-value
// boundary faces, phib_bar[nfb][NC] (+=, may be NULL).  For an internal face the cotangent of the
// face value is (gbar_O/V_O - gbar_N/V_N).S, shared to O and N with the interpolation weights.
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_gradT(MeshView<double> m, int table, const double* __restrict__ gbar,
                                                 double* __restrict__ phibar, double* __restrict__ phib_bar) {
  const int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i < m.nc) {
    SlotRange R = slots_of(m, i);
    double rvi = 1.0 / m.V[i];
    double gi[NC][3];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int e = 0; e < 3; ++e) gi[c][e] = gbar[((size_t)i * NC + c) * 3 + e] * rvi;
    double acc[NC], pb0[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      acc[c] = 0.0;
      pb0[c] = phibar[(size_t)i * NC + c];  // read before the row's loads, added after
    }
    const int8_t* code = m.bcode + table * m.nfb;
    // slots in layout order; for one component the first four with every load issued before any
    // is used (indices in range whatever the slot holds).  For three components one at a time: two
    // at a time took 47.7 µs against 42.6 at 401k cells (nine gathered values per slot), and staging
    // the rows' stores through LDS made either form slower still.
    walk_row<(NC == 3 ? 1 : 4)>(R.width, [&](auto Wc, int k0) {
      constexpr int N = decltype(Wc)::value;
      int sf[N], j[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        int at = R.base + (k0 + k) * SLICE;
        sf[k] = m.slot_face[at];
        j[k] = m.slot_col[at];
      }
      Geo<double>::v4 g[N];
      double vj[N], gj[N][NC][3];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        g[k] = m.geomS[slot_face_index(sf[k], m.nfi)];
        vj[k] = m.V[j[k]];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int e = 0; e < 3; ++e) gj[k][c][e] = gbar[((size_t)j[k] * NC + c) * 3 + e];
      }
#pragma unroll
      for (int k = 0; k < N; ++k) {
        if (sf[k] == SLOT_PAD) continue;
        if (sf[k] < m.nfi) {
          bool nb = sf[k] < 0;
          double wself = nb ? 1.0 - g[k].w : g[k].w;
          double sg = nb ? -1.0 : 1.0;
          double rvj = 1.0 / vj[k];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            double t = (gi[c][0] - gj[k][c][0] * rvj) * g[k].x + (gi[c][1] - gj[k][c][1] * rvj) * g[k].y +
                       (gi[c][2] - gj[k][c][2] * rvj) * g[k].z;
            acc[c] += wself * sg * t;
          }
        } else {
          int b = sf[k] - m.nfi;
          auto gb = m.bgeom[b];
          bool fixed = code[b] == BC_FIXED;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            double t = gi[c][0] * gb.x + gi[c][1] * gb.y + gi[c][2] * gb.z;
            if (fixed) {
              if (phib_bar) phib_bar[(size_t)b * NC + c] += t;
            } else {
              acc[c] += t;
            }
          }
        }
      }
    });
#pragma unroll
    for (int c = 0; c < NC; ++c) phibar[(size_t)i * NC + c] = pb0[c] + acc[c];
  }
}

// transposed momentum off-diagonals: the slot of (O,N) takes the coefficient of (N,O) and back
__global__ __launch_bounds__(BLOCK) void k_swap_slots(int nfi, const int32_t* __restrict__ own_slot,
                                                      const int32_t* __restrict__ nbr_slot, const double* __restrict__ val,
                                                      double* __restrict__ valT) {
  int f = blockIdx.x * BLOCK + threadIdx.x;
  if (f >= nfi) return;
  int a = own_slot[f], b = nbr_slot[f];
  valT[a] = val[b];
  valT[b] = val[a];
}

// ---------------------------------------------------------------------------------------------
// reverse of the correctors
// ---------------------------------------------------------------------------------------------
// U = HbyA - rAU grad(p):  HbyAbar = Ubar, rAUbar -= Ubar.grad(p), gbar = -rAU Ubar
__global__ __launch_bounds__(BLOCK) void k_adj_ucorr(int nc, const double* __restrict__ Ubar, const double* __restrict__ gpn,
                                                     const double* __restrict__ rAU, double* __restrict__ HbyAbar,
                                                     double* __restrict__ rAUbar, double* __restrict__ gbar) {
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= nc) return;
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double u = Ubar[3 * (size_t)i + c];
    HbyAbar[3 * (size_t)i + c] = u;
    s += u * gpn[3 * (size_t)i + c];
    gbar[3 * (size_t)i + c] = -rAU[i] * u;
  }
  rAUbar[i] -= s;
}

// cotangents of the face quantities of a corrector, seeded by the step's output flux
// (phi = phiH - aF (p_N - p_O) - ncorr; boundary: fixed p: phiH - aF_b (p_b - p_O); else phiH)
__global__ __launch_bounds__(BLOCK) void k_adj_flux(MeshView<double> m, int seed, const double* __restrict__ phibar,
                                                    const double* __restrict__ rAU, const double* __restrict__ p,
                                                    const double* __restrict__ pbv, double* __restrict__ fHb,
                                                    double* __restrict__ faF, double* __restrict__ fnc,
                                                    double* __restrict__ g, double* __restrict__ pbvbar) {
  int f = blockIdx.x * BLOCK + threadIdx.x;
  if (f < m.nfi) {
    double fb = seed ? phibar[f] : 0.0;
    int O = m.own[f], N = m.nbr[f];
    double w = m.w[f];
    double aF = (w * rAU[O] + (1.0 - w) * rAU[N]) * m.geomK[f].w;
    fHb[f] = fb;
    faF[f] = -fb * (p[N] - p[O]);
    fnc[f] = -fb;
    g[f] = aF * fb;
  } else if (f < m.nfi + m.nfb) {
    int b = f - m.nfi;
    double fb = seed ? phibar[f] : 0.0;
    int8_t cp = m.bcode[DIFVM_BC_P * m.nfb + b];
    int O = m.bown[b];
    fHb[f] = cp == BC_EMPTY ? 0.0 : fb;
    faF[f] = 0.0;
    g[f] = 0.0;
    if (cp == BC_FIXED) {
      double aF = rAU[O] * m.bgeom[b].w;
      faF[f] = -fb * (pbv[b] - p[O]);
      pbvbar[b] -= aF * fb;
      g[f] = aF * fb;
    }
  }
}

// after the pressure solve: lambda = K^-1 pbar.  K pattern cotangent -lambda p^T, right-hand side
// cotangent lambda, pushed to the face quantities (aF, phiH, ncorr) and the boundary pressures
__global__ __launch_bounds__(BLOCK) void k_adj_psolve(MeshView<double> m, const double* __restrict__ lam,
                                                      const double* __restrict__ p, const double* __restrict__ rAU,
                                                      const double* __restrict__ pbv,
                                                      const int8_t* __restrict__ is_ref, double pref,
                                                      double* __restrict__ fHb, double* __restrict__ faF,
                                                      double* __restrict__ fnc, double* __restrict__ pbvbar) {
  int f = blockIdx.x * BLOCK + threadIdx.x;
  if (f < m.nfi) {
    int O = m.own[f], N = m.nbr[f];
    double dl = lam[N] - lam[O], dp = p[N] - p[O];
    double a = -dl * dp;
    // reference row (doubled diagonal, d pref on the right): a segment holds at most one such cell
    if (is_ref[O]) a += lam[O] * (pref - p[O]);
    if (is_ref[N]) a += lam[N] * (pref - p[N]);
    faF[f] += a;
    fHb[f] += dl;
    fnc[f] -= dl;
  } else if (f < m.nfi + m.nfb) {
    int b = f - m.nfi;
    int8_t cp = m.bcode[DIFVM_BC_P * m.nfb + b];
    if (cp == BC_EMPTY) return;
    int O = m.bown[b];
    double lo = lam[O];
    fHb[f] -= lo;
    if (cp == BC_FIXED) {
      faF[f] += lo * (pbv[b] - p[O]);
      pbvbar[b] += rAU[O] * m.bgeom[b].w * lo;
    }
  }
}

// face cotangents -> cells: rAU_f = w rAU_O + (1-w) rAU_N with rAUbar_f = aFbar delta + ncbar k.gbar,
// phiH_f = interp(HbyA).S, ncorr_f = rAU_f k.interp(grad p_old)
__global__ __launch_bounds__(BLOCK) void k_adj_corr_cells(MeshView<double> m, const double* __restrict__ fHb,
                                                          const double* __restrict__ faF, const double* __restrict__ fnc,
                                                          const double* __restrict__ rAU, const double* __restrict__ gpo,
                                                          double* __restrict__ rAUbar, double* __restrict__ HbyAbar,
                                                          double* __restrict__ gpobar) {
  const int base = xcd_tile(blockIdx.x, gridDim.x) * BLOCK;
  const int i = base + threadIdx.x;
  __shared__ double lds[3 * BLOCK];
  double hout[3], gb[3] = {0.0, 0.0, 0.0};
  if (i < m.nc) {
    SlotRange R = slots_of(m, i);
    double ra = 0.0, hb[3] = {0.0, 0.0, 0.0};
    double gi[3] = {gpo[3 * (size_t)i], gpo[3 * (size_t)i + 1], gpo[3 * (size_t)i + 2]};
    const double rAUi = rAU[i];
    // the accumulated cotangents of this cell, read before the row's loads and added after
    const double ra0 = rAUbar[i];
    double hb0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) hb0[c] = HbyAbar[3 * (size_t)i + c];
    const int8_t* codeU = m.bcode + DIFVM_BC_U * m.nfb;
    const int8_t* codeP = m.bcode + DIFVM_BC_P * m.nfb;
    // slots in layout order, two at a time with every load issued before any is used
    walk_row<2>(R.width, [&](auto Wc, int k0) {
      constexpr int N = decltype(Wc)::value;
      int sf[N], j[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        int at = R.base + (k0 + k) * SLICE;
        sf[k] = m.slot_face[at];
        j[k] = m.slot_col[at];
      }
      Geo<double>::v4 g[N], kd[N];
      double rj[N], gj[N][3], ncf[N], af[N], hf[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        int f = slot_face_index(sf[k], m.nfi);  // 0 for boundary and padding slots
        g[k] = m.geomS[f];
        kd[k] = m.geomK[f];
        ncf[k] = fnc[f];
        af[k] = faF[f];
        hf[k] = fHb[f];
        rj[k] = rAU[j[k]];
#pragma unroll
        for (int e = 0; e < 3; ++e) gj[k][e] = gpo[3 * (size_t)j[k] + e];
      }
#pragma unroll
      for (int k = 0; k < N; ++k) {
        if (sf[k] == SLOT_PAD) continue;
        if (sf[k] < m.nfi) {
          bool nb = sf[k] < 0;
          double wself = nb ? 1.0 - g[k].w : g[k].w;
          double rf = wself * rAUi + (1.0 - wself) * rj[k];
          double kg = kd[k].x * (wself * gi[0] + (1.0 - wself) * gj[k][0]) +
                      kd[k].y * (wself * gi[1] + (1.0 - wself) * gj[k][1]) +
                      kd[k].z * (wself * gi[2] + (1.0 - wself) * gj[k][2]);
          ra += wself * (af[k] * kd[k].w + ncf[k] * kg);
          double h = wself * hf[k];
          hb[0] += h * g[k].x;
          hb[1] += h * g[k].y;
          hb[2] += h * g[k].z;
          double t = wself * ncf[k] * rf;
          gb[0] += t * kd[k].x;
          gb[1] += t * kd[k].y;
          gb[2] += t * kd[k].z;
        } else {
          int b = sf[k] - m.nfi;
          auto gbd = m.bgeom[b];
          if (codeP[b] == BC_FIXED) ra += faF[m.nfi + b] * gbd.w;
          if (codeU[b] == BC_ZEROGRAD) {
            double h = fHb[m.nfi + b];
            hb[0] += h * gbd.x;
            hb[1] += h * gbd.y;
            hb[2] += h * gbd.z;
          }
        }
      }
    });
    rAUbar[i] = ra0 + ra;
#pragma unroll
    for (int c = 0; c < 3; ++c) hout[c] = hb0[c] + hb[c];
  }
  store_rows<3>(HbyAbar, base, m.nc, hout, lds);
  store_rows<3>(gpobar, base, m.nc, gb, lds);
}

// HbyA = H / d: Hbar = HbyAbar / d, dbar -= HbyAbar.HbyA / d, bbar += Hbar
__global__ __launch_bounds__(BLOCK) void k_adj_hbya(int nc, const double* __restrict__ HbyAbar,
                                                    const double* __restrict__ HbyA, const double* __restrict__ dM,
                                                    double* __restrict__ Hbar, double* __restrict__ dbar,
                                                    double* __restrict__ bbar) {
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= nc) return;
  double d = dM[i], s = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double hb = HbyAbar[3 * (size_t)i + c];
    double h = hb / d;
    Hbar[3 * (size_t)i + c] = h;
    bbar[3 * (size_t)i + c] += h;
    s += hb * HbyA[3 * (size_t)i + c];
  }
  dbar[i] -= s / d;
}

// H = b - offdiag(M) Uin:  valbar(i,j) -= Hbar_i.Uin_j ;  Ubar = -offdiag(M)^T Hbar  (written)
// also used for the predictor with xbar = mu: valbar -= mu_i.U*_j (then Ubar unused)
__global__ __launch_bounds__(BLOCK) void k_adj_offdiag(int nc, const int32_t* __restrict__ slice_start, int uw,
                                                       const int32_t* __restrict__ col, const double* __restrict__ valT,
                                                       const double* __restrict__ ybar, const double* __restrict__ x,
                                                       double* __restrict__ valbar, double* __restrict__ Ubar) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= nc) return;
  SlotRange R = slots_of(slice_start, uw, i);
  double yi[3] = {ybar[3 * (size_t)i], ybar[3 * (size_t)i + 1], ybar[3 * (size_t)i + 2]};
  double u[3] = {0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k = 0; k < R.width; ++k) {
    int at = R.base + k * SLICE;
    int j = col[at];
    const double* xj = x + 3 * (size_t)j;
    const double* yj = ybar + 3 * (size_t)j;
    valbar[at] -= yi[0] * xj[0] + yi[1] * xj[1] + yi[2] * xj[2];
    double a = valT[at];
    u[0] -= a * yj[0];
    u[1] -= a * yj[1];
    u[2] -= a * yj[2];
  }
  if (Ubar)
#pragma unroll
    for (int c = 0; c < 3; ++c) Ubar[3 * (size_t)i + c] = u[c];
}

// predictor U* = M^-1 (b - V grad p): dbar -= mu.U*, bbar += mu, gbar = -V mu
__global__ __launch_bounds__(BLOCK) void k_adj_pred(int nc, const double* __restrict__ mu, const double* __restrict__ Us,
                                                    const double* __restrict__ V, double* __restrict__ dbar,
                                                    double* __restrict__ bbar, double* __restrict__ gbar) {
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= nc) return;
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double m = mu[3 * (size_t)i + c];
    s += m * Us[3 * (size_t)i + c];
    bbar[3 * (size_t)i + c] += m;
    gbar[3 * (size_t)i + c] = -V[i] * m;
  }
  dbar[i] -= s;
}

// rAU = V / d:  dbar -= rAUbar rAU / d
__global__ __launch_bounds__(BLOCK) void k_adj_rau(int nc, const double* __restrict__ rAUbar, const double* __restrict__ rAU,
                                                   const double* __restrict__ dM, double* __restrict__ dbar) {
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= nc) return;
  dbar[i] -= rAUbar[i] * rAU[i] / dM[i];
}

// b = V/dt U^n + fixed-U boundary terms + nu sum sigma k.interp(grad U^n) + deferred correction:
// Ubar^n = V/dt bbar (written), gUbar_i = nu sum_slots wself sigma (bbar_i - bbar_j) (x) k; the
// deferred correction t_f = F_f Delta_f(U^n, grad U^n) (b_O -= t, b_N += t) adds, with
// Deltabar = sF (bbar_i - bbar_j) seen from cell i (sF = -F owner side, +F neighbour side), the
// cell's own partial derivatives of Delta (upwind branch frozen)
// With a time scheme theta < 1, b also holds -(1 - theta) A U^n (A: the upwind convection and orthogonal
// diffusion coefficients of the lagged flux), whose transpose adds -(1 - theta) (A^T bbar)_i.
template <int CONV>
__global__ __launch_bounds__(BLOCK) void k_adj_bsrc(MeshView<double> m, const double* __restrict__ nu_cell, double dt,
                                                    double theta, const double* __restrict__ bbar,
                                                    const double* __restrict__ flux, const double4* __restrict__ rO,
                                                    const double4* __restrict__ rN, double* __restrict__ Ubar0,
                                                    double* __restrict__ gUbar) {
  const int base = xcd_tile(blockIdx.x, gridDim.x) * BLOCK;
  const int i = base + threadIdx.x;
  __shared__ double lds[9 * BLOCK];
  double uo[3], go[9];
  if (i < m.nc) {
  SlotRange R = slots_of(m, i);
  double nu = nu_cell[i];
  const double* bi = bbar + 3 * (size_t)i;
  double gu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double ub[3] = {0, 0, 0};
  const double ex = 1.0 - theta;  // explicit share of the matrix part
#pragma unroll 4
  for (int k = 0; k < R.width; ++k) {
    int at = R.base + k * SLICE;
    int sf = m.slot_face[at];
    if (sf == SLOT_PAD) continue;
    if (sf >= m.nfi) {
      if (ex != 0.0) {
        int bf = sf - m.nfi;
        int8_t code = m.bcode[DIFVM_BC_U * m.nfb + bf];
        double a = code == BC_FIXED ? nu * m.bgeom[bf].w : (code == BC_ZEROGRAD ? flux[m.nfi + bf] : 0.0);
#pragma unroll
        for (int c = 0; c < 3; ++c) ub[c] -= ex * a * bi[c];
      }
      continue;
    }
    bool nb = sf < 0;
    int f = nb ? -sf - 1 : sf;
    int j = m.slot_col[at];
    auto kd = m.geomK[f];
    double w = m.w[f];
    double wself = nb ? 1.0 - w : w;
    double sg = nb ? -nu : nu;
    const double* bj = bbar + 3 * (size_t)j;
    if (ex != 0.0) {
      double F = flux[f], nd = nu * kd.w;
      double Fp = F >= 0.0 ? F : 0.0, Fm = F < 0.0 ? F : 0.0;
      double ad = nb ? -Fm + nd : Fp + nd;  // self's diagonal part
      double aj = nb ? Fm - nd : -Fp - nd;  // the other row's coefficient of self (upper / lower)
#pragma unroll
      for (int c = 0; c < 3; ++c) ub[c] -= ex * (ad * bi[c] + aj * bj[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double t = wself * sg * (bi[c] - bj[c]);
      gu[c][0] += t * kd.x;
      gu[c][1] += t * kd.y;
      gu[c][2] += t * kd.z;
    }
    if constexpr (CONV != DIFVM_CONV_UPWIND) {
      double F = flux[f];
      bool up = dc_self_up(F, nb);
      double sF = nb ? F : -F;
      double4 rs = nb ? rN[f] : rO[f], ro = nb ? rO[f] : rN[f];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double Db = sF * (bi[c] - bj[c]);
        if constexpr (CONV == DIFVM_CONV_LINEAR) {
          ub[c] += Db * (wself - (up ? 1.0 : 0.0));
        } else if constexpr (CONV == DIFVM_CONV_SOU) {
          if (up) {
            gu[c][0] += Db * rs.x;
            gu[c][1] += Db * rs.y;
            gu[c][2] += Db * rs.z;
          }
        } else {
          ub[c] += up ? -0.25 * Db : 0.25 * Db;
          if (up) {
            gu[c][0] += 0.25 * Db * (rs.x - ro.x);
            gu[c][1] += 0.25 * Db * (rs.y - ro.y);
            gu[c][2] += 0.25 * Db * (rs.z - ro.z);
          }
        }
      }
    }
  }
  double vdt = m.V[i] / dt;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    uo[c] = vdt * bi[c] + ub[c];
#pragma unroll
    for (int e = 0; e < 3; ++e) go[3 * c + e] = gu[c][e];
  }
  }
  // rows staged through LDS so every store writes whole cache lines
  store_rows<3>(Ubar0, base, m.nc, uo, lds);
  store_rows<9>(gUbar, base, m.nc, go, lds);
}

// momentum coefficients (and the deferred correction t_f = F_f Delta_f, whose Delta is taken from
// U^n and its gradient) -> lagged flux (upwind branch frozen at the forward's choice)
// (theta: the stored coefficients carry theta; the explicit share 1 - theta of the matrix part acts on U^n)
template <int CONV>
__global__ __launch_bounds__(BLOCK) void k_adj_phi(MeshView<double> m, double theta, const int32_t* __restrict__ own_slot,
                                                   const int32_t* __restrict__ nbr_slot, const double* __restrict__ phi,
                                                   const double* __restrict__ valbar, const double* __restrict__ dbar,
                                                   const double* __restrict__ bbar, const double* __restrict__ Ub,
                                                   const double* __restrict__ Un, const double* __restrict__ gUn,
                                                   const double4* __restrict__ rO, const double4* __restrict__ rN,
                                                   double* __restrict__ phibar) {
  int f = blockIdx.x * BLOCK + threadIdx.x;
  if (f < m.nfi) {
    int O = m.own[f], N = m.nbr[f];
    double F = phi[f];
    double ub = valbar[own_slot[f]], lb = valbar[nbr_slot[f]];
    double v = theta * (F >= 0.0 ? dbar[O] - lb : ub - dbar[N]);
    if (theta != 1.0) {
      int Cc = F >= 0.0 ? O : N;  // upwind cell
#pragma unroll
      for (int c = 0; c < 3; ++c)
        v -= (1.0 - theta) * (bbar[3 * (size_t)O + c] - bbar[3 * (size_t)N + c]) * Un[3 * (size_t)Cc + c];
    }
    if constexpr (CONV != DIFVM_CONV_UPWIND) {
      bool up = dc_self_up(F, false);
      double4 ro_ = rO[f], rn_ = rN[f];
      double w = m.w[f];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double D = dc_delta<CONV>(up, w, Un[3 * (size_t)O + c], Un[3 * (size_t)N + c], gUn + 9 * (size_t)O + 3 * c,
                                  gUn + 9 * (size_t)N + 3 * c, ro_, rn_);
        v -= D * (bbar[3 * (size_t)O + c] - bbar[3 * (size_t)N + c]);
      }
    }
    phibar[f] = v;
  } else if (f < m.nfi + m.nfb) {
    int b = f - m.nfi;
    int8_t cu = m.bcode[DIFVM_BC_U * m.nfb + b];
    int O = m.bown[b];
    double v = 0.0;
    if (cu == BC_FIXED)
      v = -(bbar[3 * (size_t)O] * Ub[3 * (size_t)b] + bbar[3 * (size_t)O + 1] * Ub[3 * (size_t)b + 1] +
            bbar[3 * (size_t)O + 2] * Ub[3 * (size_t)b + 2]);
    else if (cu == BC_ZEROGRAD) {
      v = theta * dbar[O];
      if (theta != 1.0)
        v -= (1.0 - theta) * (bbar[3 * (size_t)O] * Un[3 * (size_t)O] + bbar[3 * (size_t)O + 1] * Un[3 * (size_t)O + 1] +
                              bbar[3 * (size_t)O + 2] * Un[3 * (size_t)O + 2]);
    }
    phibar[f] = v;
  }
}

// Fixed velocity boundary values U_b enter a step through the face flux of HbyA (phiH_b = U_b . S_b in
// every corrector), the momentum source (b_O += (nu delta_b - F_b) U_b) and the Gauss gradient of
// U^n (handled by k_gradT).  Both kernels add into Ubbar[nfb*3], one thread per boundary face.
__global__ __launch_bounds__(BLOCK) void k_adj_ub_flux(MeshView<double> m, const double* __restrict__ fHb,
                                                       double* __restrict__ Ubbar) {
  int b = blockIdx.x * BLOCK + threadIdx.x;
  if (b >= m.nfb || m.bcode[DIFVM_BC_U * m.nfb + b] != BC_FIXED) return;
  auto g = m.bgeom[b];
  double h = fHb[m.nfi + b];
  Ubbar[3 * (size_t)b] += h * g.x;
  Ubbar[3 * (size_t)b + 1] += h * g.y;
  Ubbar[3 * (size_t)b + 2] += h * g.z;
}

__global__ __launch_bounds__(BLOCK) void k_adj_ub_src(MeshView<double> m, const double* __restrict__ nu_cell,
                                                      const double* __restrict__ phi, const double* __restrict__ bbar,
                                                      double* __restrict__ Ubbar) {
  int b = blockIdx.x * BLOCK + threadIdx.x;
  if (b >= m.nfb || m.bcode[DIFVM_BC_U * m.nfb + b] != BC_FIXED) return;
  int O = m.bown[b];
  double a = nu_cell[O] * m.bgeom[b].w - phi[m.nfi + b];
#pragma unroll
  for (int c = 0; c < 3; ++c) Ubbar[3 * (size_t)b + c] += a * bbar[3 * (size_t)O + c];
}

// Windkessel: sum of boundary-pressure cotangents over each outlet (fixed order), and the outlet flow
// cotangent spread back to its faces
__global__ __launch_bounds__(BLOCK) void k_adj_wk_sum(const int32_t* __restrict__ wk_start, const int32_t* __restrict__ wk_faces,
                                                      const double* __restrict__ pbvbar, double* __restrict__ out) {
  int j = blockIdx.x;
  double v[1] = {0.0};
  for (int q = wk_start[j] + threadIdx.x; q < wk_start[j + 1]; q += BLOCK) v[0] += pbvbar[wk_faces[q]];
  __shared__ double lds[1][BLOCK / 64];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) out[j] = v[0];
}

__global__ __launch_bounds__(BLOCK) void k_adj_wk_spread(int nfi, const int32_t* __restrict__ wk_start,
                                                         const int32_t* __restrict__ wk_faces, const double* __restrict__ Qbar,
                                                         double* __restrict__ phibar) {
  int j = blockIdx.x;
  for (int q = wk_start[j] + threadIdx.x; q < wk_start[j + 1]; q += BLOCK) phibar[nfi + wk_faces[q]] += Qbar[j];
}

// Windkessel reverse of one step, one thread per outlet.  Forward: E = exp(-dt/(Rd C)),
// p_c' = p_c E + Rd Q (1 - E), p_o = p_c' + Rp Q.  In: pobar_Qbar[j] = cotangent of p_o (summed over
// the outlet's faces), pcbar[j] = cotangent of p_c'.  Out: pcbar[j] = cotangent of p_c, wkbar[3j..]
// += cotangents of (Rp, C, Rd), pobar_Qbar[j] = cotangent of Q.
__global__ void k_adj_wk_step(int nwk, double dt, const double* __restrict__ wk, const double* __restrict__ wk_out,
                              const double* __restrict__ pc_in, double* __restrict__ pobar_Qbar,
                              double* __restrict__ pcbar, double* __restrict__ wkbar) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nwk) return;
  double Rp = wk[3 * j], Cc = wk[3 * j + 1], Rd = wk[3 * j + 2];
  double Q = wk_out[2 * j], pc0 = pc_in[j];
  double E = exp(-dt / (Rd * Cc));
  double pob = pobar_Qbar[j];
  double pc1bar = pcbar[j] + pob;  // p_o = p_c' + Rp Q
  double Qb = pob * Rp + pc1bar * Rd * (1.0 - E);
  double Eb = pc1bar * (pc0 - Rd * Q);
  wkbar[3 * j] += pob * Q;
  wkbar[3 * j + 1] += Eb * E * dt / (Rd * Cc * Cc);
  wkbar[3 * j + 2] += pc1bar * Q * (1.0 - E) + Eb * E * dt / (Rd * Rd * Cc);
  pcbar[j] = pc1bar * E;
  pobar_Qbar[j] = Qb;
}

// clears n doubles (a kernel, not a memset, so the reverse sweep can be captured)
__global__ void k_zero(size_t n, double* __restrict__ a) {
  size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

__global__ void k_axpy(size_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

}  // namespace difvm

// =============================================================================================
// tape: checkpoints every K steps; a segment is recomputed once with full step records
// =============================================================================================
struct difvm_tape {
  difvm_piso* piso = nullptr;
  int nsteps = 0, every = 1, nseg = 0, recorded = 0, reversed = 0;
  int rec_seg = -1;  // the segment whose step records `rec` holds (-1: none)
  std::vector<double*> ckU, ckp, ckphi;   // per checkpoint, internal order
  std::vector<std::vector<double>> ckpc;  // host copies of the capacitor pressures
  std::vector<difvm::StepRecord> rec;     // one per step of a segment
  // reverse-sweep work
  double *Ubar = nullptr, *pbar = nullptr, *phibar = nullptr, *phibar_in = nullptr, *pbvbar = nullptr;
  double *HbyAbar = nullptr, *rAUbar = nullptr, *gbar = nullptr, *gUbar = nullptr, *Hbar = nullptr, *bbar = nullptr;
  double *dbar = nullptr, *valbar = nullptr, *valT = nullptr, *fHb = nullptr, *faF = nullptr, *fnc = nullptr;
  double *g = nullptr, *tmp = nullptr, *lam = nullptr, *mu = nullptr, *Ubar0 = nullptr, *wkbar = nullptr;
  double* gUn = nullptr;  // grad U^n of the step being reversed (deferred-correction schemes)
  double* Ubbar = nullptr;  // cotangent of the fixed velocity boundary values, summed over the window [nfb*3]
  double *endU = nullptr, *endp = nullptr, *endphi = nullptr;
  std::vector<double> endpc;
  double *pcbar = nullptr, *wkacc = nullptr;  // device: capacitor and parameter cotangents [n_wk], [3 n_wk]
  std::vector<void*> allocs;
  // Graph mode of the reverse sweep: each full checkpoint segment is recomputed by one replayed graph
  // (graph 0: `every` forward steps with their records) and reversed by another (graph 1: `every`
  // reverse steps), with a budget per solve kind as in the forward graph mode.
  struct Graph {
    bool on = false;
    int extra = 16, margin = 2;
    hipStream_t cap = nullptr;
    hipGraph_t g[2] = {nullptr, nullptr};
    hipGraphExec_t x[2] = {nullptr, nullptr};
    int bud_u[2] = {0, 0}, bud_p[2] = {0, 0};
    double tol = -1.0;                 // adjoint tolerance the reverse graph was captured with
    void* state_dev = nullptr;         // solver states of one segment: [graph][step][momentum, correctors]
    void* state_host = nullptr;
    size_t bytes_u = 0, bytes_p = 0, per_step = 0;
    double* backup = nullptr;          // cotangents entering a reverse segment
    long long replays = 0, redos = 0, captures = 0;
  } gr;
};

namespace difvm {

static double* tape_alloc(difvm_tape* T, size_t n) {
  double* a = dalloc<double>(ctx_of(T->piso->mesh), n);
  T->allocs.push_back(a);
  DIFVM_HIP(hipMemsetAsync(a, 0, sizeof(double) * (n ? n : 1), stream_of(T->piso->mesh)));
  return a;
}

static void zero(double* a, size_t n, hipStream_t s) {
  if (!n) return;
  k_zero<<<(unsigned)((n + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(n, a);
  DIFVM_HIP(hipGetLastError());
}

static void host_pc(difvm_piso* P, std::vector<double>& out) {
  int nwk = P->mesh->d.n_wk;
  out.assign(nwk, 0.0);
  if (nwk) {
    DIFVM_HIP(hipMemcpyAsync(out.data(), P->pc, sizeof(double) * nwk, hipMemcpyDeviceToHost, stream_of(P->mesh)));
    DIFVM_HIP(hipStreamSynchronize(stream_of(P->mesh)));
  }
}

static void set_pc(difvm_piso* P, const std::vector<double>& v) {
  if (!v.empty()) {
    DIFVM_HIP(hipMemcpyAsync(P->pc, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice, stream_of(P->mesh)));
    DIFVM_HIP(hipStreamSynchronize(stream_of(P->mesh)));
  }
}

void tape_create(difvm_piso* P, int nsteps, int every, difvm_tape** out) {
  DIFVM_CHECK(nsteps >= 1 && every >= 1, DIFVM_ERR_INVALID_ARG, "nsteps and ckpt_every must be >= 1");
  difvm_tape* T = new difvm_tape();
  try {
    T->piso = P;
    T->nsteps = nsteps;
    T->every = std::min(every, nsteps);
    T->nseg = (nsteps + T->every - 1) / T->every;
    const DMesh& d = P->mesh->d;
    size_t nc = d.nc, nf = (size_t)d.nfi + d.nfb;
    int nwk = std::max(1, d.n_wk);
    for (int k = 0; k < T->nseg; ++k) {
      T->ckU.push_back(tape_alloc(T, 3 * nc));
      T->ckp.push_back(tape_alloc(T, nc));
      T->ckphi.push_back(tape_alloc(T, nf));
    }
    T->ckpc.resize(T->nseg);
    T->rec.resize(T->every);
    int ncorr = P->prm.n_corr;
    for (auto& r : T->rec) {
      r.phi_in = tape_alloc(T, nf);
      r.pbv = tape_alloc(T, d.nfb);
      r.dM = tape_alloc(T, nc);
      r.valM = tape_alloc(T, d.nslot);
      r.Ustar = tape_alloc(T, 3 * nc);
      r.rAU = tape_alloc(T, nc);
      r.wk_out = tape_alloc(T, 2 * nwk);
      r.pc_in = tape_alloc(T, nwk);
      if (P->prm.conv != DIFVM_CONV_UPWIND || P->prm.time != DIFVM_TIME_BACKWARD_EULER) r.Un = tape_alloc(T, 3 * nc);
      for (int c = 0; c < ncorr; ++c) {
        r.Uin[c] = tape_alloc(T, 3 * nc);
        r.pold[c] = tape_alloc(T, nc);
        r.pnew[c] = tape_alloc(T, nc);
        r.HbyA[c] = tape_alloc(T, 3 * nc);
        r.gpo[c] = tape_alloc(T, 3 * nc);
        r.gpn[c] = tape_alloc(T, 3 * nc);
      }
    }
    T->Ubar = tape_alloc(T, 3 * nc); T->pbar = tape_alloc(T, nc); T->phibar = tape_alloc(T, nf);
    T->phibar_in = tape_alloc(T, nf); T->pbvbar = tape_alloc(T, d.nfb); T->HbyAbar = tape_alloc(T, 3 * nc);
    T->rAUbar = tape_alloc(T, nc); T->gbar = tape_alloc(T, 3 * nc); T->gUbar = tape_alloc(T, 9 * nc);
    T->Hbar = tape_alloc(T, 3 * nc); T->bbar = tape_alloc(T, 3 * nc); T->dbar = tape_alloc(T, nc);
    T->valbar = tape_alloc(T, d.nslot); T->valT = tape_alloc(T, d.nslot); T->fHb = tape_alloc(T, nf);
    T->faF = tape_alloc(T, nf); T->fnc = tape_alloc(T, std::max<size_t>(1, d.nfi)); T->g = tape_alloc(T, nf);
    T->tmp = tape_alloc(T, 3 * nc); T->mu = tape_alloc(T, 3 * nc);
    T->lam = tape_alloc(T, (size_t)P->prm.n_corr * nc);  // one pressure multiplier per corrector
    T->Ubar0 = tape_alloc(T, 3 * nc); T->wkbar = tape_alloc(T, nwk); T->Ubbar = tape_alloc(T, 3 * (size_t)d.nfb);
    if (P->prm.conv != DIFVM_CONV_UPWIND) T->gUn = tape_alloc(T, 9 * nc);
    T->endU = tape_alloc(T, 3 * nc); T->endp = tape_alloc(T, nc); T->endphi = tape_alloc(T, nf);
    T->pcbar = tape_alloc(T, nwk); T->wkacc = tape_alloc(T, 3 * (size_t)nwk);
  } catch (...) {
    for (void* a : T->allocs) dfree(ctx_of(P->mesh), a);
    delete T;
    throw;
  }
  P->refs++;
  *out = T;
}

static void tape_graph_drop(difvm_tape* T) {
  for (int k = 0; k < 2; ++k) {
    if (T->gr.x[k]) (void)hipGraphExecDestroy(T->gr.x[k]);
    if (T->gr.g[k]) (void)hipGraphDestroy(T->gr.g[k]);
    T->gr.x[k] = nullptr;
    T->gr.g[k] = nullptr;
  }
}

void tape_destroy(difvm_tape* T) {
  if (!T) return;
  (void)hipStreamSynchronize(stream_of(T->piso->mesh));
  tape_graph_drop(T);
  if (T->gr.cap) (void)hipStreamDestroy(T->gr.cap);
  if (T->gr.state_host) (void)hipHostFree(T->gr.state_host);
  for (void* a : T->allocs) dfree(ctx_of(T->piso->mesh), a);
  difvm_piso* P = T->piso;
  delete T;
  piso_release(P);
}

static void save_state(difvm_piso* P, double* U, double* p, double* phi, std::vector<double>& pc) {
  const DMesh& d = P->mesh->d;
  hipStream_t s = stream_of(P->mesh);
  dcopy(U, P->U, 3 * (size_t)d.nc, s);
  dcopy(p, P->p, d.nc, s);
  dcopy(phi, P->phi, (size_t)d.nfi + d.nfb, s);
  host_pc(P, pc);
}

static void load_state(difvm_piso* P, const double* U, const double* p, const double* phi, const std::vector<double>& pc) {
  const DMesh& d = P->mesh->d;
  hipStream_t s = stream_of(P->mesh);
  dcopy(P->U, U, 3 * (size_t)d.nc, s);
  dcopy(P->p, p, d.nc, s);
  dcopy(P->phi, phi, (size_t)d.nfi + d.nfb, s);
  set_pc(P, pc);
}

// The last segment's steps keep their records, so the reverse sweep that follows need not recompute
// that segment from its checkpoint (the recomputation would reproduce the same bits).
int forward_record(difvm_piso* P, difvm_tape* T, difvm_step_stats* stats) {
  int worst = 0;
  const int last = T->nseg - 1, last_s0 = last * T->every;
  T->rec_seg = -1;
  for (int n = 0; n < T->nsteps; ++n) {
    if (n % T->every == 0) {
      int k = n / T->every;
      save_state(P, T->ckU[k], T->ckp[k], T->ckphi[k], T->ckpc[k]);
    }
    difvm_step_stats st{};
    piso_advance(P, &st, n >= last_s0 ? &T->rec[n - last_s0] : nullptr);
    worst = std::max(worst, st.status);
    if (stats) stats[n] = st;
  }
  save_state(P, T->endU, T->endp, T->endphi, T->endpc);
  T->recorded = 1;
  T->rec_seg = last;
  return worst;
}

// Reverse of one recorded step.  On entry T->Ubar, T->pbar, T->phibar_in (flux cotangent) and
// T->pcbar hold the cotangents of the step's outputs; on exit they hold those of its inputs, and the
// Windkessel parameter cotangents are added to T->wkacc.  With q (capture), every solve queues its
// budget and leaves its state at q's state_out (nothing is read back, counts untouched); otherwise
// counts (may be NULL) receive the iterations of the momentum solve (largest component) and of each
// corrector's pressure solve.
static int reverse_step(difvm_piso* P, difvm_tape* T, const StepRecord& R, const double* phi_n, double adj_tol,
                        const StepQueue* q, int* counts) {
  difvm_mesh* m = P->mesh;
  const DMesh& d = m->d;
  hipStream_t s = stream_of(m);
  MeshView<double> mv = view<double>(d);
  const difvm_piso_params& prm = P->prm;
  int Gc = grid_for(d.nc), Gf = grid_for(d.nfi + d.nfb);
  size_t nc = d.nc, nf = (size_t)d.nfi + d.nfb;
  int worst = 0;
  int maxit_p = std::max(prm.maxit_p, 20000), maxit_u = std::max(prm.maxit_u, 5000);

  zero(T->rAUbar, nc, s);
  zero(T->bbar, 3 * nc, s);
  zero(T->dbar, nc, s);
  zero(T->valbar, d.nslot, s);
  zero(T->pbvbar, d.nfb, s);
  // momentum transpose (and the pressure matrix, which depends only on rAU)
  if (d.nfi) k_swap_slots<<<grid_for(d.nfi), BLOCK, 0, s>>>(d.nfi, d.face_slot_own, d.face_slot_nbr, R.valM, T->valT);
  piso_pressure_matrix(P, R.HbyA[0], R.rAU, R.gpo[0], R.pbv);
  for (int c = prm.n_corr - 1; c >= 0; --c) {
    // U = HbyA - rAU grad(p_new)
    k_adj_ucorr<<<Gc, BLOCK, 0, s>>>(d.nc, T->Ubar, R.gpn[c], R.rAU, T->HbyAbar, T->rAUbar, T->gbar);
    k_gradT<1><<<Gc, BLOCK, 0, s>>>(mv, DIFVM_BC_P, T->gbar, T->pbar, T->pbvbar);
    // flux output of the last corrector
    k_adj_flux<<<Gf, BLOCK, 0, s>>>(mv, c == prm.n_corr - 1, T->phibar_in, R.rAU, R.pnew[c], R.pbv, T->fHb, T->faF,
                                    T->fnc, T->g, T->pbvbar);
    op_div(m, DIFVM_F64, DIFVM_SCHEME_ONE, 1, DIFVM_BC_P, T->g, nullptr, nullptr, T->tmp);
    k_axpy<<<Gc, BLOCK, 0, s>>>(nc, 1.0, T->tmp, T->pbar);
    // pressure solve: lambda = K^-1 pbar (K symmetric), started from this corrector's lambda of the
    // step reversed before (the later time step: the multipliers change little from step to step, so
    // the solve needs far fewer iterations than from zero; the sweep's first step starts from zero)
    double* lam = T->lam + (size_t)c * nc;
    SolveResult rp = pcg(m, SellMatrix{P->dK, P->valK}, T->pbar, lam, adj_tol, maxit_p, q ? &q->p[c] : nullptr,
                         P->amg, &P->hint_adj_p[c]);
    worst = std::max(worst, rp.status);
    if (counts && !q) counts[1 + c] = rp.iters[0];
    k_adj_psolve<<<Gf, BLOCK, 0, s>>>(mv, lam, R.pnew[c], R.rAU, R.pbv, P->is_ref, prm.p_ref_value, T->fHb, T->faF,
                                      T->fnc, T->pbvbar);
    k_adj_corr_cells<<<Gc, BLOCK, 0, s>>>(mv, T->fHb, T->faF, T->fnc, R.rAU, R.gpo[c], T->rAUbar, T->HbyAbar, T->gbar);
    if (d.nfb) k_adj_ub_flux<<<grid_for(d.nfb), BLOCK, 0, s>>>(mv, T->fHb, T->Ubbar);
    // pressure entering the corrector: only through grad(p_old)
    zero(T->pbar, nc, s);
    k_gradT<1><<<Gc, BLOCK, 0, s>>>(mv, DIFVM_BC_P, T->gbar, T->pbar, T->pbvbar);
    // HbyA = (b - offdiag U_in) / d
    k_adj_hbya<<<Gc, BLOCK, 0, s>>>(d.nc, T->HbyAbar, R.HbyA[c], R.dM, T->Hbar, T->dbar, T->bbar);
    k_adj_offdiag<<<Gc, BLOCK, 0, s>>>(d.nc, d.slice_start, d.uw, d.slot_col, T->valT, T->Hbar, R.Uin[c], T->valbar, T->Ubar);
    DIFVM_HIP(hipGetLastError());
  }
  // predictor: U* = M^-1 (b - V grad p^n);  mu = M^-T Ubar
  zero(T->mu, 3 * nc, s);
  SolveResult ru = bicgstab(m, 3, SellMatrix{R.dM, T->valT}, T->Ubar, T->mu, adj_tol, maxit_u, q ? &q->u : nullptr,
                            &P->hint_adj_u);
  worst = std::max(worst, ru.status);
  if (counts && !q) counts[0] = std::max(ru.iters[0], std::max(ru.iters[1], ru.iters[2]));
  k_adj_offdiag<<<Gc, BLOCK, 0, s>>>(d.nc, d.slice_start, d.uw, d.slot_col, T->valT, T->mu, R.Ustar, T->valbar, nullptr);
  k_adj_pred<<<Gc, BLOCK, 0, s>>>(d.nc, T->mu, R.Ustar, d.V, T->dbar, T->bbar, T->gbar);
  k_gradT<1><<<Gc, BLOCK, 0, s>>>(mv, DIFVM_BC_P, T->gbar, T->pbar, T->pbvbar);
  k_adj_rau<<<Gc, BLOCK, 0, s>>>(d.nc, T->rAUbar, R.rAU, R.dM, T->dbar);
  // momentum source and coefficients
  if (prm.conv != DIFVM_CONV_UPWIND) op_grad(m, DIFVM_F64, 3, DIFVM_BC_U, R.Un, P->Ub, T->gUn);
  const double theta = time_theta(prm.time);
  switch (prm.conv) {
#define DIFVM_ADJ_SRC(CV)                                                                                            \
  case CV:                                                                                                            \
    k_adj_bsrc<CV><<<Gc, BLOCK, 0, s>>>(mv, P->nu_cell, prm.dt, theta, T->bbar, phi_n, d.face_rO, d.face_rN,          \
                                        T->Ubar0, T->gUbar);                                                          \
    k_gradT<3><<<Gc, BLOCK, 0, s>>>(mv, DIFVM_BC_U, T->gUbar, T->Ubar0, T->Ubbar);                                     \
    k_adj_phi<CV><<<Gf, BLOCK, 0, s>>>(mv, theta, d.face_slot_own, d.face_slot_nbr, phi_n, T->valbar, T->dbar,        \
                                       T->bbar, P->Ub, R.Un, T->gUn, d.face_rO, d.face_rN, T->phibar);                \
    break;
    DIFVM_ADJ_SRC(DIFVM_CONV_UPWIND)
    DIFVM_ADJ_SRC(DIFVM_CONV_LINEAR)
    DIFVM_ADJ_SRC(DIFVM_CONV_SOU)
    DIFVM_ADJ_SRC(DIFVM_CONV_QUICK)
#undef DIFVM_ADJ_SRC
  }
  if (d.nfb) k_adj_ub_src<<<grid_for(d.nfb), BLOCK, 0, s>>>(mv, P->nu_cell, phi_n, T->bbar, T->Ubbar);
  DIFVM_HIP(hipGetLastError());
  // Windkessel (pbv = p_o on each outlet): one thread per outlet, on the device
  int nwk = d.n_wk;
  if (nwk) {
    k_adj_wk_sum<<<nwk, BLOCK, 0, s>>>(d.wk_start, d.wk_faces, T->pbvbar, T->wkbar);
    k_adj_wk_step<<<1, 64, 0, s>>>(nwk, prm.dt, P->wk, R.wk_out, R.pc_in, T->wkbar, T->pcbar, T->wkacc);
    k_adj_wk_spread<<<nwk, BLOCK, 0, s>>>(d.nfi, d.wk_start, d.wk_faces, T->wkbar, T->phibar);
    DIFVM_HIP(hipGetLastError());
  }
  // outputs become the next (earlier) step's incoming cotangents
  dcopy(T->Ubar, T->Ubar0, 3 * nc, s);
  dcopy(T->phibar_in, T->phibar, nf, s);
  return worst;
}

// ---- graph mode of the reverse sweep ----------------------------------------------------------
// the words backup_cot saves, in its order
static size_t seg_words(const DMesh& d, int n_corr) {
  return 4 * (size_t)d.nc + d.nfi + d.nfb + 3 * (size_t)d.nfb + 4 * (size_t)d.n_wk + (size_t)n_corr * d.nc;
}

// save (to backup) or restore the state entering a reverse segment: the cotangents Ubar, pbar,
// phibar_in, Ubbar (summed over the window) and the Windkessel cotangents, and the pressure
// multipliers the segment's first solves start from
static void backup_cot(difvm_tape* T, bool save, hipStream_t s) {
  const DMesh& d = T->piso->mesh->d;
  size_t nc = d.nc, nf = (size_t)d.nfi + d.nfb;
  int nwk = d.n_wk;
  double* b = T->gr.backup;
  double* a[7] = {T->Ubar, T->pbar, T->phibar_in, T->Ubbar, T->pcbar, T->wkacc, T->lam};
  size_t len[7] = {3 * nc, nc, nf, 3 * (size_t)d.nfb, (size_t)nwk, 3 * (size_t)nwk,
                   (size_t)T->piso->prm.n_corr * nc};
  for (int k = 0; k < 7; ++k) {
    if (save) dcopy(b, a[k], len[k], s);
    else dcopy(a[k], b, len[k], s);
    b += len[k];
  }
}

static char* seg_state(difvm_tape* T, int graph, int step) {
  return static_cast<char*>(T->gr.state_dev) + ((size_t)graph * T->every + step) * T->gr.per_step;
}

// recompute (graph 0) or reverse (graph 1) one full segment, queue-only, captured on the private stream
static void tape_capture(difvm_tape* T, int graph, double adj_tol) {
  difvm_piso* P = T->piso;
  difvm_mesh* m = P->mesh;
  Ctx& c = ctx_of(m);
  auto& G = T->gr;
  hipStream_t orig = c.stream;
  c.stream = G.cap;
  c.capturing = true;
  DIFVM_HIP(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
  try {
    auto queue_of = [&](int step) {
      StepQueue qu;
      char* st = seg_state(T, graph, step);
      qu.u = QueueOnly{G.bud_u[graph], st};
      for (int k = 0; k < P->prm.n_corr; ++k) qu.p[k] = QueueOnly{G.bud_p[graph], st + G.bytes_u + k * G.bytes_p};
      return qu;
    };
    if (graph == 0) {
      for (int n = 0; n < T->every; ++n) {
        StepQueue qu = queue_of(n);
        piso_advance_q(P, nullptr, &T->rec[n], &qu);
      }
    } else {
      backup_cot(T, true, G.cap);
      for (int n = T->every - 1; n >= 0; --n) {
        StepQueue qu = queue_of(n);
        reverse_step(P, T, T->rec[n], T->rec[n].phi_in, adj_tol, &qu, nullptr);
      }
    }
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(G.cap, &g);
    if (g) (void)hipGraphDestroy(g);
    c.stream = orig;
    c.capturing = false;
    throw;
  }
  hipError_t e = hipStreamEndCapture(G.cap, &G.g[graph]);
  c.stream = orig;
  c.capturing = false;
  DIFVM_HIP(e);
  DIFVM_HIP(hipGraphInstantiate(&G.x[graph], G.g[graph], nullptr, nullptr, 0));
  if (graph == 1) G.tol = adj_tol;
  G.captures++;
}

static void tape_drop_one(difvm_tape* T, int graph) {
  if (T->gr.x[graph]) (void)hipGraphExecDestroy(T->gr.x[graph]);
  if (T->gr.g[graph]) (void)hipGraphDestroy(T->gr.g[graph]);
  T->gr.x[graph] = nullptr;
  T->gr.g[graph] = nullptr;
}

// replays graph `graph` and reads its solver states: true when every solve stopped within its budget;
// the largest counts per kind go to cu / cp
static bool tape_replay(difvm_tape* T, int graph, int* cu, int* cp, int* worst) {
  difvm_piso* P = T->piso;
  difvm_mesh* m = P->mesh;
  hipStream_t s = stream_of(m);
  auto& G = T->gr;
  DIFVM_HIP(hipGraphLaunch(G.x[graph], s));
  size_t bytes = (size_t)T->every * G.per_step;
  DIFVM_HIP(hipMemcpyAsync(G.state_host, seg_state(T, graph, 0), bytes, hipMemcpyDeviceToHost, s));
  DIFVM_HIP(hipStreamSynchronize(s));
  bool ok = true;
  int w = 0;
  *cu = *cp = 0;
  for (int n = 0; n < T->every; ++n) {
    const char* hs = static_cast<const char*>(G.state_host) + (size_t)n * G.per_step;
    bool c1 = true;
    SolveResult ru = bicgstab_result(m, 3, hs, &c1);
    ok = ok && c1;
    *cu = std::max(*cu, std::max(ru.iters[0], std::max(ru.iters[1], ru.iters[2])));
    w = std::max(w, ru.status);
    for (int k = 0; k < P->prm.n_corr; ++k) {
      SolveResult rp = pcg_result(m, hs + G.bytes_u + k * G.bytes_p, &c1);
      ok = ok && c1;
      *cp = std::max(*cp, rp.iters[0]);
      w = std::max(w, rp.status);
    }
  }
  // a replay that ran out of budget is discarded (counted as a redo by the caller): its
  // (incomplete) solves' statuses do not count
  if (ok) {
    *worst = std::max(*worst, w);
    G.replays++;
  }
  return ok;
}

static void set_tape_budgets(difvm_tape* T, int graph, int cu, int cp, bool grow_only) {
  auto& G = T->gr;
  int bu = cu + G.margin + cu / 64, bp = cp + G.margin + cp / 64;
  G.bud_u[graph] = grow_only ? std::max(G.bud_u[graph], bu) : bu;
  G.bud_p[graph] = grow_only ? std::max(G.bud_p[graph], bp) : bp;
}

void tape_set_graph(difvm_tape* T, int enable, int extra) {
  DIFVM_CHECK(extra >= 0, DIFVM_ERR_INVALID_ARG, "extra_iters must be >= 0");
  difvm_piso* P = T->piso;
  auto& G = T->gr;
  tape_graph_drop(T);
  G.on = enable != 0;
  G.extra = extra;
  G.margin = std::min(2, extra);
  if (!G.on) return;
  difvm_mesh* m = P->mesh;
  if (!G.cap) DIFVM_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
  G.bytes_u = bicgstab_state_bytes(m);
  G.bytes_p = pcg_state_bytes(m);
  G.per_step = G.bytes_u + (size_t)P->prm.n_corr * G.bytes_p;
  if (!G.state_dev) {
    size_t bytes = 2 * (size_t)T->every * G.per_step;
    G.state_dev = tape_alloc(T, (bytes + 7) / 8);
    G.backup = tape_alloc(T, seg_words(m->d, P->prm.n_corr));
    DIFVM_HIP(hipHostMalloc(&G.state_host, (size_t)T->every * G.per_step, hipHostMallocDefault));
  }
}

// eager recompute of steps [s0, s1) from the loaded checkpoint; largest counts per kind
static int recompute_eager(difvm_tape* T, int s0, int s1, int* cu, int* cp) {
  difvm_piso* P = T->piso;
  int worst = 0;
  *cu = *cp = 0;
  for (int n = s0; n < s1; ++n) {
    difvm_step_stats st{};
    piso_advance(P, &st, &T->rec[n - s0]);
    worst = std::max(worst, st.status);
    *cu = std::max(*cu, std::max(st.it_u[0], std::max(st.it_u[1], st.it_u[2])));
    for (int k = 0; k < P->prm.n_corr; ++k) *cp = std::max(*cp, st.it_p[k]);
  }
  return worst;
}

static int reverse_eager(difvm_tape* T, int s0, int s1, double adj_tol, int* cu, int* cp) {
  difvm_piso* P = T->piso;
  int worst = 0;
  *cu = *cp = 0;
  for (int n = s1 - 1; n >= s0; --n) {
    int cnt[1 + StepRecord::MAXC] = {};
    worst = std::max(worst, reverse_step(P, T, T->rec[n - s0], T->rec[n - s0].phi_in, adj_tol, nullptr, cnt));
    *cu = std::max(*cu, cnt[0]);
    for (int k = 0; k < P->prm.n_corr; ++k) *cp = std::max(*cp, cnt[1 + k]);
  }
  return worst;
}

int adjoint(difvm_piso* P, difvm_tape* T, const double* gU, const double* gp, const double* gphi, const double* gpc_host,
            double adj_tol, double* gU0, double* gp0, double* gphi0, double* gpc0_host, double* gwk_host) {
  DIFVM_CHECK(T->recorded, DIFVM_ERR_INVALID_ARG, "tape has no forward record");
  difvm_mesh* m = P->mesh;
  const DMesh& d = m->d;
  hipStream_t s = stream_of(m);
  size_t nc = d.nc, nf = (size_t)d.nfi + d.nfb;
  int nwk = d.n_wk;
  // incoming cotangents (user -> internal order)
  zero(T->Ubar, 3 * nc, s);
  zero(T->pbar, nc, s);
  zero(T->phibar_in, nf, s);
  zero(T->Ubbar, 3 * (size_t)d.nfb, s);
  zero(T->wkacc, 3 * (size_t)nwk, s);
  zero(T->pcbar, nwk, s);
  zero(T->lam, (size_t)P->prm.n_corr * nc, s);  // the sweep's first pressure solves start from zero
  if (gU) permute(m, DIFVM_F64, 3, DIFVM_KIND_CELL, DIFVM_TO_INTERNAL, gU, T->Ubar);
  if (gp) permute(m, DIFVM_F64, 1, DIFVM_KIND_CELL, DIFVM_TO_INTERNAL, gp, T->pbar);
  if (gphi) permute(m, DIFVM_F64, 1, DIFVM_KIND_FACE_FLUX, DIFVM_TO_INTERNAL, gphi, T->phibar_in);
  if (gpc_host && nwk) {
    DIFVM_HIP(hipMemcpyAsync(T->pcbar, gpc_host, sizeof(double) * nwk, hipMemcpyHostToDevice, s));
    DIFVM_HIP(hipStreamSynchronize(s));
  }
  auto& G = T->gr;
  if (G.on && G.x[1] && G.tol != adj_tol) tape_drop_one(T, 1);  // the tolerance is baked into the graph
  int worst = 0;
  for (int seg = T->nseg - 1; seg >= 0; --seg) {
    int s0 = seg * T->every, s1 = std::min(T->nsteps, s0 + T->every);
    bool graphed = G.on && s1 - s0 == T->every;
    int cu = 0, cp = 0;
    // recompute the segment from its checkpoint, keeping every step's intermediates, unless the
    // records still hold this segment (the window's last, right after the forward record)
    const bool have_records = seg == T->rec_seg;
    if (!have_records) {
      load_state(P, T->ckU[seg], T->ckp[seg], T->ckphi[seg], T->ckpc[seg]);
      T->rec_seg = seg;
    }
    if (have_records) {
      // nothing to recompute
    } else if (!graphed) {
      worst = std::max(worst, recompute_eager(T, s0, s1, &cu, &cp));
    } else if (!G.x[0]) {
      worst = std::max(worst, recompute_eager(T, s0, s1, &cu, &cp));
      set_tape_budgets(T, 0, cu, cp, false);
      tape_capture(T, 0, adj_tol);
    } else if (!tape_replay(T, 0, &cu, &cp, &worst)) {
      // some solve outran its budget: redo the segment eagerly, widen the margin, recapture
      load_state(P, T->ckU[seg], T->ckp[seg], T->ckphi[seg], T->ckpc[seg]);
      worst = std::max(worst, recompute_eager(T, s0, s1, &cu, &cp));
      G.margin = std::min(G.margin + 1, G.extra);
      set_tape_budgets(T, 0, cu, cp, true);
      tape_drop_one(T, 0);
      tape_capture(T, 0, adj_tol);
      G.redos++;
    } else if (G.bud_u[0] - (cu + G.margin + cu / 64) >= 2 || G.bud_p[0] - (cp + G.margin + cp / 64) >= 2) {
      set_tape_budgets(T, 0, cu, cp, false);  // counts fell: tighter budgets
      tape_drop_one(T, 0);
      tape_capture(T, 0, adj_tol);
    }
    // reverse sweep of the segment; the sweep's first segment runs eagerly: its first pressure
    // solves start from zero and take more iterations than a replay's budget allows for the others
    if (!graphed || seg == T->nseg - 1) {
      worst = std::max(worst, reverse_eager(T, s0, s1, adj_tol, &cu, &cp));
    } else if (!G.x[1]) {
      worst = std::max(worst, reverse_eager(T, s0, s1, adj_tol, &cu, &cp));
      set_tape_budgets(T, 1, cu, cp, false);
      tape_capture(T, 1, adj_tol);
    } else if (!tape_replay(T, 1, &cu, &cp, &worst)) {
      backup_cot(T, false, s);  // the graph's first nodes saved the segment's incoming cotangents
      worst = std::max(worst, reverse_eager(T, s0, s1, adj_tol, &cu, &cp));
      G.margin = std::min(G.margin + 1, G.extra);
      set_tape_budgets(T, 1, cu, cp, true);
      tape_drop_one(T, 1);
      tape_capture(T, 1, adj_tol);
      G.redos++;
    } else if (G.bud_u[1] - (cu + G.margin + cu / 64) >= 2 || G.bud_p[1] - (cp + G.margin + cp / 64) >= 2) {
      set_tape_budgets(T, 1, cu, cp, false);
      tape_drop_one(T, 1);
      tape_capture(T, 1, adj_tol);
    }
  }
  // outgoing cotangents (internal -> user order)
  if (gU0) permute(m, DIFVM_F64, 3, DIFVM_KIND_CELL, DIFVM_FROM_INTERNAL, T->Ubar, gU0);
  if (gp0) permute(m, DIFVM_F64, 1, DIFVM_KIND_CELL, DIFVM_FROM_INTERNAL, T->pbar, gp0);
  if (gphi0) permute(m, DIFVM_F64, 1, DIFVM_KIND_FACE_FLUX, DIFVM_FROM_INTERNAL, T->phibar_in, gphi0);
  if (nwk && (gpc0_host || gwk_host)) {
    std::vector<double> pcb(nwk), wkb(3 * nwk);
    DIFVM_HIP(hipMemcpyAsync(pcb.data(), T->pcbar, sizeof(double) * nwk, hipMemcpyDeviceToHost, s));
    DIFVM_HIP(hipMemcpyAsync(wkb.data(), T->wkacc, sizeof(double) * 3 * nwk, hipMemcpyDeviceToHost, s));
    DIFVM_HIP(hipStreamSynchronize(s));
    if (gpc0_host) for (int j = 0; j < nwk; ++j) gpc0_host[j] = pcb[j];
    if (gwk_host) for (int j = 0; j < 3 * nwk; ++j) gwk_host[j] = wkb[j];
  }
  T->reversed = 1;
  // leave the PISO at the end of the forward window
  load_state(P, T->endU, T->endp, T->endphi, T->endpc);
  DIFVM_HIP(hipStreamSynchronize(s));
  return worst;
}

}  // namespace difvm

using namespace difvm;

extern "C" {

difvm_status difvm_tape_create(difvm_piso* piso, int32_t nsteps, int32_t ckpt_every, difvm_tape** out) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(piso && out, DIFVM_ERR_INVALID_ARG, "piso and out must not be NULL");
  tape_create(piso, nsteps, ckpt_every, out);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_tape_destroy(difvm_tape* tape) {
  DIFVM_API_BEGIN
  tape_destroy(tape);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_forward_record(difvm_piso* piso, difvm_tape* tape, difvm_step_stats* stats_host) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(piso && tape && tape->piso == piso, DIFVM_ERR_INVALID_ARG, "tape does not belong to this PISO");
  int st = forward_record(piso, tape, stats_host);
  DIFVM_HIP(hipStreamSynchronize(stream_of(piso->mesh)));
  return st;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_tape_set_graph(difvm_tape* tape, int32_t enable, int32_t extra_iters) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(tape, DIFVM_ERR_INVALID_ARG, "tape is NULL");
  tape_set_graph(tape, enable, extra_iters);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_tape_graph_info(const difvm_tape* tape, int64_t* replays, int64_t* redos, int64_t* captures) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(tape, DIFVM_ERR_INVALID_ARG, "tape is NULL");
  if (replays) *replays = tape->gr.replays;
  if (redos) *redos = tape->gr.redos;
  if (captures) *captures = tape->gr.captures;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_tape_boundary_cotangent(const difvm_tape* tape, void* gU_b) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(tape && gU_b, DIFVM_ERR_INVALID_ARG, "tape and gU_b must not be NULL");
  DIFVM_CHECK(tape->reversed, DIFVM_ERR_INVALID_ARG, "difvm_piso_adjoint has not run on this tape");
  difvm_mesh* m = tape->piso->mesh;
  if (m->d.nfb) permute(m, DIFVM_F64, 3, DIFVM_KIND_BFACE, DIFVM_FROM_INTERNAL, tape->Ubbar, gU_b);
  DIFVM_HIP(hipStreamSynchronize(stream_of(m)));
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_adjoint(difvm_piso* piso, difvm_tape* tape, const void* gU_N, const void* gp_N, const void* gphi_N,
                                const double* gpc_N_host, double adj_tol, void* gU_0, void* gp_0, void* gphi_0,
                                double* gpc_0_host, double* gwk_host) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(piso && tape && tape->piso == piso, DIFVM_ERR_INVALID_ARG, "tape does not belong to this PISO");
  DIFVM_CHECK(adj_tol > 0, DIFVM_ERR_INVALID_ARG, "adj_tol must be > 0");
  return adjoint(piso, tape, (const double*)gU_N, (const double*)gp_N, (const double*)gphi_N, gpc_N_host, adj_tol,
                 (double*)gU_0, (double*)gp_0, (double*)gphi_0, gpc_0_host, gwk_host);
  DIFVM_API_END
  return DIFVM_OK;
}

}  // extern "C"
