// Oracle: a plain, slow, FP64 CPU face-loop implementation of the DiFVM hot path.
//
// TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's CPU-baseline leg may
// load this library.  It shares no source, header, table or helper with the GPU library
// (paper_2603_15920_amd/csrc); both consume only the seeded inputs from meshgen.
//
// Every operator is the plain finite-volume definition evaluated face by face, in face order, on the
// mesh exactly as given (user numbering):  for f: acc[owner f] += t_f; acc[neighbour f] -= t_f.
// The paper's graph form (Sec. "Graph-Based Reformulation") computes exactly these sums, only
// reorganised as per-edge messages and per-node aggregation, so the definition is the oracle.
//
// Notation (paper Sec. "Mesh data structure"): internal faces f in [0,Fi) with owner O_f, neighbour
// N_f; boundary faces b in [Fi, Fi+Fb) with owner O_b; S outward from the owner; d_f = C_N - C_O,
// d_b = Cf_b - C_O; the face vector is split as S = Delta + k with Delta = delta d along d (eq.
// nonortho_flux); delta_f follows the chosen correction scheme (over-relaxed by default, see
// face_split), delta_b likewise with d_b and k_b = 0.  Empty faces are skipped everywhere.
//
// Timing variant: built with -fopenmp (liboracle_omp.so) the double-precision LDU product, dot
// products and vector updates of the Krylov solvers, where a PISO step spends its time, run on all
// host threads: faces are split into one contiguous range per thread, each thread sums its faces
// into its own accumulator (covering the cells its range touches), and the accumulators are added
// in thread order; dot products add per-thread partial sums in thread order.  Results are
// deterministic for a given thread count and differ from the serial build only by rounding order.
// The parity tests use the serial build (liboracle.so).
//
// Parity pins live in tests/test_oracle_*.py.  Readings of points the paper leaves open are listed in
// the repository's design notes; the ones used here are restated at each function.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------------------------------------------------
// scalar types: double, and a forward-mode dual number carrying up to ND tangent directions
// ------------------------------------------------------------------------------------------------
constexpr int ND = 10;

struct Dual {
  double v;
  double d[ND];
  Dual() : v(0) { for (int k = 0; k < ND; ++k) d[k] = 0; }
  Dual(double x) : v(x) { for (int k = 0; k < ND; ++k) d[k] = 0; }
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) { Dual r(a.v / b.v); for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v); return r; }
inline Dual operator+(const Dual& a, double b) { Dual r = a; r.v += b; return r; }
inline Dual operator+(double a, const Dual& b) { return b + a; }
inline Dual operator-(const Dual& a, double b) { Dual r = a; r.v -= b; return r; }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b; return r; }
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { Dual r(a.v / b); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / b; return r; }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, const Dual& b) { a = a - b; return a; }
inline Dual exp(const Dual& a) { double e = std::exp(a.v); Dual r(e); for (int k = 0; k < ND; ++k) r.d[k] = e * a.d[k]; return r; }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::exp;

// ------------------------------------------------------------------------------------------------
// mesh as given by the caller (user numbering); mirrors om_mesh in oracle.py
// ------------------------------------------------------------------------------------------------
}  // namespace

extern "C" {
typedef struct {
  int32_t nc, nfi, nfb, npatch;
  const int32_t* owner;      // [nfi+nfb]
  const int32_t* nbr;        // [nfi]
  const double* Sf;          // [(nfi+nfb)*3]
  const double* Cf;          // [(nfi+nfb)*3]
  const double* C;           // [nc*3]
  const double* V;           // [nc]
  const double* w;           // [nfi]
  const int32_t* pstart;     // [npatch] first face of patch (absolute face index)
  const int32_t* psize;
  const int32_t* putype;     // 0 fixed, 1 zeroGradient, 2 empty
  const int32_t* pptype;     // 0 zeroGradient, 1 fixed, 2 Windkessel, 3 empty
  const int32_t* pwk;        // Windkessel id or -1
  int32_t nonorth;           // correction scheme: 0 over-relaxed, 1 minimum, 2 orthogonal, 3 none
} om_mesh;

typedef struct {
  double nu, dt;
  int32_t n_corr;
  double tol_p, tol_u;
  int32_t maxit_p, maxit_u;
  int32_t p_ref_cell;        // user numbering
  double p_ref_value;
  double tol_tangent;        // tolerance of the tangent (implicitly differentiated) solves
  int32_t conv;              // convection scheme: 0 upwind, 1 linear, 2 SOU, 3 QUICK (see deferred_correction)
  int32_t time;              // time scheme: 0 backward Euler, 1 forward Euler, 2 Crank-Nicolson (see time_theta)
} om_piso_params;
}

namespace {

enum { BC_FIXED = 0, BC_ZEROGRAD = 1, BC_EMPTY = 2 };
enum { TABLE_U = 0, TABLE_P = 1, TABLE_ALL_FIXED = 2, TABLE_ALL_ZEROGRAD = 3 };

// per-boundary-face BC code (fixed / zeroGradient / empty) for one of the tables
std::vector<int> bc_codes(const om_mesh& m, int table) {
  std::vector<int> code(m.nfb, BC_ZEROGRAD);
  for (int p = 0; p < m.npatch; ++p) {
    int c;
    bool empty = (m.putype[p] == 2) || (m.pptype[p] == 3);
    if (empty) c = BC_EMPTY;
    else if (table == TABLE_U) c = (m.putype[p] == 0) ? BC_FIXED : BC_ZEROGRAD;
    else if (table == TABLE_P) c = (m.pptype[p] == 1 || m.pptype[p] == 2) ? BC_FIXED : BC_ZEROGRAD;
    else if (table == TABLE_ALL_FIXED) c = BC_FIXED;
    else c = BC_ZEROGRAD;
    for (int b = m.pstart[p]; b < m.pstart[p] + m.psize[p]; ++b) code[b - m.nfi] = c;
  }
  return code;
}

inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

enum { NONORTH_OVERRELAXED = 0, NONORTH_MINIMUM = 1, NONORTH_ORTHOGONAL = 2, NONORTH_NONE = 3 };

// Split of the face vector S into Delta = delta d (along the cell-to-cell vector d) and k = S - Delta
// (Sec. "Diffusive flux discretization", eq. nonortho_flux), so that the orthogonal part of the
// face-normal gradient is delta (phi_N - phi_O).  The schemes differ only in |Delta|:
//   over-relaxed  |Delta| = |S| / |S^ . d^|   ->  delta = |S|^2 / (S.d)
//   minimum       Delta = (S . d^) d^         ->  delta = (S.d) / |d|^2
//   orthogonal    |Delta| = |S|               ->  delta = |S| / |d|
//   none          two-point stencil of eq. diff_ortho: delta = |S| / |d| and no correction (k = 0)
double face_split(int scheme, const double S[3], const double d[3], double k[3]) {
  double delta;
  if (scheme == NONORTH_MINIMUM) delta = dot3(S, d) / dot3(d, d);
  else if (scheme == NONORTH_ORTHOGONAL || scheme == NONORTH_NONE) delta = std::sqrt(dot3(S, S)) / std::sqrt(dot3(d, d));
  else delta = dot3(S, S) / dot3(S, d);
  for (int c = 0; c < 3; ++c) k[c] = (scheme == NONORTH_NONE) ? 0.0 : S[c] - delta * d[c];
  return delta;
}

// d_f, delta_f, k_f of an internal face
void face_geom(const om_mesh& m, int f, double d[3], double& delta, double k[3]) {
  const double* S = m.Sf + 3 * f;
  const double* CO = m.C + 3 * m.owner[f];
  const double* CN = m.C + 3 * m.nbr[f];
  for (int c = 0; c < 3; ++c) d[c] = CN[c] - CO[c];
  delta = face_split(m.nonorth, S, d, k);
}

// delta_b of a boundary face: the same scheme with d_b = Cf - C_O; the correction k_b is dropped
double bface_delta(const om_mesh& m, int f) {
  const double* S = m.Sf + 3 * f;
  const double* CO = m.C + 3 * m.owner[f];
  const double* Cf = m.Cf + 3 * f;
  double d[3] = {Cf[0] - CO[0], Cf[1] - CO[1], Cf[2] - CO[2]};
  double k[3];
  return face_split(m.nonorth, S, d, k);
}

// ------------------------------------------------------------------------------------------------
// operators (templated on the field scalar; geometry is double)
// ------------------------------------------------------------------------------------------------

// Linear face interpolation (Sec. "Spatial discretization": phi_f by linear interpolation):
// phi_f = w phi_O + (1-w) phi_N; boundary fixed -> given value, zeroGradient -> owner value.
template <class T>
void interp(const om_mesh& m, int ncomp, const std::vector<int>& code, const T* phi, const T* phib, T* out) {
  for (int f = 0; f < m.nfi; ++f) {
    double w = m.w[f];
    for (int c = 0; c < ncomp; ++c)
      out[f * ncomp + c] = w * phi[m.owner[f] * ncomp + c] + (1.0 - w) * phi[m.nbr[f] * ncomp + c];
  }
  for (int f = m.nfi; f < m.nfi + m.nfb; ++f) {
    int b = f - m.nfi;
    for (int c = 0; c < ncomp; ++c) {
      T v = T(0.0);
      if (code[b] == BC_FIXED) v = phib[b * ncomp + c];
      else if (code[b] == BC_ZEROGRAD) v = phi[m.owner[f] * ncomp + c];
      out[f * ncomp + c] = v;
    }
  }
}

// Gauss-Green gradient from face values (eq. gauss_green): G_i = (1/V_i) sum_f sigma phi_f S_f.
// Output layout [nc][ncomp][3].
template <class T>
void grad_from_faces(const om_mesh& m, int ncomp, const std::vector<int>& code, const T* phif, T* out) {
  std::fill(out, out + (size_t)m.nc * ncomp * 3, T(0.0));
  for (int f = 0; f < m.nfi; ++f) {
    const double* S = m.Sf + 3 * f;
    for (int c = 0; c < ncomp; ++c)
      for (int d = 0; d < 3; ++d) {
        T t = phif[f * ncomp + c] * S[d];
        out[(m.owner[f] * ncomp + c) * 3 + d] += t;
        out[(m.nbr[f] * ncomp + c) * 3 + d] -= t;
      }
  }
  for (int f = m.nfi; f < m.nfi + m.nfb; ++f) {
    if (code[f - m.nfi] == BC_EMPTY) continue;
    const double* S = m.Sf + 3 * f;
    for (int c = 0; c < ncomp; ++c)
      for (int d = 0; d < 3; ++d) out[(m.owner[f] * ncomp + c) * 3 + d] += phif[f * ncomp + c] * S[d];
  }
  for (int i = 0; i < m.nc; ++i)
    for (int j = 0; j < ncomp * 3; ++j) out[i * ncomp * 3 + j] = out[i * ncomp * 3 + j] / m.V[i];
}

template <class T>
void grad(const om_mesh& m, int ncomp, const std::vector<int>& code, const T* phi, const T* phib, T* out) {
  std::vector<T> phif((size_t)(m.nfi + m.nfb) * ncomp);
  interp(m, ncomp, code, phi, phib, phif.data());
  grad_from_faces(m, ncomp, code, phif.data(), out);
}

// Face-sum divergence (eqs. conv_face_flux, upwind, aggregate): D_i = sum_f sigma F_f psi_f, not
// divided by V.  scheme 0: psi_f = 1; 1: upwind (F >= 0 picks the owner, eq. upwind); 2: linear.
// Boundary psi from the BC: fixed -> given value, zeroGradient -> owner value.
template <class T>
void div(const om_mesh& m, int scheme, int ncomp, const std::vector<int>& code, const T* flux, const T* psi,
         const T* psib, T* out) {
  std::fill(out, out + (size_t)m.nc * ncomp, T(0.0));
  for (int f = 0; f < m.nfi; ++f) {
    int O = m.owner[f], N = m.nbr[f];
    for (int c = 0; c < ncomp; ++c) {
      T pf;
      if (scheme == 0) pf = T(1.0);
      else if (scheme == 1) pf = (val(flux[f]) >= 0.0) ? psi[O * ncomp + c] : psi[N * ncomp + c];
      else pf = m.w[f] * psi[O * ncomp + c] + (1.0 - m.w[f]) * psi[N * ncomp + c];
      T t = flux[f] * pf;
      out[O * ncomp + c] += t;
      out[N * ncomp + c] -= t;
    }
  }
  for (int f = m.nfi; f < m.nfi + m.nfb; ++f) {
    int b = f - m.nfi;
    if (code[b] == BC_EMPTY) continue;
    int O = m.owner[f];
    for (int c = 0; c < ncomp; ++c) {
      T pf;
      if (scheme == 0) pf = T(1.0);
      else pf = (code[b] == BC_FIXED) ? psib[b * ncomp + c] : psi[O * ncomp + c];
      out[O * ncomp + c] += flux[f] * pf;
    }
  }
}

enum { TIME_BACKWARD_EULER = 0, TIME_FORWARD_EULER = 1, TIME_CRANK_NICOLSON = 2 };

// The three time schemes of the scheme table as one theta-method on the matrix part of the transport
// operator A (convection of the lagged flux, orthogonal diffusion):
//   (V/dt)(u' - u^n) + theta A u' + (1 - theta) A u^n = explicit terms,
// theta = 1 backward Euler, 1/2 Crank-Nicolson, 0 forward Euler (then the matrix is V/dt alone and
// the predictor is the explicit update of eq. momentum_predictor).  One set of boundary values serves
// both halves; the caller gives them at t^n + theta dt (new level, mid-step, old level).  The explicit
// terms (non-orthogonal and deferred corrections, pressure gradient) are taken whole from the old
// level.
double time_theta(int scheme) {
  if (scheme == TIME_FORWARD_EULER) return 0.0;
  if (scheme == TIME_CRANK_NICOLSON) return 0.5;
  return 1.0;
}

enum { CONV_UPWIND = 0, CONV_LINEAR = 1, CONV_SOU = 2, CONV_QUICK = 3 };

// Deferred correction of the convection term (eq. deferred_correction): the upwind face value stays
// implicit and F_f (phi_f^HO - phi_f^U) is added explicitly, i.e. as a source on the right-hand side:
//   src_i += - sum_f sigma F_f (phi_f^HO - phi_f^U)          (internal faces; sigma = +1 owner, -1 neighbour)
// with C the upwind cell of f (the owner when F >= 0, eq. upwind), D the other cell, g the given
// cell gradients and phi_f^U = phi_C.  The higher-order face values:
//   linear  phi^HO = w phi_O + (1-w) phi_N                     (central, Table "schemes")
//   SOU     phi^HO = phi_C + g_C . (x_f - x_C)                 (eq. sou)
//   QUICK   phi^HO = phi_C + (phi_D - phi_C)/4 + g_C . (x_D - x_C)/4
// QUICK here is the classical upwind-biased quadratic 3/8 phi_D + 6/8 phi_C - 1/8 phi_U of a uniform
// line of cells with the far-upwind value, which an unstructured mesh does not have, replaced by
// phi_U = phi_D - 2 g_C . (x_D - x_C); on a uniform line with the central-difference gradient it is the
// classical stencil exactly.  Boundary faces carry no correction (their face value is the boundary
// value or the owner value for every scheme).  Upwind adds nothing.
template <class T>
void deferred_correction(const om_mesh& m, int conv, int ncomp, const T* F, const T* phi, const T* g, T* src) {
  if (conv == CONV_UPWIND) return;
  for (int f = 0; f < m.nfi; ++f) {
    int O = m.owner[f], N = m.nbr[f];
    bool own_up = val(F[f]) >= 0.0;
    int Cc = own_up ? O : N, Dc = own_up ? N : O;
    const double* xf = m.Cf + 3 * f;
    const double* xC = m.C + 3 * Cc;
    const double* xD = m.C + 3 * Dc;
    double w = m.w[f];
    for (int c = 0; c < ncomp; ++c) {
      const T* gC = g + ((size_t)Cc * ncomp + c) * 3;
      T pC = phi[(size_t)Cc * ncomp + c], pD = phi[(size_t)Dc * ncomp + c];
      T ho;
      if (conv == CONV_LINEAR) {
        ho = w * phi[(size_t)O * ncomp + c] + (1.0 - w) * phi[(size_t)N * ncomp + c];
      } else if (conv == CONV_SOU) {
        ho = pC + (gC[0] * (xf[0] - xC[0]) + gC[1] * (xf[1] - xC[1]) + gC[2] * (xf[2] - xC[2]));
      } else {
        T gd = gC[0] * (xD[0] - xC[0]) + gC[1] * (xD[1] - xC[1]) + gC[2] * (xD[2] - xC[2]);
        ho = pC + 0.25 * (pD - pC) + 0.25 * gd;
      }
      T t = F[f] * (ho - pC);
      src[(size_t)O * ncomp + c] -= t;
      src[(size_t)N * ncomp + c] += t;
    }
  }
}

// Laplacian with non-orthogonal correction (scheme of face_split) (eqs. diff_ortho, nonortho_flux):
// L_i = sum_f sigma G_f [delta_f (phi_N - phi_O) + k_f . (w g_O + (1-w) g_N)]
//       + sum_{b fixed} G_b delta_b (phi_b - phi_O);  zeroGradient boundaries add nothing.
// The face gradient in the correction is the linear interpolate of the given cell gradients.
template <class T>
void laplacian(const om_mesh& m, const std::vector<int>& code, const double* gamma, const T* phi, const T* g,
               const T* phib, T* out) {
  std::fill(out, out + m.nc, T(0.0));
  for (int f = 0; f < m.nfi; ++f) {
    int O = m.owner[f], N = m.nbr[f];
    double d[3], delta, k[3];
    face_geom(m, f, d, delta, k);
    double w = m.w[f];
    double G = gamma ? gamma[f] : 1.0;
    T corr = T(0.0);
    for (int c = 0; c < 3; ++c) corr += k[c] * (w * g[O * 3 + c] + (1.0 - w) * g[N * 3 + c]);
    T t = G * (delta * (phi[N] - phi[O]) + corr);
    out[O] += t;
    out[N] -= t;
  }
  for (int f = m.nfi; f < m.nfi + m.nfb; ++f) {
    int b = f - m.nfi;
    if (code[b] != BC_FIXED) continue;
    double G = gamma ? gamma[f] : 1.0;
    int O = m.owner[f];
    out[O] += G * bface_delta(m, f) * (phib[b] - phi[O]);
  }
}

// LDU matrix-vector product (eq. Ap_H's matrix in OpenFOAM-style LDU form):
// y_i = d_i x_i + sum_{O_f=i} u_f x_{N_f} + sum_{N_f=i} l_f x_{O_f}; the transpose swaps u and l.
template <class T>
void spmv(const om_mesh& m, int ncomp, bool transpose, const T* diag, const T* upper, const T* lower, const T* x,
          T* y) {
  const T* u = transpose ? lower : upper;
  const T* l = transpose ? upper : lower;
  for (int i = 0; i < m.nc; ++i)
    for (int c = 0; c < ncomp; ++c) y[i * ncomp + c] = diag[i] * x[i * ncomp + c];
  for (int f = 0; f < m.nfi; ++f) {
    int O = m.owner[f], N = m.nbr[f];
    for (int c = 0; c < ncomp; ++c) {
      y[O * ncomp + c] += u[f] * x[N * ncomp + c];
      y[N * ncomp + c] += l[f] * x[O * ncomp + c];
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Krylov solvers on double.  Both follow the textbook algorithms with the stopping rule
// ||r||_2 <= tol ||b||_2 checked after each update (paper Sec. "Numerical schemes and linear
// solvers": CG for the symmetric pressure system, BiCGStab for momentum; Jacobi preconditioning).
// ------------------------------------------------------------------------------------------------
double dotv(const double* a, const double* b, int n) {
#ifdef _OPENMP
  std::vector<double> part(omp_get_max_threads(), 0.0);
#pragma omp parallel
  {
    int t = omp_get_thread_num(), T = omp_get_num_threads();
    int lo = (int)((long long)n * t / T), hi = (int)((long long)n * (t + 1) / T);
    double s = 0.0;
    for (int i = lo; i < hi; ++i) s += a[i] * b[i];
    part[t] = s;
  }
  double s = 0.0;
  for (double v : part) s += v;
  return s;
#else
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
#endif
}

#ifdef _OPENMP
// all-threads LDU product of the timing variant (see the file header), one component
void spmv_threads(const om_mesh& m, const double* diag, const double* u, const double* l, const double* x, double* y) {
  int T = omp_get_max_threads();
  std::vector<std::vector<double>> acc(T);
  std::vector<int> lo(T, 0), hi(T, -1);
#pragma omp parallel num_threads(T)
  {
    int t = omp_get_thread_num();
    int f0 = (int)((long long)m.nfi * t / T), f1 = (int)((long long)m.nfi * (t + 1) / T);
    int a = m.nc, b = -1;
    for (int f = f0; f < f1; ++f) {
      a = std::min(a, std::min(m.owner[f], m.nbr[f]));
      b = std::max(b, std::max(m.owner[f], m.nbr[f]));
    }
    lo[t] = a;
    hi[t] = b;
    std::vector<double>& c = acc[t];
    c.assign(b >= a ? b - a + 1 : 0, 0.0);
    for (int f = f0; f < f1; ++f) {
      int O = m.owner[f], N = m.nbr[f];
      c[O - a] += u[f] * x[N];
      c[N - a] += l[f] * x[O];
    }
#pragma omp barrier
#pragma omp for schedule(static)
    for (int i = 0; i < m.nc; ++i) {
      double v = diag[i] * x[i];
      for (int q = 0; q < T; ++q)
        if (i >= lo[q] && i <= hi[q]) v += acc[q][i - lo[q]];
      y[i] = v;
    }
  }
}
#endif

struct SolveInfo { int iters; double res; int status; };  // status 0 ok, 1 not converged, 2 breakdown

// y = A x for one component (all threads in the timing variant)
void ldu_apply(const om_mesh& m, const double* d, const double* u, const double* l, const double* x, double* y) {
#ifdef _OPENMP
  spmv_threads(m, d, u, l, x, y);
#else
  spmv<double>(m, 1, false, d, u, l, x, y);
#endif
}

// Jacobi-preconditioned CG for a symmetric LDU matrix (upper == lower).
SolveInfo pcg(const om_mesh& m, const double* diag, const double* upper, const double* b, double* x, double tol,
              int maxit) {
  int n = m.nc;
  std::vector<double> r(n), z(n), p(n), q(n);
  ldu_apply(m, diag, upper, upper, x, q.data());
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
  double bn = std::sqrt(dotv(b, b, n));
  SolveInfo info{0, 0.0, 0};
  if (bn == 0.0) { for (int i = 0; i < n; ++i) x[i] = 0.0; return info; }
  double rn = std::sqrt(dotv(r.data(), r.data(), n));
  info.res = rn / bn;
  if (rn <= tol * bn) return info;
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) { z[i] = r[i] / diag[i]; p[i] = z[i]; }
  double rho = dotv(r.data(), z.data(), n);
  while (true) {
    if (info.iters >= maxit) { info.status = 1; return info; }
    ldu_apply(m, diag, upper, upper, p.data(), q.data());
    double alpha = rho / dotv(p.data(), q.data(), n);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    info.iters++;
    rn = std::sqrt(dotv(r.data(), r.data(), n));
    info.res = rn / bn;
    if (rn <= tol * bn) return info;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) z[i] = r[i] / diag[i];
    double rho1 = dotv(r.data(), z.data(), n);
    double beta = rho1 / rho;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    rho = rho1;
  }
}

// Right-Jacobi-preconditioned BiCGStab (van der Vorst 1992) for one component of an LDU system.
SolveInfo bicgstab(const om_mesh& m, const double* diag, const double* upper, const double* lower, const double* b,
                   double* x, double tol, int maxit) {
  int n = m.nc;
  std::vector<double> r(n), rh(n), p(n, 0.0), v(n, 0.0), y(n), s(n), z(n), t(n);
  ldu_apply(m, diag, upper, lower, x, t.data());
  #pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) { r[i] = b[i] - t[i]; rh[i] = r[i]; }
  double bn = std::sqrt(dotv(b, b, n));
  SolveInfo info{0, 0.0, 0};
  if (bn == 0.0) { for (int i = 0; i < n; ++i) x[i] = 0.0; return info; }
  double rn = std::sqrt(dotv(r.data(), r.data(), n));
  info.res = rn / bn;
  if (rn <= tol * bn) return info;
  double rho = 1.0, alpha = 1.0, omega = 1.0;
  while (true) {
    if (info.iters >= maxit) { info.status = 1; return info; }
    double rho1 = dotv(rh.data(), r.data(), n);
    if (rho1 == 0.0) { info.status = 2; return info; }
    double beta = (rho1 / rho) * (alpha / omega);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) { p[i] = r[i] + beta * (p[i] - omega * v[i]); y[i] = p[i] / diag[i]; }
    ldu_apply(m, diag, upper, lower, y.data(), v.data());
    alpha = rho1 / dotv(rh.data(), v.data(), n);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
    double sn = std::sqrt(dotv(s.data(), s.data(), n));
    if (sn <= tol * bn) {
      #pragma omp parallel for schedule(static)
      for (int i = 0; i < n; ++i) x[i] += alpha * y[i];
      info.iters++;
      info.res = sn / bn;
      return info;
    }
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) z[i] = s[i] / diag[i];
    ldu_apply(m, diag, upper, lower, z.data(), t.data());
    double tt = dotv(t.data(), t.data(), n);
    if (tt == 0.0) { info.status = 2; return info; }
    omega = dotv(t.data(), s.data(), n) / tt;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) { x[i] += alpha * y[i] + omega * z[i]; r[i] = s[i] - omega * t[i]; }
    rho = rho1;
    info.iters++;
    rn = std::sqrt(dotv(r.data(), r.data(), n));
    info.res = rn / bn;
    if (rn <= tol * bn) return info;
  }
}

// ------------------------------------------------------------------------------------------------
// Linear solves on the generic scalar.  For dual numbers the solve is differentiated implicitly
// (paper Sec. "Gradient checkpointing and implicit differentiation", eq. implicit_diff):
// A x = b  =>  A xdot = bdot - Adot x, each tangent solved with the same solver on the value matrix.
// ------------------------------------------------------------------------------------------------
SolveInfo solve_sym(const om_mesh& m, const double* d, const double* u, const double* b, double* x, double tol,
                    int maxit, double) {
  return pcg(m, d, u, b, x, tol, maxit);
}
SolveInfo solve_nonsym(const om_mesh& m, const double* d, const double* u, const double* l, const double* b,
                       double* x, double tol, int maxit, double) {
  return bicgstab(m, d, u, l, b, x, tol, maxit);
}

template <bool SYM>
SolveInfo solve_dual(const om_mesh& m, const Dual* d, const Dual* u, const Dual* l, const Dual* b, Dual* x, double tol,
                     int maxit, double tol_tan) {
  int n = m.nc, nf = m.nfi;
  std::vector<double> dv(n), uv(nf), lv(nf), bv(n), xv(n);
  for (int i = 0; i < n; ++i) { dv[i] = d[i].v; bv[i] = b[i].v; xv[i] = x[i].v; }
  for (int f = 0; f < nf; ++f) { uv[f] = u[f].v; lv[f] = l[f].v; }
  SolveInfo info = SYM ? pcg(m, dv.data(), uv.data(), bv.data(), xv.data(), tol, maxit)
                       : bicgstab(m, dv.data(), uv.data(), lv.data(), bv.data(), xv.data(), tol, maxit);
  std::vector<double> rhs(n), xt(n);
  std::vector<std::vector<double>> tang(ND, std::vector<double>(n, 0.0));
  for (int k = 0; k < ND; ++k) {
    bool any = false;
    for (int i = 0; i < n && !any; ++i) any = (b[i].d[k] != 0.0 || d[i].d[k] != 0.0);
    for (int f = 0; f < nf && !any; ++f) any = (u[f].d[k] != 0.0 || l[f].d[k] != 0.0);
    if (!any) continue;
    for (int i = 0; i < n; ++i) rhs[i] = b[i].d[k] - d[i].d[k] * xv[i];
    for (int f = 0; f < nf; ++f) {
      rhs[m.owner[f]] -= u[f].d[k] * xv[m.nbr[f]];
      rhs[m.nbr[f]] -= l[f].d[k] * xv[m.owner[f]];
    }
    std::fill(xt.begin(), xt.end(), 0.0);
    if (SYM) pcg(m, dv.data(), uv.data(), rhs.data(), xt.data(), tol_tan, 100000);
    else bicgstab(m, dv.data(), uv.data(), lv.data(), rhs.data(), xt.data(), tol_tan, 100000);
    tang[k] = xt;
  }
  for (int i = 0; i < n; ++i) {
    x[i] = Dual(xv[i]);
    for (int k = 0; k < ND; ++k) x[i].d[k] = tang[k][i];
  }
  return info;
}
SolveInfo solve_sym(const om_mesh& m, const Dual* d, const Dual* u, const Dual* b, Dual* x, double tol, int maxit,
                    double tol_tan) {
  return solve_dual<true>(m, d, u, u, b, x, tol, maxit, tol_tan);
}
SolveInfo solve_nonsym(const om_mesh& m, const Dual* d, const Dual* u, const Dual* l, const Dual* b, Dual* x,
                       double tol, int maxit, double tol_tan) {
  return solve_dual<false>(m, d, u, l, b, x, tol, maxit, tol_tan);
}

// Verification of a solution computed elsewhere: x is taken as given (no solve) and the true relative
// residual ||b - A x||_2 / ||b||_2 of the system is returned (0 when b = 0), with A x the plain LDU
// product above.  The stopping rule of both Krylov solvers bounds this quantity by tol, up to the
// rounding by which a recursively updated residual drifts from the true one.
double true_residual(const om_mesh& m, const double* d, const double* u, const double* l, const double* b,
                     const double* x) {
  std::vector<double> ax(m.nc);
  spmv<double>(m, 1, false, d, u, l, x, ax.data());
  double rr = 0.0, bb = 0.0;
  for (int i = 0; i < m.nc; ++i) {
    double r = b[i] - ax[i];
    rr += r * r;
    bb += b[i] * b[i];
  }
  return bb == 0.0 ? 0.0 : std::sqrt(rr) / std::sqrt(bb);
}
double true_residual(const om_mesh&, const Dual*, const Dual*, const Dual*, const Dual*, const Dual*) {
  return -1.0;  // verification runs on plain doubles only
}

// ------------------------------------------------------------------------------------------------
// PISO (paper Sec. "PISO as divergence-free constrained message passing", eqs. momentum_predictor,
// Ap_H, pressure_poisson, velocity_correction; Windkessel eqs. windkessel_Q, windkessel_discrete).
// Readings used (the paper leaves these open): implicit backward-Euler predictor with implicit upwind
// convection in a_P; H from the latest velocity in every corrector; one explicit non-orthogonal
// correction per solve from the latest gradient; Windkessel flow lagged to the start of the step;
// pressure reference by diagonal doubling when no pressure value is fixed.
// ------------------------------------------------------------------------------------------------
struct StepStats {
  int it_u[3];
  double res_u[3];
  int it_p[8];
  double res_p[8];
  int status;
};

template <class T>
struct Piso {
  const om_mesh& m;
  om_piso_params prm;
  std::vector<int> codeU, codeP;
  std::vector<double> delta, kf, deltab;
  std::vector<T> Ub, pb;                 // fixed boundary values (pb: fixed p; Windkessel faces overwritten)
  std::vector<T> wk;                     // [nwk*3] Rp, C, Rd
  std::vector<int> wk_of_face;           // per boundary face: Windkessel id or -1
  int nwk = 0;
  bool has_fixed_p = false;
  // Verification mode (plain doubles): the solutions of the step's linear systems are supplied by
  // the caller instead of solved here, the predictor's U*[nc*3] and the pressure after each corrector
  // [n_corr*nc]; the true relative residual of each system is recorded.  Every other operation of
  // the step is unchanged, so the step's outputs are those implied by the supplied solutions.
  const double* given_U = nullptr;
  const double* given_p = nullptr;
  double given_res_u[3] = {0, 0, 0}, given_res_p[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // when set, the values of those solutions are copied out (same layouts) after every solve
  double* trace_U = nullptr;
  double* trace_p = nullptr;
  Piso(const om_mesh& mesh, const om_piso_params& p) : m(mesh), prm(p) {
    codeU = bc_codes(m, TABLE_U);
    codeP = bc_codes(m, TABLE_P);
    delta.resize(m.nfi);
    kf.resize(3 * m.nfi);
    for (int f = 0; f < m.nfi; ++f) { double d[3]; face_geom(m, f, d, delta[f], &kf[3 * f]); }
    deltab.resize(m.nfb);
    for (int b = 0; b < m.nfb; ++b) deltab[b] = bface_delta(m, m.nfi + b);
    wk_of_face.assign(m.nfb, -1);
    for (int q = 0; q < m.npatch; ++q) {
      if (m.pptype[q] == 2) {
        nwk = std::max(nwk, m.pwk[q] + 1);
        for (int f = m.pstart[q]; f < m.pstart[q] + m.psize[q]; ++f) wk_of_face[f - m.nfi] = m.pwk[q];
      }
    }
    for (int b = 0; b < m.nfb; ++b) if (codeP[b] == BC_FIXED) has_fixed_p = true;
  }

  // one step: U, p, phi, pc are updated in place
  void step(std::vector<T>& U, std::vector<T>& p, std::vector<T>& phi, std::vector<T>& pc, StepStats& st) {
    const int nc = m.nc, nfi = m.nfi, nfb = m.nfb;
    const double dt = prm.dt, nu = prm.nu;
    st.status = 0;
    // S0: Windkessel update from the flux at the start of the step (eq. windkessel_discrete)
    std::vector<T> pbv = pb;
    for (int j = 0; j < nwk; ++j) {
      T Q = T(0.0);
      for (int b = 0; b < nfb; ++b) if (wk_of_face[b] == j) Q += phi[nfi + b];
      T Rp = wk[3 * j], Cc = wk[3 * j + 1], Rd = wk[3 * j + 2];
      T E = exp(-dt / (Rd * Cc));
      pc[j] = pc[j] * E + Rd * Q * (1.0 - E);
      T po = pc[j] + Rp * Q;
      for (int b = 0; b < nfb; ++b) if (wk_of_face[b] == j) pbv[b] = po;
    }
    // S1: momentum LDU from the lagged flux: the time scheme's theta-weighted upwind convection and
    // orthogonal diffusion (implicit Euler at theta = 1); the non-orthogonal diffusion part and the
    // deferred correction of a higher-order convection scheme are explicit from U^n and grad(U^n).
    const double th = time_theta(prm.time);
    std::vector<T> gU((size_t)nc * 9);
    grad(m, 3, codeU, U.data(), Ub.data(), gU.data());
    std::vector<T> dM(nc), uM(nfi), lM(nfi), bM((size_t)nc * 3);
    for (int i = 0; i < nc; ++i) {
      dM[i] = T(m.V[i] / dt);
      for (int c = 0; c < 3; ++c) bM[i * 3 + c] = (m.V[i] / dt) * U[i * 3 + c];
    }
    for (int f = 0; f < nfi; ++f) {
      int O = m.owner[f], N = m.nbr[f];
      T F = phi[f];
      T Fp = (val(F) >= 0.0) ? F : T(0.0);   // max(F, 0); the tie F = 0 belongs to the owner side
      T Fm = (val(F) < 0.0) ? F : T(0.0);    // min(F, 0)
      double nd = nu * delta[f];
      T aO = Fp + nd, aN = (-Fm) + nd;       // max(-F, 0) = -min(F, 0)
      T up = Fm - nd, lo = -Fp - nd;
      dM[O] += th * aO;
      dM[N] += th * aN;
      uM[f] = th * up;
      lM[f] = th * lo;
      if (th != 1.0)
        for (int c = 0; c < 3; ++c) {
          bM[O * 3 + c] -= (1.0 - th) * (aO * U[O * 3 + c] + up * U[N * 3 + c]);
          bM[N * 3 + c] -= (1.0 - th) * (aN * U[N * 3 + c] + lo * U[O * 3 + c]);
        }
      double w = m.w[f];
      for (int c = 0; c < 3; ++c) {
        T corr = T(0.0);
        for (int e = 0; e < 3; ++e) corr += kf[3 * f + e] * (w * gU[(O * 3 + c) * 3 + e] + (1.0 - w) * gU[(N * 3 + c) * 3 + e]);
        bM[O * 3 + c] += nu * corr;
        bM[N * 3 + c] -= nu * corr;
      }
    }
    for (int b = 0; b < nfb; ++b) {
      int O = m.owner[nfi + b];
      if (codeU[b] == BC_FIXED) {
        double nd = nu * deltab[b];
        dM[O] += T(th * nd);
        for (int c = 0; c < 3; ++c) bM[O * 3 + c] += (nd - phi[nfi + b]) * Ub[b * 3 + c];
        if (th != 1.0) for (int c = 0; c < 3; ++c) bM[O * 3 + c] -= (1.0 - th) * nd * U[O * 3 + c];
      } else if (codeU[b] == BC_ZEROGRAD) {
        dM[O] += th * phi[nfi + b];
        if (th != 1.0) for (int c = 0; c < 3; ++c) bM[O * 3 + c] -= (1.0 - th) * phi[nfi + b] * U[O * 3 + c];
      }
    }
    // higher-order convection as an explicit source from U^n (part of b, hence of H in every corrector)
    deferred_correction(m, prm.conv, 3, phi.data(), U.data(), gU.data(), bM.data());
    // S2: predictor M U* = b - V grad(p^n), BiCGStab per component from U^n
    std::vector<T> gp((size_t)nc * 3);
    grad(m, 1, codeP, p.data(), pbv.data(), gp.data());
    {
      std::vector<T> rhs(nc), x(nc);
      for (int c = 0; c < 3; ++c) {
        for (int i = 0; i < nc; ++i) { rhs[i] = bM[i * 3 + c] - m.V[i] * gp[i * 3 + c]; x[i] = U[i * 3 + c]; }
        SolveInfo si{0, 0.0, 0};
        if (given_U) {
          for (int i = 0; i < nc; ++i) x[i] = T(given_U[i * 3 + c]);
          given_res_u[c] = true_residual(m, dM.data(), uM.data(), lM.data(), rhs.data(), x.data());
        } else {
          si = solve_nonsym(m, dM.data(), uM.data(), lM.data(), rhs.data(), x.data(), prm.tol_u, prm.maxit_u,
                            prm.tol_tangent);
        }
        if (trace_U) for (int i = 0; i < nc; ++i) trace_U[i * 3 + c] = val(x[i]);
        st.it_u[c] = si.iters;
        st.res_u[c] = si.res;
        if (si.status) st.status = std::max(st.status, si.status);
        for (int i = 0; i < nc; ++i) U[i * 3 + c] = x[i];
      }
    }
    // S3: correctors
    std::vector<T> H((size_t)nc * 3), HbyA((size_t)nc * 3), rAU(nc), phiH(nfi + nfb), rAUf(nfi + nfb);
    std::vector<T> dK(nc), uK(nfi), rhs(nc);
    int ref = -1;
    if (!has_fixed_p) ref = prm.p_ref_cell;
    for (int corr = 0; corr < prm.n_corr; ++corr) {
      // H = b - offdiag(U), HbyA = H/a_P, rAU = V/a_P (eq. Ap_H)
      for (int i = 0; i < nc * 3; ++i) H[i] = bM[i];
      for (int f = 0; f < nfi; ++f) {
        int O = m.owner[f], N = m.nbr[f];
        for (int c = 0; c < 3; ++c) {
          H[O * 3 + c] -= uM[f] * U[N * 3 + c];
          H[N * 3 + c] -= lM[f] * U[O * 3 + c];
        }
      }
      for (int i = 0; i < nc; ++i) {
        rAU[i] = m.V[i] / dM[i];
        for (int c = 0; c < 3; ++c) HbyA[i * 3 + c] = H[i * 3 + c] / dM[i];
      }
      // face flux of HbyA and face value of 1/a_P (linear interpolation; boundary: owner value)
      for (int f = 0; f < nfi; ++f) {
        int O = m.owner[f], N = m.nbr[f];
        double w = m.w[f];
        const double* S = m.Sf + 3 * f;
        T s = T(0.0);
        for (int c = 0; c < 3; ++c) s += (w * HbyA[O * 3 + c] + (1.0 - w) * HbyA[N * 3 + c]) * S[c];
        phiH[f] = s;
        rAUf[f] = w * rAU[O] + (1.0 - w) * rAU[N];
      }
      for (int b = 0; b < nfb; ++b) {
        int f = nfi + b, O = m.owner[f];
        const double* S = m.Sf + 3 * f;
        T s = T(0.0);
        if (codeU[b] == BC_FIXED) for (int c = 0; c < 3; ++c) s += Ub[b * 3 + c] * S[c];
        else if (codeU[b] == BC_ZEROGRAD) for (int c = 0; c < 3; ++c) s += HbyA[O * 3 + c] * S[c];
        phiH[f] = s;
        rAUf[f] = rAU[O];
      }
      // pressure equation (eq. pressure_poisson), negated to its SPD form
      std::vector<T> p_old = p;
      grad(m, 1, codeP, p_old.data(), pbv.data(), gp.data());
      std::fill(dK.begin(), dK.end(), T(0.0));
      std::fill(rhs.begin(), rhs.end(), T(0.0));
      std::vector<T> ncorr(nfi);
      for (int f = 0; f < nfi; ++f) {
        int O = m.owner[f], N = m.nbr[f];
        double w = m.w[f];
        T a = rAUf[f] * delta[f];
        uK[f] = -a;
        dK[O] += a;
        dK[N] += a;
        T kg = T(0.0);
        for (int e = 0; e < 3; ++e) kg += kf[3 * f + e] * (w * gp[O * 3 + e] + (1.0 - w) * gp[N * 3 + e]);
        ncorr[f] = rAUf[f] * kg;
        rhs[O] += -phiH[f] + ncorr[f];
        rhs[N] -= -phiH[f] + ncorr[f];
      }
      for (int b = 0; b < nfb; ++b) {
        int f = nfi + b, O = m.owner[f];
        if (codeP[b] == BC_EMPTY) continue;
        rhs[O] -= phiH[f];
        if (codeP[b] == BC_FIXED) {
          T a = rAUf[f] * deltab[b];
          dK[O] += a;
          rhs[O] += a * pbv[b];
        }
      }
      if (ref >= 0) {
        T d0 = dK[ref];
        rhs[ref] += d0 * prm.p_ref_value;
        dK[ref] = d0 + d0;
      }
      SolveInfo si{0, 0.0, 0};
      if (given_p) {
        for (int i = 0; i < nc; ++i) p[i] = T(given_p[(size_t)corr * nc + i]);
        if (corr < 8) given_res_p[corr] = true_residual(m, dK.data(), uK.data(), uK.data(), rhs.data(), p.data());
      } else {
        si = solve_sym(m, dK.data(), uK.data(), rhs.data(), p.data(), prm.tol_p, prm.maxit_p, prm.tol_tangent);
      }
      if (trace_p) for (int i = 0; i < nc; ++i) trace_p[(size_t)corr * nc + i] = val(p[i]);
      if (corr < 8) { st.it_p[corr] = si.iters; st.res_p[corr] = si.res; }
      if (si.status) st.status = std::max(st.status, si.status);
      // flux correction with the same explicit correction as the right-hand side
      for (int f = 0; f < nfi; ++f) {
        int O = m.owner[f], N = m.nbr[f];
        phi[f] = phiH[f] - (rAUf[f] * delta[f] * (p[N] - p[O]) + ncorr[f]);
      }
      for (int b = 0; b < nfb; ++b) {
        int f = nfi + b, O = m.owner[f];
        if (codeP[b] == BC_EMPTY) { phi[f] = T(0.0); continue; }
        if (codeP[b] == BC_FIXED) phi[f] = phiH[f] - rAUf[f] * deltab[b] * (pbv[b] - p[O]);
        else phi[f] = phiH[f];
      }
      // velocity correction (eq. velocity_correction): U = HbyA - rAU grad(p)
      grad(m, 1, codeP, p.data(), pbv.data(), gp.data());
      for (int i = 0; i < nc; ++i)
        for (int c = 0; c < 3; ++c) U[i * 3 + c] = HbyA[i * 3 + c] - rAU[i] * gp[i * 3 + c];
    }
  }
};

// ------------------------------------------------------------------------------------------------
// renumbering: reverse Cuthill-McKee with George-Liu pseudo-peripheral start, then face re-orientation
// and sorting.  The tie-breaks are fixed so that the result is unique (repository design notes).
// ------------------------------------------------------------------------------------------------
struct Graph {
  std::vector<int> start, adj, deg;
};

Graph cell_graph(const om_mesh& m) {
  Graph g;
  g.deg.assign(m.nc, 0);
  for (int f = 0; f < m.nfi; ++f) { g.deg[m.owner[f]]++; g.deg[m.nbr[f]]++; }
  g.start.assign(m.nc + 1, 0);
  for (int i = 0; i < m.nc; ++i) g.start[i + 1] = g.start[i] + g.deg[i];
  g.adj.assign(g.start[m.nc], 0);
  std::vector<int> fill(g.start.begin(), g.start.end() - 1);
  for (int f = 0; f < m.nfi; ++f) {
    g.adj[fill[m.owner[f]]++] = m.nbr[f];
    g.adj[fill[m.nbr[f]]++] = m.owner[f];
  }
  return g;
}

// BFS from s: returns eccentricity and fills `last` with the deepest level
int bfs_last_level(const Graph& g, int s, std::vector<int>& mark, int stamp, std::vector<int>& last) {
  std::vector<int> level{s};
  mark[s] = stamp;
  int ecc = 0;
  while (true) {
    std::vector<int> next;
    for (int v : level)
      for (int e = g.start[v]; e < g.start[v + 1]; ++e) {
        int u = g.adj[e];
        if (mark[u] != stamp) { mark[u] = stamp; next.push_back(u); }
      }
    if (next.empty()) break;
    level.swap(next);
    ecc++;
  }
  last = level;
  return ecc;
}

std::vector<int> rcm_order(const om_mesh& m) {
  Graph g = cell_graph(m);
  int n = m.nc;
  std::vector<int> visited(n, 0), mark(n, -1), L;
  L.reserve(n);
  int stamp = 0;
  auto less_dv = [&](int a, int b) { return g.deg[a] != g.deg[b] ? g.deg[a] < g.deg[b] : a < b; };
  for (int s0 = 0; s0 < n; ++s0) {
    if (visited[s0]) continue;
    // component of s0 (its smallest index is s0): minimum (degree, index) vertex starts the search
    std::vector<int> comp;
    bfs_last_level(g, s0, mark, ++stamp, comp);  // marks the component with `stamp`
    int r = s0;
    for (int v = s0; v < n; ++v) if (mark[v] == stamp && less_dv(v, r)) r = v;
    std::vector<int> last;
    int ecc = bfs_last_level(g, r, mark, ++stamp, last);
    while (true) {
      int x = last[0];
      for (int v : last) if (less_dv(v, x)) x = v;
      std::vector<int> last2;
      int ecc2 = bfs_last_level(g, x, mark, ++stamp, last2);
      if (ecc2 > ecc) { r = x; ecc = ecc2; last.swap(last2); }
      else break;
    }
    // Cuthill-McKee from r: neighbours appended in (degree, index) order, marked on enqueue
    std::deque<int> q{r};
    visited[r] = 1;
    while (!q.empty()) {
      int v = q.front();
      q.pop_front();
      L.push_back(v);
      std::vector<int> nb;
      for (int e = g.start[v]; e < g.start[v + 1]; ++e) if (!visited[g.adj[e]]) nb.push_back(g.adj[e]);
      std::sort(nb.begin(), nb.end(), less_dv);
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
      for (int u : nb) { visited[u] = 1; q.push_back(u); }
    }
  }
  return L;
}

}  // namespace

// ================================================================================================
// C entry points (called from tests through ctypes)
// ================================================================================================
extern "C" {

int oracle_version(void) { return 6; }  // 6: verification step with supplied solutions
// host threads the Krylov kernels use: 1 in the serial build, the OpenMP thread count in the timing build
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Renumbering.  rcm = 0 keeps the cell order.  Outputs (new -> old where a permutation):
//  cell_perm[nc], face_perm[nfi], face_flip[nfi], owner[nfi], nbr[nfi], own_start[nc+1],
//  losort[nfi], losort_start[nc+1], bface_perm[nfb] (index within [0,nfb)), bowner[nfb].
int oracle_renumber(const om_mesh* m, int rcm, int32_t* cell_perm, int32_t* face_perm, uint8_t* face_flip,
                    int32_t* owner, int32_t* nbr, int32_t* own_start, int32_t* losort, int32_t* losort_start,
                    int32_t* bface_perm, int32_t* bowner) {
  int nc = m->nc, nfi = m->nfi;
  std::vector<int> newof(nc);
  if (rcm) {
    std::vector<int> L = rcm_order(*m);
    for (int k = 0; k < nc; ++k) { cell_perm[nc - 1 - k] = L[k]; newof[L[k]] = nc - 1 - k; }
  } else {
    for (int i = 0; i < nc; ++i) { cell_perm[i] = i; newof[i] = i; }
  }
  struct F { int o, n, orig; bool flip; };
  std::vector<F> fs(nfi);
  for (int f = 0; f < nfi; ++f) {
    int o = newof[m->owner[f]], n = newof[m->nbr[f]];
    bool flip = o > n;
    if (flip) std::swap(o, n);
    fs[f] = {o, n, f, flip};
  }
  std::stable_sort(fs.begin(), fs.end(), [](const F& a, const F& b) { return a.o != b.o ? a.o < b.o : a.n < b.n; });
  for (int f = 0; f < nfi; ++f) {
    face_perm[f] = fs[f].orig; face_flip[f] = fs[f].flip ? 1 : 0; owner[f] = fs[f].o; nbr[f] = fs[f].n;
  }
  for (int i = 0; i <= nc; ++i) own_start[i] = 0;
  for (int f = 0; f < nfi; ++f) own_start[owner[f] + 1]++;
  for (int i = 0; i < nc; ++i) own_start[i + 1] += own_start[i];
  std::vector<int> lo(nfi);
  for (int f = 0; f < nfi; ++f) lo[f] = f;
  std::stable_sort(lo.begin(), lo.end(), [&](int a, int b) { return nbr[a] < nbr[b]; });
  for (int f = 0; f < nfi; ++f) losort[f] = lo[f];
  for (int i = 0; i <= nc; ++i) losort_start[i] = 0;
  for (int f = 0; f < nfi; ++f) losort_start[nbr[f] + 1]++;
  for (int i = 0; i < nc; ++i) losort_start[i + 1] += losort_start[i];
  // boundary faces: stable by new owner inside each patch, patch order kept
  for (int p = 0; p < m->npatch; ++p) {
    std::vector<int> ids;
    for (int f = m->pstart[p]; f < m->pstart[p] + m->psize[p]; ++f) ids.push_back(f - nfi);
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return newof[m->owner[nfi + a]] < newof[m->owner[nfi + b]]; });
    for (size_t k = 0; k < ids.size(); ++k) {
      int dst = m->pstart[p] - nfi + (int)k;
      bface_perm[dst] = ids[k];
      bowner[dst] = newof[m->owner[nfi + ids[k]]];
    }
  }
  return 0;
}

// Matrix bandwidth max |O_f - N_f| of the mesh as given.
int oracle_bandwidth(const om_mesh* m) {
  int bw = 0;
  for (int f = 0; f < m->nfi; ++f) bw = std::max(bw, std::abs(m->owner[f] - m->nbr[f]));
  return bw;
}

// derived geometry per internal face: delta[nfi], k[nfi*3]; boundary deltab[nfb]
int oracle_geometry(const om_mesh* m, double* delta, double* k, double* deltab) {
  for (int f = 0; f < m->nfi; ++f) { double d[3]; face_geom(*m, f, d, delta[f], k + 3 * f); }
  for (int b = 0; b < m->nfb; ++b) deltab[b] = bface_delta(*m, m->nfi + b);
  return 0;
}

int oracle_interp(const om_mesh* m, int ncomp, int table, const double* phi, const double* phib, double* out) {
  interp<double>(*m, ncomp, bc_codes(*m, table), phi, phib, out);
  return 0;
}

int oracle_grad(const om_mesh* m, int ncomp, int table, const double* phi, const double* phib, double* out) {
  grad<double>(*m, ncomp, bc_codes(*m, table), phi, phib, out);
  return 0;
}

// Gauss-Green surface sum from given face values phif[(nfi+nfb)*ncomp]
int oracle_grad_surface(const om_mesh* m, int ncomp, int table, const double* phif, double* out) {
  grad_from_faces<double>(*m, ncomp, bc_codes(*m, table), phif, out);
  return 0;
}

int oracle_div(const om_mesh* m, int scheme, int ncomp, int table, const double* flux, const double* psi,
               const double* psib, double* out) {
  div<double>(*m, scheme, ncomp, bc_codes(*m, table), flux, psi, psib, out);
  return 0;
}

// per-cell sum of |terms| of D(F, psi), used to scale cancellation-aware comparisons
int oracle_div_absterms(const om_mesh* m, int scheme, int ncomp, int table, const double* flux, const double* psi,
                        const double* psib, double* out) {
  std::vector<double> af(m->nfi + m->nfb), ap((size_t)m->nc * ncomp), apb((size_t)m->nfb * ncomp);
  for (int f = 0; f < m->nfi + m->nfb; ++f) af[f] = std::fabs(flux[f]);
  for (size_t i = 0; i < ap.size(); ++i) ap[i] = std::fabs(psi[i]);
  for (size_t i = 0; i < apb.size(); ++i) apb[i] = psib ? std::fabs(psib[i]) : 0.0;
  // upwind selection must follow the signed flux, so evaluate with the signed flux and |psi| per face
  std::vector<int> code = bc_codes(*m, table);
  std::fill(out, out + (size_t)m->nc * ncomp, 0.0);
  for (int f = 0; f < m->nfi; ++f) {
    int O = m->owner[f], N = m->nbr[f];
    for (int c = 0; c < ncomp; ++c) {
      double pf = scheme == 0 ? 1.0 : scheme == 1 ? (flux[f] >= 0 ? ap[O * ncomp + c] : ap[N * ncomp + c])
                                                  : m->w[f] * ap[O * ncomp + c] + (1 - m->w[f]) * ap[N * ncomp + c];
      out[O * ncomp + c] += af[f] * pf;
      out[N * ncomp + c] += af[f] * pf;
    }
  }
  for (int f = m->nfi; f < m->nfi + m->nfb; ++f) {
    int b = f - m->nfi;
    if (code[b] == BC_EMPTY) continue;
    int O = m->owner[f];
    for (int c = 0; c < ncomp; ++c) {
      double pf = scheme == 0 ? 1.0 : (code[b] == BC_FIXED ? apb[b * ncomp + c] : ap[O * ncomp + c]);
      out[O * ncomp + c] += af[f] * pf;
    }
  }
  return 0;
}

int oracle_laplacian(const om_mesh* m, int table, const double* gamma, const double* phi, const double* g,
                     const double* phib, double* out) {
  laplacian<double>(*m, bc_codes(*m, table), gamma, phi, g, phib, out);
  return 0;
}

int oracle_spmv(const om_mesh* m, int ncomp, int transpose, const double* diag, const double* upper,
                const double* lower, const double* x, double* y) {
  spmv<double>(*m, ncomp, transpose != 0, diag, upper, lower ? lower : upper, x, y);
  return 0;
}

// Deferred-correction source alone (see deferred_correction): src[nc*ncomp] = - sum_f sigma F (phi^HO - phi^U)
int oracle_deferred_correction(const om_mesh* m, int conv, int ncomp, const double* flux, const double* phi,
                               const double* g, double* src) {
  std::fill(src, src + (size_t)m->nc * ncomp, 0.0);
  deferred_correction(*m, conv, ncomp, flux, phi, g, src);
  return 0;
}

// Orthogonal (implicit) part of -div(G grad phi) as an SPD LDU matrix K with boundary source:
// upper_f = -G_f delta_f; diag_i = sum G_f delta_f + sum_{b fixed} G_b delta_b;
// rhs_bc_i = sum_{b fixed} G_b delta_b phi_b.
int oracle_assemble_laplace(const om_mesh* m, int table, const double* gamma, const double* phib, double* diag,
                            double* upper, double* rhs_bc) {
  std::vector<int> code = bc_codes(*m, table);
  std::fill(diag, diag + m->nc, 0.0);
  std::fill(rhs_bc, rhs_bc + m->nc, 0.0);
  for (int f = 0; f < m->nfi; ++f) {
    double d[3], delta, k[3];
    face_geom(*m, f, d, delta, k);
    double a = (gamma ? gamma[f] : 1.0) * delta;
    upper[f] = -a;
    diag[m->owner[f]] += a;
    diag[m->nbr[f]] += a;
  }
  for (int b = 0; b < m->nfb; ++b) {
    if (code[b] != BC_FIXED) continue;
    int f = m->nfi + b;
    double a = (gamma ? gamma[f] : 1.0) * bface_delta(*m, f);
    diag[m->owner[f]] += a;
    rhs_bc[m->owner[f]] += a * phib[b];
  }
  return 0;
}

// Momentum LDU (step S1 of the PISO step) for given flux, U^n, boundary values
int oracle_assemble_momentum(const om_mesh* m, double nu, double dt, const double* phi, const double* U,
                             const double* Ub, double* diag, double* upper, double* lower, double* b) {
  std::vector<int> codeU = bc_codes(*m, TABLE_U);
  std::vector<double> gU((size_t)m->nc * 9);
  grad<double>(*m, 3, codeU, U, Ub, gU.data());
  for (int i = 0; i < m->nc; ++i) {
    diag[i] = m->V[i] / dt;
    for (int c = 0; c < 3; ++c) b[i * 3 + c] = (m->V[i] / dt) * U[i * 3 + c];
  }
  for (int f = 0; f < m->nfi; ++f) {
    int O = m->owner[f], N = m->nbr[f];
    double d[3], delta, k[3];
    face_geom(*m, f, d, delta, k);
    double F = phi[f], nd = nu * delta, w = m->w[f];
    double Fp = F >= 0 ? F : 0.0, Fm = F < 0 ? F : 0.0;
    diag[O] += Fp + nd;
    diag[N] += -Fm + nd;
    upper[f] = Fm - nd;
    lower[f] = -Fp - nd;
    for (int c = 0; c < 3; ++c) {
      double corr = 0.0;
      for (int e = 0; e < 3; ++e) corr += k[e] * (w * gU[(O * 3 + c) * 3 + e] + (1 - w) * gU[(N * 3 + c) * 3 + e]);
      b[O * 3 + c] += nu * corr;
      b[N * 3 + c] -= nu * corr;
    }
  }
  for (int bb = 0; bb < m->nfb; ++bb) {
    int f = m->nfi + bb, O = m->owner[f];
    if (codeU[bb] == BC_FIXED) {
      double nd = nu * bface_delta(*m, f);
      diag[O] += nd;
      for (int c = 0; c < 3; ++c) b[O * 3 + c] += (nd - phi[f]) * Ub[bb * 3 + c];
    } else if (codeU[bb] == BC_ZEROGRAD) {
      diag[O] += phi[f];
    }
  }
  return 0;
}

int oracle_pcg(const om_mesh* m, const double* diag, const double* upper, const double* b, double* x, double tol,
               int maxit, int32_t* iters, double* res) {
  SolveInfo si = pcg(*m, diag, upper, b, x, tol, maxit);
  *iters = si.iters; *res = si.res;
  return si.status;
}

// component-wise BiCGStab: b, x are [nc*ncomp] interleaved; iters/res per component
int oracle_bicgstab(const om_mesh* m, int ncomp, const double* diag, const double* upper, const double* lower,
                    const double* b, double* x, double tol, int maxit, int32_t* iters, double* res) {
  int st = 0;
  std::vector<double> bc(m->nc), xc(m->nc);
  for (int c = 0; c < ncomp; ++c) {
    for (int i = 0; i < m->nc; ++i) { bc[i] = b[i * ncomp + c]; xc[i] = x[i * ncomp + c]; }
    SolveInfo si = bicgstab(*m, diag, upper, lower, bc.data(), xc.data(), tol, maxit);
    for (int i = 0; i < m->nc; ++i) x[i * ncomp + c] = xc[i];
    iters[c] = si.iters; res[c] = si.res;
    st = std::max(st, si.status);
  }
  return st;
}

// Passive scalar over one time step with a given face flux (the momentum predictor's discretisation
// applied to one transported scalar c with diffusivity D, Sec. "Spatial discretization"):
//   (V/dt)(c^{n+1} - c^n) + sum_f F_f c_f^upwind - D sum_f (delta_f (c_N - c_O) + k_f . grad c^n_f) = 0,
// convection upwind of the given flux (tie F = 0 to the owner) plus the deferred correction of the
// scheme conv from c^n, diffusion in its orthogonal part and explicit in the non-orthogonal correction
// from the Gauss gradient of c^n, the matrix part weighted by the time scheme (time_theta; implicit
// Euler by default);
// boundary faces by the table's codes with values cb (fixed) or c of the owner (zeroGradient).
// Solved by BiCGStab from c^n; c is overwritten.
int oracle_transport_scalar(const om_mesh* m, int table, int conv, int time, double D, double dt, const double* phi,
                            const double* cb, double* c, double tol, int maxit, int32_t* iters, double* res) {
  const double th = time_theta(time);
  std::vector<int> code = bc_codes(*m, table);
  std::vector<double> g((size_t)m->nc * 3);
  grad<double>(*m, 1, code, c, cb, g.data());
  std::vector<double> diag(m->nc), upper(std::max(1, m->nfi)), lower(std::max(1, m->nfi)), b(m->nc);
  for (int i = 0; i < m->nc; ++i) {
    diag[i] = m->V[i] / dt;
    b[i] = (m->V[i] / dt) * c[i];
  }
  for (int f = 0; f < m->nfi; ++f) {
    int O = m->owner[f], N = m->nbr[f];
    double d[3], delta, k[3];
    face_geom(*m, f, d, delta, k);
    double F = phi[f], nd = D * delta, w = m->w[f];
    double Fp = F >= 0 ? F : 0.0, Fm = F < 0 ? F : 0.0;
    double aO = Fp + nd, aN = -Fm + nd, up = Fm - nd, lo = -Fp - nd;
    diag[O] += th * aO;
    diag[N] += th * aN;
    upper[f] = th * up;
    lower[f] = th * lo;
    if (th != 1.0) {
      b[O] -= (1.0 - th) * (aO * c[O] + up * c[N]);
      b[N] -= (1.0 - th) * (aN * c[N] + lo * c[O]);
    }
    double corr = 0.0;
    for (int e = 0; e < 3; ++e) corr += k[e] * (w * g[O * 3 + e] + (1 - w) * g[N * 3 + e]);
    b[O] += D * corr;
    b[N] -= D * corr;
  }
  for (int bb = 0; bb < m->nfb; ++bb) {
    int f = m->nfi + bb, O = m->owner[f];
    if (code[bb] == BC_FIXED) {
      double nd = D * bface_delta(*m, f);
      diag[O] += th * nd;
      b[O] += (nd - phi[f]) * cb[bb];
      if (th != 1.0) b[O] -= (1.0 - th) * nd * c[O];
    } else if (code[bb] == BC_ZEROGRAD) {
      diag[O] += th * phi[f];
      if (th != 1.0) b[O] -= (1.0 - th) * phi[f] * c[O];
    }
  }
  deferred_correction(*m, conv, 1, phi, c, g.data(), b.data());
  SolveInfo si = bicgstab(*m, diag.data(), upper.data(), lower.data(), b.data(), c, tol, maxit);
  *iters = si.iters;
  *res = si.res;
  return si.status;
}

// Initial flux phi0 = interp(U0).S with boundary values from the velocity BC.
int oracle_initial_flux(const om_mesh* m, const double* U, const double* Ub, double* phi) {
  std::vector<int> code = bc_codes(*m, TABLE_U);
  std::vector<double> Uf((size_t)(m->nfi + m->nfb) * 3);
  interp<double>(*m, 3, code, U, Ub, Uf.data());
  for (int f = 0; f < m->nfi + m->nfb; ++f) phi[f] = dot3(&Uf[3 * f], m->Sf + 3 * f);
  return 0;
}

int oracle_piso_run_trace(const om_mesh* m, const om_piso_params* prm, const double* Ub, const double* pb,
                          const double* wk, int nwk, double* pc, double* U, double* p, double* phi, int nsteps,
                          int32_t* iters, double* res, double* Ustar, double* pcorr);

// PISO run: nsteps steps from (U, p, phi, pc); all updated in place.  Ub[nfb*3] / pb[nfb] hold the
// fixed values (ignored on other faces); wk[nwk*3] = (Rp, C, Rd) per Windkessel.
// stats: per step [3 it_u, n_corr it_p] as int32 and [3 res_u, n_corr res_p] as double.
int oracle_piso_run(const om_mesh* m, const om_piso_params* prm, const double* Ub, const double* pb, const double* wk,
                    int nwk, double* pc, double* U, double* p, double* phi, int nsteps, int32_t* iters,
                    double* res) {
  return oracle_piso_run_trace(m, prm, Ub, pb, wk, nwk, pc, U, p, phi, nsteps, iters, res, nullptr, nullptr);
}

// As oracle_piso_run, also copying out the solution of every linear solve (may be NULL):
// Ustar[nsteps*nc*3] (predictor) and pcorr[nsteps*n_corr*nc] (pressure after each corrector).
int oracle_piso_run_trace(const om_mesh* m, const om_piso_params* prm, const double* Ub, const double* pb,
                          const double* wk, int nwk, double* pc, double* U, double* p, double* phi, int nsteps,
                          int32_t* iters, double* res, double* Ustar, double* pcorr) {
  Piso<double> S(*m, *prm);
  S.Ub.assign(Ub, Ub + (size_t)m->nfb * 3);
  S.pb.assign(pb, pb + m->nfb);
  S.wk.assign(wk, wk + 3 * std::max(nwk, S.nwk));
  std::vector<double> vU(U, U + (size_t)m->nc * 3), vp(p, p + m->nc), vphi(phi, phi + m->nfi + m->nfb),
      vpc(pc, pc + std::max(nwk, S.nwk));
  int status = 0;
  int per = 3 + prm->n_corr;
  for (int s = 0; s < nsteps; ++s) {
    StepStats st{};
    S.trace_U = Ustar ? Ustar + (size_t)s * m->nc * 3 : nullptr;
    S.trace_p = pcorr ? pcorr + (size_t)s * prm->n_corr * m->nc : nullptr;
    S.step(vU, vp, vphi, vpc, st);
    status = std::max(status, st.status);
    if (iters) {
      for (int c = 0; c < 3; ++c) { iters[s * per + c] = st.it_u[c]; res[s * per + c] = st.res_u[c]; }
      for (int c = 0; c < prm->n_corr && c < 8; ++c) { iters[s * per + 3 + c] = st.it_p[c]; res[s * per + 3 + c] = st.res_p[c]; }
    }
  }
  std::copy(vU.begin(), vU.end(), U);
  std::copy(vp.begin(), vp.end(), p);
  std::copy(vphi.begin(), vphi.end(), phi);
  std::copy(vpc.begin(), vpc.end(), pc);
  return status;
}

// One PISO step from (U, p, phi, pc) with the solutions of its linear systems supplied (verification
// mode of Piso): Ustar[nc*3] for the predictor, pcorr[n_corr*nc] for the pressure after each
// corrector.  The state is updated in place to what the step computes from those solutions, and
// res_u[3] / res_p[n_corr] receive the true relative residual of each system.
int oracle_piso_check_step(const om_mesh* m, const om_piso_params* prm, const double* Ub, const double* pb,
                           const double* wk, int nwk, double* pc, double* U, double* p, double* phi,
                           const double* Ustar, const double* pcorr, double* res_u, double* res_p) {
  if (prm->n_corr < 1 || prm->n_corr > 8) return -1;
  Piso<double> S(*m, *prm);
  S.Ub.assign(Ub, Ub + (size_t)m->nfb * 3);
  S.pb.assign(pb, pb + m->nfb);
  S.wk.assign(wk, wk + 3 * std::max(nwk, S.nwk));
  S.given_U = Ustar;
  S.given_p = pcorr;
  std::vector<double> vU(U, U + (size_t)m->nc * 3), vp(p, p + m->nc), vphi(phi, phi + m->nfi + m->nfb),
      vpc(pc, pc + std::max(nwk, S.nwk));
  StepStats st{};
  S.step(vU, vp, vphi, vpc, st);
  std::copy(vU.begin(), vU.end(), U);
  std::copy(vp.begin(), vp.end(), p);
  std::copy(vphi.begin(), vphi.end(), phi);
  std::copy(vpc.begin(), vpc.end(), pc);
  for (int c = 0; c < 3; ++c) res_u[c] = S.given_res_u[c];
  for (int c = 0; c < prm->n_corr; ++c) res_p[c] = S.given_res_p[c];
  return 0;
}

// Tangent (forward-mode) PISO run with nd <= 10 directions.  Seeds per direction k:
//  dwk[k*nwk*3 + ...], dU0[k*nc*3], dp0[k*nc], dphi0[k*(nfi+nfb)], dpc0[k*nwk] (any may be NULL = 0).
// Outputs the final state values (U, p, phi, pc in place) and its tangents tU[k*nc*3], tp, tphi, tpc.
int oracle_piso_tangent(const om_mesh* m, const om_piso_params* prm, const double* Ub, const double* pb,
                        const double* wk, int nwk, double* pc, double* U, double* p, double* phi, int nsteps, int nd,
                        const double* dwk, const double* dU0, const double* dp0, const double* dphi0,
                        const double* dpc0, const double* dUb, double* tU, double* tp, double* tphi, double* tpc) {
  if (nd > ND || nd < 0) return -1;
  Piso<Dual> S(*m, *prm);
  int nc = m->nc, nf = m->nfi + m->nfb;
  int nw = std::max(nwk, S.nwk);
  S.Ub.resize((size_t)m->nfb * 3);
  for (size_t i = 0; i < S.Ub.size(); ++i) {
    S.Ub[i] = Dual(Ub[i]);
    for (int k = 0; k < nd; ++k) S.Ub[i].d[k] = dUb ? dUb[(size_t)k * m->nfb * 3 + i] : 0.0;
  }
  S.pb.resize(m->nfb);
  for (int i = 0; i < m->nfb; ++i) S.pb[i] = Dual(pb[i]);
  S.wk.resize(3 * nw);
  for (int j = 0; j < 3 * nw; ++j) {
    S.wk[j] = Dual(wk[j]);
    for (int k = 0; k < nd; ++k) S.wk[j].d[k] = dwk ? dwk[(size_t)k * 3 * nw + j] : 0.0;
  }
  std::vector<Dual> vU((size_t)nc * 3), vp(nc), vphi(nf), vpc(nw);
  for (int i = 0; i < nc * 3; ++i) { vU[i] = Dual(U[i]); for (int k = 0; k < nd; ++k) vU[i].d[k] = dU0 ? dU0[(size_t)k * nc * 3 + i] : 0.0; }
  for (int i = 0; i < nc; ++i) { vp[i] = Dual(p[i]); for (int k = 0; k < nd; ++k) vp[i].d[k] = dp0 ? dp0[(size_t)k * nc + i] : 0.0; }
  for (int i = 0; i < nf; ++i) { vphi[i] = Dual(phi[i]); for (int k = 0; k < nd; ++k) vphi[i].d[k] = dphi0 ? dphi0[(size_t)k * nf + i] : 0.0; }
  for (int j = 0; j < nw; ++j) { vpc[j] = Dual(pc[j]); for (int k = 0; k < nd; ++k) vpc[j].d[k] = dpc0 ? dpc0[(size_t)k * nw + j] : 0.0; }
  int status = 0;
  for (int s = 0; s < nsteps; ++s) {
    StepStats st{};
    S.step(vU, vp, vphi, vpc, st);
    status = std::max(status, st.status);
  }
  for (int i = 0; i < nc * 3; ++i) { U[i] = vU[i].v; for (int k = 0; k < nd; ++k) tU[(size_t)k * nc * 3 + i] = vU[i].d[k]; }
  for (int i = 0; i < nc; ++i) { p[i] = vp[i].v; for (int k = 0; k < nd; ++k) tp[(size_t)k * nc + i] = vp[i].d[k]; }
  for (int i = 0; i < nf; ++i) { phi[i] = vphi[i].v; for (int k = 0; k < nd; ++k) tphi[(size_t)k * nf + i] = vphi[i].d[k]; }
  for (int j = 0; j < nw; ++j) { pc[j] = vpc[j].v; for (int k = 0; k < nd; ++k) tpc[(size_t)k * nw + j] = vpc[j].d[k]; }
  return status;
}

}  // extern "C"
