// Device side of the smoothed-aggregation AMG preconditioner for the pressure CG.
//
// One V-cycle, z = M^-1 r, from level 0 (the cell-slot matrix K of the mesh, internal order) down to
// a coarsest level solved with its dense inverse:
//   down, level l:  x_l = S_l(b_l) (smoothing from zero),  res_l = b_l - A_l x_l,
//                   b_{l+1} = R_l res_l                         (b_0 = r)
//   coarsest:       x_L = A_L^-1 b_L
//   up, level l:    t_l = x_l + P_l x_{l+1},  x_l = t_l + S_l(b_l - A_l t_l)   (z = x_0)
// Every smoother is one degree-2 Chebyshev sweep in D_l^-1 A_l over [hi_l / 10, hi_l] (a fixed
// polynomial in D^-1 A times D^-1), the same before and after the coarse correction, and R_l = P_l^T,
// so M^-1 is symmetric; it is positive definite while the spectrum of D^-1 A stays below
// hi + lo = 1.1 hi, where the smoothing polynomial contracts.  hi_0 is a Gershgorin bound of D^-1 K
// (at least 2, which bounds every weakly diagonally dominant K); hi_l = 1.1 times the setup's
// power-iteration estimate of rho(D_l^-1 A_l) on the stored coarse operators, capped by their
// Gershgorin bound.  A sweep takes two passes over the level's operator: from zero, D^-1 b gives d0
// without one; on the way up the first pass uses b_l - A_l t_l = res_l - (A_l P_l) x_{l+1}, with
// A_l P_l stored, so prolongation and that residual are one pass on levels l >= 1 (level 0 smooths
// with the operator of the current solve and keeps the prolongation a pass of its own).  Degree-2 Chebyshev on every level takes about half the
// CG iterations of one damped-Jacobi step per level, which more than pays for the extra passes.
// Each stage is one kernel: row kernels on the cell-slot layout for level 0, CSR kernels with SW
// lanes per row (rows summed by a fixed shuffle tree) elsewhere, so every result is deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "amg_dev.h"
#include "krylov_util.h"

namespace difvm {

namespace {

struct DevCsr {
  int n = 0, nnz = 0, sw = 1;  // sw: lanes per row in the CSR kernels
  int32_t *ptr = nullptr, *col = nullptr;
  double *val = nullptr, *diag = nullptr;
  double* val2 = nullptr;  // A P: P's values on its pattern
};
}  // namespace

struct AmgDev {
  difvm_mesh* mesh = nullptr;
  int L = 0;                     // coarse levels 1..L (level L is the coarsest)
  std::vector<DevCsr> A;         // A[l], l = 1..L (A[0] unused: level 0 is K)
  DevCsr P0;                     // prolongation from level 1 to level 0
  std::vector<DevCsr> R, AP;     // R[l]: rows of level l+1, columns of l; AP[l] (l >= 1): rows of l
  std::vector<double*> b, bd, res, x;  // per level (index 0: res only; bd: D^-1 b, levels 1..L-1)
  std::vector<double*> xs, t, d0;      // levels 0..L-1: pre-smoothed x, xs + P x_{l+1}, first
                                       // post-smoothing step
  std::vector<double> hi;        // levels 0..L-1: upper end of the Chebyshev interval
  double* cinv = nullptr;        // dense inverse of A_L, row-major
  std::vector<int> rows;
  std::vector<void*> allocs;
};

namespace {

template <class T>
T* up(AmgDev* a, const std::vector<T>& v, hipStream_t s) {
  T* p = dalloc<T>(ctx_of(a->mesh), v.size());
  a->allocs.push_back(p);
  upload(p, v, s);
  return p;
}
double* work(AmgDev* a, size_t n) {
  double* p = dalloc<double>(ctx_of(a->mesh), n);
  a->allocs.push_back(p);
  return p;
}

// Lanes per CSR row: per_lane to 2 per_lane entries per lane on average.  The single-product kernels
// take 4 to 8 (their eight loads in flight hide the gather latency without many short-lived waves;
// they wait on memory latency more than on bandwidth); the two-product pass over A P takes 2 to 4.
// A matrix of few rows gets more lanes (down to 2 entries each) until the launch has 64k threads:
// there the chip is far from full and each lane's chain of loads is the whole kernel's time.
int lanes_for(int n, size_t nnz, int per_lane) {
  double avg = n ? (double)nnz / n : 0.0;
  int sw = 1;
  while (sw < 64 && sw * 2 * per_lane <= avg) sw *= 2;
  while (sw < 64 && (size_t)n * sw < 65536 && sw * 4 <= avg) sw *= 2;
  return sw;
}

DevCsr upload_csr(AmgDev* a, const AmgCsr& M, bool with_diag, hipStream_t s, int per_lane = 4) {
  DevCsr d;
  d.n = M.n;
  d.nnz = (int)M.col.size();
  d.sw = lanes_for(M.n, M.col.size(), per_lane);
  d.ptr = up(a, M.ptr, s);
  d.col = up(a, M.col, s);
  d.val = up(a, M.val, s);
  if (with_diag) d.diag = up(a, M.diag, s);
  return d;
}

// ---- kernels ------------------------------------------------------------------------------------
// Every segment's CG stopped: the V-cycle of an iteration queued past the stop has nothing to do.
// The flags are written only by the CG kernels queued before the V-cycle on the same stream, so they
// do not change while a V-cycle kernel runs: every wave reads them itself, one segment per lane, and
// votes (no barrier), and whole blocks return together.  Called first thing, with every lane active.
struct StopFlags {
  const PcgCtl* ctl;  // nullptr: never stopped
  int nseg;
};
__device__ __forceinline__ bool stopped(const StopFlags& st) {
  if (!st.ctl) return false;
  int all = 1;
  for (int g = threadIdx.x & 63; g < st.nseg; g += 64) all &= st.ctl[g].done;
  return __all(all) != 0;
}

// Sum of val[q] x(col[q]) over q = lo, lo + SW, lo + 2 SW, ... < hi (one lane's share of a CSR row),
// in that order, with the loads of UN entries in flight together (rows of a few entries per lane
// would otherwise wait on one load chain per entry; with 4 to 8 entries per lane, one round).  Entries past the row's end load its last entry
// (no branch around a load, which would make each one wait) and are not added.
template <int SW, int UN = 8, class X>
__device__ __forceinline__ double csr_lane_dot(int lo, int hi, const int32_t* __restrict__ col,
                                               const double* __restrict__ val, X&& x) {
  double s = 0.0;
  for (int q = lo; q < hi; q += UN * SW) {
    int c[UN];
    double v[UN], xv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      int k = min(q + u * SW, hi - 1);
      c[u] = col[k];
      v[u] = val[k];
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) xv[u] = x(c[u]);
#pragma unroll
    for (int u = 0; u < UN; ++u)
      if (q + u * SW < hi) s += v[u] * xv[u];
  }
  return s;
}

// The same for two value arrays on one pattern: sa = sum va[q] x(col[q]), sb = sum vb[q] x(col[q]).
template <int SW, int UN = 4, class X>
__device__ __forceinline__ void csr_lane_dot2(int lo, int hi, const int32_t* __restrict__ col,
                                              const double* __restrict__ va, const double* __restrict__ vb, X&& x,
                                              double& sa, double& sb) {
  sa = 0.0;
  sb = 0.0;
  for (int q = lo; q < hi; q += UN * SW) {
    int c[UN];
    double a[UN], b[UN], xv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      int k = min(q + u * SW, hi - 1);
      c[u] = col[k];
      a[u] = va[k];
      b[u] = vb[k];
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) xv[u] = x(c[u]);
#pragma unroll
    for (int u = 0; u < UN; ++u)
      if (q + u * SW < hi) {
        sa += a[u] * xv[u];
        sb += b[u] * xv[u];
      }
  }
}

// column of slot `at` in row i (16-bit offsets when the mesh has them)
template <bool OFF16>
__device__ __forceinline__ int slot_col_of(const SellView& K, int i, int at) {
  if constexpr (OFF16) return i + K.off16[at];
  else return K.col[at];
}

// Off-diagonal part of row i of K applied to f: sum over the row's slots of K_ij f(j) (padding and
// boundary slots hold 0 and the row's own index)
// (slots in layout order, the first four with every load issued before any is used)
template <bool OFF16, class F>
__device__ __forceinline__ double sell_offdiag(const SellView& K, int i, SlotRange R, F&& f) {
  double acc = 0.0;
  walk_row<4>(R.width, [&](auto Wc, int k0) {
    constexpr int N = decltype(Wc)::value;
    double a[N], fj[N];
    int j[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      int at = R.base + (k0 + k) * SLICE;
      a[k] = K.val[at];
      j[k] = slot_col_of<OFF16>(K, i, at);
    }
#pragma unroll
    for (int k = 0; k < N; ++k) fj[k] = f(j[k]);
#pragma unroll
    for (int k = 0; k < N; ++k) acc += a[k] * fj[k];
  });
  return acc;
}

// The degree-2 Chebyshev sweep in D^-1 A over [lo, hi] (hi bounds the spectrum of D^-1 A), the same
// before and after the coarse correction.  From x with residual rh0 = D^-1 (b - A x):  d0 = rh0 / theta,  rh1 = rh0 - D^-1 K d0,  d1 = c_d d0 + c_r rh1,
// x <- x + d0 + d1,  with theta = (hi + lo) / 2, delta = (hi - lo) / 2, sigma = theta / delta,
// rho0 = 1 / sigma, rho1 = 1 / (2 sigma - rho0), c_d = rho1 rho0, c_r = 2 rho1 / delta.
struct Cheb {
  double theta, inv_theta, c_d, c_r;
};

Cheb cheb_coefficients(double lo, double hi) {
  double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  double sigma = theta / delta, rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
  return {theta, 1.0 / theta, rho1 * rho0, 2.0 * rho1 / delta};
}

// level 0, down, first pass (x = 0, b = r): xs = d0 + d1, with d0 = D^-1 r / theta
template <bool OFF16>
__global__ __launch_bounds__(BLOCK) void k_amg_cheb_pre1(SellView K, const double* __restrict__ r,
                                                         double* __restrict__ xs, Cheb c, StopFlags ctl) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  // row range loaded at a clamped index, without a branch around the load, so that it is in flight
  // together with the flag reads
  SlotRange R = slots_of(K, min(i, K.nc - 1));
  if (stopped(ctl) || i >= K.nc) return;
  double di = K.diag[i], rh0 = r[i] / di;
  double d0 = rh0 * c.inv_theta;
  double kd0 = di * d0 + sell_offdiag<OFF16>(K, i, R, [&](int j) { return r[j] / K.diag[j] * c.inv_theta; });
  double rh1 = rh0 - kd0 / di;
  xs[i] = d0 + (c.c_d * d0 + c.c_r * rh1);
}

// level 0, down, second pass: res = r - K xs
template <bool OFF16>
__global__ __launch_bounds__(BLOCK) void k_amg_cheb_pre2(SellView K, const double* __restrict__ r,
                                                         const double* __restrict__ xs, double* __restrict__ res,
                                                         StopFlags ctl) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  SlotRange R = slots_of(K, min(i, K.nc - 1));
  if (stopped(ctl) || i >= K.nc) return;
  const double ri = r[i];
  double kx = K.diag[i] * xs[i] + sell_offdiag<OFF16>(K, i, R, [&](int j) { return xs[j]; });
  res[i] = ri - kx;
}

// level 0, up, first pass (x = t): d0 = D^-1 (r - K t) / theta
template <bool OFF16>
__global__ __launch_bounds__(BLOCK) void k_amg_cheb_post1(SellView K, const double* __restrict__ r,
                                                          const double* __restrict__ t, double* __restrict__ d0,
                                                          Cheb c, StopFlags ctl) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  SlotRange R = slots_of(K, min(i, K.nc - 1));
  if (stopped(ctl) || i >= K.nc) return;
  const double di = K.diag[i], ri = r[i];
  double kt = di * t[i] + sell_offdiag<OFF16>(K, i, R, [&](int j) { return t[j]; });
  d0[i] = (ri - kt) / di * c.inv_theta;
}

// level 0, up, second pass: z = t + d0 + d1 with rh1 = theta d0 - D^-1 K d0, and per-tile partials
// of r.z.  A block per tile and one cell per thread, like the other finest-level passes (four cells
// per thread in 256-thread blocks left each thread's rows one after another).
constexpr int POST2_NT = TILE;
template <bool OFF16>
__global__ __launch_bounds__(POST2_NT) void k_amg_cheb_post2(SellView K, Tiles T, const double* __restrict__ r,
                                                             const double* __restrict__ t, const double* __restrict__ d0,
                                                             double* __restrict__ z, double* __restrict__ part, Cheb c,
                                                             StopFlags ctl) {
  TileIdx ti = tile_idx(T);
  if (stopped(ctl)) return;
  double v[1] = {0.0};
  if (const int i = ti.lo + (int)threadIdx.x; i < ti.hi) {
    SlotRange R = slots_of(K, i);
    const double di = K.diag[i], d0i = d0[i], ti = t[i], ri = r[i];
    double kd0 = di * d0i + sell_offdiag<OFF16>(K, i, R, [&](int j) { return d0[j]; });
    double rh1 = c.theta * d0i - kd0 / di;
    double zi = ti + d0i + (c.c_d * d0i + c.c_r * rh1);
    z[i] = zi;
    v[0] = ri * zi;
  }
  if (part) put_partial<1, POST2_NT>(v, part, T.ntile, ti.t);
}

// SW lanes per row: partial sums of the row's entries, then a fixed xor-shuffle tree
template <int SW>
__device__ __forceinline__ double lane_sum(double s) {
#pragma unroll
  for (int off = SW / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, SW);
  return s;
}

// Coarse levels smooth with the same degree-2 Chebyshev sweep as level 0 (interval [hi / 10, hi],
// hi from the setup), two CSR passes per sweep.
// Row bounds are loaded at a clamped index before the flag reads (no branch around the loads, so
// both are in flight together); rows past the end get an empty range.  The kernels load their own
// row's values (at the clamped index rr) before the row's entries, so that those loads are in flight
// with the entries' and not issued after the gathers.  Blocks map to rows XCD by XCD
// (each XCD a contiguous run of rows), so the finer-level entries that neighbouring rows gather meet
// in one L2.
#define DIFVM_AMG_ROW(ptr, n)                                  \
  int g = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x; \
  int row = g / SW, lane = g % SW;                             \
  const int rr = min(row, n - 1);                              \
  int p0 = ptr[rr], p1 = ptr[rr + 1];                          \
  if (stopped(ctl)) return;                                    \
  int lo = p0 + lane, hi = row < n ? p1 : 0

// out = R x (rows of the coarser level); with diag, also outd = out / diag (what the coarser level's
// pre-smoothing gathers)
template <int SW>
__global__ __launch_bounds__(BLOCK) void k_amg_restrict(int n, const int32_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ col, const double* __restrict__ val,
                                                        const double* __restrict__ xin, const double* __restrict__ diag,
                                                        double* __restrict__ out, double* __restrict__ outd,
                                                        StopFlags ctl) {
  DIFVM_AMG_ROW(ptr, n);
  const double dg = diag ? diag[rr] : 1.0;
  double s = csr_lane_dot<SW>(lo, hi, col, val, [&](int j) { return xin[j]; });
  s = lane_sum<SW>(s);
  if (row < n && lane == 0) {
    out[row] = s;
    if (diag) outd[row] = s / dg;
  }
}

// coarse level, down, first pass (x = 0): xs = d0 + d1 with d0 = bd / theta (bd = D^-1 b)
template <int SW>
__global__ __launch_bounds__(BLOCK) void k_amg_cpre1(int n, const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col, const double* __restrict__ val,
                                                     const double* __restrict__ diag, const double* __restrict__ bd,
                                                     double* __restrict__ xs, Cheb c, StopFlags ctl) {
  DIFVM_AMG_ROW(ptr, n);
  const double di = diag[rr], rh0 = bd[rr];
  double s = csr_lane_dot<SW>(lo, hi, col, val, [&](int j) { return bd[j]; });
  s = lane_sum<SW>(s);
  if (row < n && lane == 0) {
    double d0 = rh0 * c.inv_theta;
    double kd0 = di * d0 + s * c.inv_theta;
    double rh1 = rh0 - kd0 / di;
    xs[row] = d0 + (c.c_d * d0 + c.c_r * rh1);
  }
}

// coarse level, down, second pass: res = b - A xs
template <int SW>
__global__ __launch_bounds__(BLOCK) void k_amg_cpre2(int n, const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col, const double* __restrict__ val,
                                                     const double* __restrict__ diag, const double* __restrict__ b,
                                                     const double* __restrict__ xs, double* __restrict__ res,
                                                     StopFlags ctl) {
  DIFVM_AMG_ROW(ptr, n);
  const double bi = b[rr], di = diag[rr], xi = xs[rr];
  double s = csr_lane_dot<SW>(lo, hi, col, val, [&](int j) { return xs[j]; });
  s = lane_sum<SW>(s);
  if (row < n && lane == 0) res[row] = bi - di * xi - s;
}

// coarse level, up, first pass: t = xs + P xc and, since b - A t = res - (A P) xc,
// d0 = D^-1 (res - (A P) xc) / theta; one pass over the pattern of A P
template <int SW>
__global__ __launch_bounds__(BLOCK) void k_amg_cup1(int n, const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col, const double* __restrict__ ap,
                                                    const double* __restrict__ pv, const double* __restrict__ diag,
                                                    const double* __restrict__ xs, const double* __restrict__ res,
                                                    const double* __restrict__ xc, double* __restrict__ t,
                                                    double* __restrict__ d0, Cheb c, StopFlags ctl) {
  DIFVM_AMG_ROW(ptr, n);
  const double xi = xs[rr], ri = res[rr], di = diag[rr];
  double sp, sq;
  csr_lane_dot2<SW>(lo, hi, col, pv, ap, [&](int j) { return xc[j]; }, sp, sq);
  sp = lane_sum<SW>(sp);
  sq = lane_sum<SW>(sq);
  if (row < n && lane == 0) {
    t[row] = xi + sp;
    d0[row] = (ri - sq) / di * c.inv_theta;
  }
}

// coarse level, up, second pass: x = t + d0 + d1 with rh1 = theta d0 - D^-1 A d0
template <int SW>
__global__ __launch_bounds__(BLOCK) void k_amg_cup2(int n, const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col, const double* __restrict__ val,
                                                    const double* __restrict__ diag, const double* __restrict__ t,
                                                    const double* __restrict__ d0, double* __restrict__ x, Cheb c,
                                                    StopFlags ctl) {
  DIFVM_AMG_ROW(ptr, n);
  const double di = diag[rr], d0i = d0[rr], ti = t[rr];
  double s = csr_lane_dot<SW>(lo, hi, col, val, [&](int j) { return d0[j]; });
  s = lane_sum<SW>(s);
  if (row < n && lane == 0) {
    double rh1 = c.theta * d0i - (di * d0i + s) / di;
    x[row] = ti + d0i + (c.c_d * d0i + c.c_r * rh1);
  }
}

// level 0, up: t = xs + P xc (one thread per row; almost every row of the finest prolongator has at
// most four entries, so four in flight)
__global__ __launch_bounds__(BLOCK) void k_amg_prolong(int n, const int32_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ col, const double* __restrict__ val,
                                                       const double* __restrict__ xs, const double* __restrict__ xc,
                                                       double* __restrict__ t, StopFlags ctl) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  int lo = ptr[min(i, n - 1)], hi = ptr[min(i, n - 1) + 1];
  if (stopped(ctl) || i >= n) return;
  const double xi = xs[i];
  double s = csr_lane_dot<1, 4>(lo, hi, col, val, [&](int j) { return xc[j]; });
  t[i] = xi + s;
}

// coarsest: x = A_L^-1 b with the dense inverse (row-major, n <= 2048): one block per row, threads
// over the columns (every load of a thread in flight at once: n / BLOCK <= 8), per-wave shuffle trees
// and the four wave sums added in order; b is read through L2
constexpr int MAX_DENSE = 2048;
__global__ __launch_bounds__(BLOCK) void k_amg_coarsest(int n, const double* __restrict__ inv,
                                                        const double* __restrict__ b, double* __restrict__ x,
                                                        StopFlags ctl) {
  if (stopped(ctl)) return;
  __shared__ double ws[BLOCK / 64];
  const double* row = inv + (size_t)blockIdx.x * n;
  constexpr int U = MAX_DENSE / BLOCK;
  double v[U], w[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {  // columns past the end load column n-1 (no branch around a load)
    int j = min((int)threadIdx.x + u * BLOCK, n - 1);
    v[u] = row[j];
    w[u] = b[j];
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if ((int)threadIdx.x + u * BLOCK < n) s += v[u] * w[u];
  s = lane_sum<64>(s);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) t += ws[w];
    x[blockIdx.x] = t;
  }
}

// Setup: in-place Gauss-Jordan inversion of the dense SPD coarsest matrix M (row-major), one pivot k
// per pair of launches.  Without pivoting: the pivots of an SPD matrix are Schur-complement diagonals,
// all positive; a pivot that is not sets *bad.
//   for i, j != k:  m_ij <- m_ij - m_ik m_kj / p;   m_kj <- m_kj / p;   m_ik <- -m_ik / p;   m_kk <- 1 / p
// with p = m_kk; after the last pivot M holds M^-1.  Row and column k are copied first, so the update
// reads no entry it writes.
__global__ __launch_bounds__(BLOCK) void k_gj_save(int n, int k, const double* __restrict__ M, double* __restrict__ rowk,
                                                   double* __restrict__ colk, int* __restrict__ bad) {
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  rowk[i] = M[(size_t)k * n + i];
  colk[i] = M[(size_t)i * n + k];
  if (i == k && !(M[(size_t)k * n + k] > 0.0)) *bad = 1;
}
__global__ __launch_bounds__(BLOCK) void k_gj_step(int n, int k, double* __restrict__ M, const double* __restrict__ rowk,
                                                   const double* __restrict__ colk) {
  size_t e = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= (size_t)n * n) return;
  int i = (int)(e / n), j = (int)(e % n);
  double p = rowk[k];
  double v;
  if (i == k) v = j == k ? 1.0 / p : rowk[j] / p;
  else if (j == k) v = -colk[i] / p;
  else v = M[e] - colk[i] * rowk[j] / p;
  M[e] = v;
}
// exact symmetry: m_ij and m_ji replaced by their mean
__global__ __launch_bounds__(BLOCK) void k_symmetrise(int n, double* __restrict__ M) {
  size_t e = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= (size_t)n * n) return;
  int i = (int)(e / n), j = (int)(e % n);
  if (j <= i) return;
  double m = 0.5 * (M[e] + M[(size_t)j * n + i]);
  M[e] = m;
  M[(size_t)j * n + i] = m;
}
__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

// M <- M^-1 for the dense SPD coarsest matrix (device, n x n); throws when a pivot is not positive
void dense_inverse_spd(const Ctx& c, int n, double* M, hipStream_t s) {
  double* rc = dalloc<double>(c, 2 * (size_t)n);
  int* bad = dalloc<int>(c, 1);
  int hbad = 0;
  try {
    k_zero_int<<<1, 64, 0, s>>>(bad);
    const int ge = (int)(((size_t)n * n + BLOCK - 1) / BLOCK);
    for (int k = 0; k < n; ++k) {
      k_gj_save<<<grid_for(n), BLOCK, 0, s>>>(n, k, M, rc, rc + n, bad);
      k_gj_step<<<ge, BLOCK, 0, s>>>(n, k, M, rc, rc + n);
    }
    k_symmetrise<<<ge, BLOCK, 0, s>>>(n, M);
    DIFVM_HIP(hipGetLastError());
    DIFVM_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    DIFVM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    dfree(c, rc);
    dfree(c, bad);
    throw;
  }
  dfree(c, rc);
  dfree(c, bad);
  DIFVM_CHECK(!hbad, DIFVM_ERR_UNSUPPORTED, "AMG setup: coarsest matrix is not positive definite");
}

#define DIFVM_AMG_LAUNCH(KERNEL, SW, N, S, ...)                                                           \
  KERNEL<SW><<<(int)(((size_t)(N) * (SW) + BLOCK - 1) / BLOCK), BLOCK, 0, S>>>(__VA_ARGS__)

#define DIFVM_AMG_DISPATCH(KERNEL, sw, N, S, ...)               \
  switch (sw) {                                                 \
    case 1: DIFVM_AMG_LAUNCH(KERNEL, 1, N, S, __VA_ARGS__); break;   \
    case 2: DIFVM_AMG_LAUNCH(KERNEL, 2, N, S, __VA_ARGS__); break;   \
    case 4: DIFVM_AMG_LAUNCH(KERNEL, 4, N, S, __VA_ARGS__); break;   \
    case 8: DIFVM_AMG_LAUNCH(KERNEL, 8, N, S, __VA_ARGS__); break;   \
    case 16: DIFVM_AMG_LAUNCH(KERNEL, 16, N, S, __VA_ARGS__); break; \
    case 32: DIFVM_AMG_LAUNCH(KERNEL, 32, N, S, __VA_ARGS__); break; \
    default: DIFVM_AMG_LAUNCH(KERNEL, 64, N, S, __VA_ARGS__); break; \
  }

}  // namespace

AmgDev* amg_create(difvm_mesh* m, SellMatrix K, const AmgOptions& opt) {
  const DMesh& d = m->d;
  const HostLayout& L = m->host;
  hipStream_t s = stream_of(m);
  std::vector<double> diag(d.nc), val(d.nslot);
  DIFVM_HIP(hipMemcpyAsync(diag.data(), K.diag, sizeof(double) * d.nc, hipMemcpyDeviceToHost, s));
  DIFVM_HIP(hipMemcpyAsync(val.data(), K.val, sizeof(double) * d.nslot, hipMemcpyDeviceToHost, s));
  DIFVM_HIP(hipStreamSynchronize(s));
  // cell-slot rows -> CSR (internal faces only; columns ascending)
  AmgCsr A0;
  A0.n = d.nc;
  A0.ptr.assign(d.nc + 1, 0);
  A0.diag = diag;
  std::vector<std::pair<int32_t, double>> row;
  for (int i = 0; i < d.nc; ++i) {
    int sl = i >> 6, base = L.slice_start[sl] + (i & (SLICE - 1));
    int width = (L.slice_start[sl + 1] - L.slice_start[sl]) >> 6;
    row.clear();
    for (int k = 0; k < width; ++k) {
      int at = base + k * SLICE;
      int sf = L.slot_face[at];
      if (sf == SLOT_PAD || sf >= d.nfi) continue;
      row.push_back({L.slot_col[at], val[at]});
    }
    std::sort(row.begin(), row.end());
    for (auto& e : row) {
      A0.col.push_back(e.first);
      A0.val.push_back(e.second);
    }
    A0.ptr[i + 1] = (int32_t)A0.col.size();
  }
  for (int i = 0; i < d.nc; ++i)
    DIFVM_CHECK(diag[i] > 0.0, DIFVM_ERR_INVALID_ARG, "AMG needs a matrix with a positive diagonal");
  AmgHierarchy H;
  try {
    amg_build(A0, opt, H);
  } catch (const AmgError& e) {
    throw Error{DIFVM_ERR_UNSUPPORTED, "AMG setup: " + e.msg};
  }
  AmgDev* a = new AmgDev();
  try {
    a->mesh = m;
    a->L = (int)H.levels.size();
    int L_ = a->L;
    a->A.resize(L_ + 1);
    a->R.resize(L_);
    a->AP.resize(L_);
    a->b.assign(L_ + 1, nullptr);
    a->bd.assign(L_ + 1, nullptr);
    a->res.assign(L_ + 1, nullptr);
    a->x.assign(L_ + 1, nullptr);
    a->rows.push_back(d.nc);
    a->P0 = upload_csr(a, H.levels[0].P, false, s);
    for (int l = 0; l < L_; ++l) {
      if (l > 0) {
        a->AP[l] = upload_csr(a, H.levels[l].AP, false, s, 1);
        a->AP[l].val2 = up(a, H.levels[l].P_on_AP, s);
      }
      a->R[l] = upload_csr(a, H.levels[l].R, false, s);
      a->A[l + 1] = upload_csr(a, H.coarse[l], true, s);
      a->rows.push_back(H.coarse[l].n);
    }
    // Gershgorin: the eigenvalues of D^-1 K lie in the discs around 1 of radius sum_j |k_ij| / k_ii.
    // At least 2, the bound of every weakly diagonally dominant K (the pressure operators), so that it
    // holds for the later operators of the same kind the preconditioner is applied with.
    double g = 2.0;
    for (int i = 0; i < d.nc; ++i) {
      double off = 0.0;
      for (int q = A0.ptr[i]; q < A0.ptr[i + 1]; ++q) off += std::fabs(A0.val[q]);
      g = std::max(g, 1.0 + off / diag[i]);
    }
    a->hi.push_back(g);
    for (int l = 1; l < L_; ++l) a->hi.push_back(H.levels[l].hi);
    for (int l = 0; l <= L_; ++l) {
      size_t n = a->rows[l];
      a->res[l] = work(a, n);
      if (l < L_) {
        a->xs.push_back(work(a, n));
        a->t.push_back(work(a, n));
        a->d0.push_back(work(a, n));
      }
      if (l > 0) {
        a->b[l] = work(a, n);
        a->x[l] = work(a, n);
        if (l < L_) a->bd[l] = work(a, n);
      }
    }
    DIFVM_CHECK(H.n_coarsest <= MAX_DENSE, DIFVM_ERR_UNSUPPORTED, "coarsest AMG level too large");
    a->cinv = up(a, H.coarsest_dense, s);
    dense_inverse_spd(ctx_of(m), H.n_coarsest, a->cinv, s);
    DIFVM_HIP(hipStreamSynchronize(s));
  } catch (...) {
    amg_free(a);
    throw;
  }
  return a;
}

void amg_free(AmgDev* a) {
  if (!a) return;
  if (a->mesh) (void)hipStreamSynchronize(stream_of(a->mesh));
  for (void* p : a->allocs) dfree(ctx_of(a->mesh), p);
  delete a;
}

int amg_levels(const AmgDev* a, int* rows, int cap) {
  int n = (int)a->rows.size();
  for (int l = 0; l < n && l < cap; ++l) rows[l] = a->rows[l];
  return n;
}

double amg_vcycle_bytes(const AmgDev* a) {
  const difvm_mesh* m = a->mesh;
  const int L = a->L;
  auto rows = [&](int l) { return (double)a->rows[l]; };
  auto csr = [](const DevCsr& M, bool diag, int val_words) {
    return 4.0 * (M.n + 1) + (4.0 + 8.0 * val_words) * M.nnz + (diag ? 8.0 * M.n : 0.0);
  };
  const double n0 = m->d.nc;
  const double K = 8.0 * n0 + 16.0 * m->d.nfi;  // LDU: diagonal; owner, neighbour, coefficient per face
  double b = 0.0;
  b += K + 16.0 * n0;  // first pre-smoothing pass: r -> xs
  b += K + 24.0 * n0;  // second: r, xs -> res
  for (int l = 0; l < L; ++l) {
    if (l > 0) {
      b += csr(a->A[l], true, 1) + 16.0 * rows(l);  // bd -> xs
      b += csr(a->A[l], true, 1) + 24.0 * rows(l);  // b, xs -> res
    }
    bool coarsest = l + 1 == L;
    b += csr(a->R[l], false, 1) + 8.0 * rows(l) + (coarsest ? 8.0 : 24.0) * rows(l + 1);  // res -> b (, D^-1 b)
  }
  b += 8.0 * rows(L) * rows(L) + 16.0 * rows(L);  // dense solve
  for (int l = L - 1; l >= 1; --l) {
    b += csr(a->AP[l], true, 2) + 32.0 * rows(l) + 8.0 * rows(l + 1);  // xs, res, x_c -> t, d0
    b += csr(a->A[l], true, 1) + 24.0 * rows(l);                       // t, d0 -> x
  }
  b += csr(a->P0, false, 1) + 16.0 * n0 + 8.0 * rows(1);  // xs, x_1 -> t
  b += K + 24.0 * n0;                                     // r, t -> d0
  b += K + 32.0 * n0;                                     // r, t, d0 -> z
  return b;
}

static void launch_vcycle(const AmgDev* a, hipStream_t s, SellMatrix Km, const double* r, double* z, double* part,
                          StopFlags ctl) {
  difvm_mesh* m = a->mesh;
  SellView K = sview(m, Km);
  const int L = a->L, nc = m->d.nc;
  std::vector<Cheb> c(L);
  for (int l = 0; l < L; ++l) c[l] = cheb_coefficients(0.1 * a->hi[l], a->hi[l]);
  // down
  if (K.off16) {
    k_amg_cheb_pre1<true><<<grid_for(nc), BLOCK, 0, s>>>(K, r, a->xs[0], c[0], ctl);
    k_amg_cheb_pre2<true><<<grid_for(nc), BLOCK, 0, s>>>(K, r, a->xs[0], a->res[0], ctl);
  } else {
    k_amg_cheb_pre1<false><<<grid_for(nc), BLOCK, 0, s>>>(K, r, a->xs[0], c[0], ctl);
    k_amg_cheb_pre2<false><<<grid_for(nc), BLOCK, 0, s>>>(K, r, a->xs[0], a->res[0], ctl);
  }
  for (int l = 0; l < L; ++l) {
    if (l > 0) {
      const DevCsr& A = a->A[l];
      DIFVM_AMG_DISPATCH(k_amg_cpre1, A.sw, A.n, s, A.n, A.ptr, A.col, A.val, A.diag, a->bd[l], a->xs[l], c[l], ctl);
      DIFVM_AMG_DISPATCH(k_amg_cpre2, A.sw, A.n, s, A.n, A.ptr, A.col, A.val, A.diag, a->b[l], a->xs[l], a->res[l],
                         ctl);
    }
    const DevCsr& R = a->R[l];
    const double* dc = l + 1 < L ? a->A[l + 1].diag : nullptr;  // the coarsest level needs no D^-1 b
    DIFVM_AMG_DISPATCH(k_amg_restrict, R.sw, R.n, s, R.n, R.ptr, R.col, R.val, a->res[l], dc, a->b[l + 1],
                       a->bd[l + 1], ctl);
  }
  k_amg_coarsest<<<a->rows[L], BLOCK, 0, s>>>(a->rows[L], a->cinv, a->b[L], a->x[L], ctl);
  // up
  for (int l = L - 1; l >= 1; --l) {
    const DevCsr& Q = a->AP[l];
    const DevCsr& A = a->A[l];
    DIFVM_AMG_DISPATCH(k_amg_cup1, Q.sw, Q.n, s, Q.n, Q.ptr, Q.col, Q.val, Q.val2, A.diag, a->xs[l], a->res[l],
                       a->x[l + 1], a->t[l], a->d0[l], c[l], ctl);
    DIFVM_AMG_DISPATCH(k_amg_cup2, A.sw, A.n, s, A.n, A.ptr, A.col, A.val, A.diag, a->t[l], a->d0[l], a->x[l], c[l],
                       ctl);
  }
  {
    const DevCsr& P = a->P0;
    k_amg_prolong<<<grid_for(P.n), BLOCK, 0, s>>>(P.n, P.ptr, P.col, P.val, a->xs[0], a->x[1], a->t[0], ctl);
  }
  Tiles T = tiles_of(m);
  if (K.off16) {
    k_amg_cheb_post1<true><<<grid_for(nc), BLOCK, 0, s>>>(K, r, a->t[0], a->d0[0], c[0], ctl);
    k_amg_cheb_post2<true><<<T.ntile, POST2_NT, 0, s>>>(K, T, r, a->t[0], a->d0[0], z, part, c[0], ctl);
  } else {
    k_amg_cheb_post1<false><<<grid_for(nc), BLOCK, 0, s>>>(K, r, a->t[0], a->d0[0], c[0], ctl);
    k_amg_cheb_post2<false><<<T.ntile, POST2_NT, 0, s>>>(K, T, r, a->t[0], a->d0[0], z, part, c[0], ctl);
  }
  DIFVM_HIP(hipGetLastError());
}

void amg_vcycle(const AmgDev* a, SellMatrix Km, const double* r, double* z, double* part, const PcgCtl* ctls) {
  difvm_mesh* m = a->mesh;
  // queued kernel by kernel on the solve's stream (inside a captured step they join that graph): the
  // host queues a cycle in well under one iteration's GPU time, and a replayed graph of the cycle
  // cost about 9 us of idle GPU between its end and the next kernel on the stream
  launch_vcycle(a, ctx_of(m).stream, Km, r, z, part, StopFlags{ctls, m->d.nseg});
}

}  // namespace difvm
