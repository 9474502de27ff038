// Krylov solvers of libdifvm on the cell-slot matrix: Jacobi-preconditioned CG (pressure) and
// right-Jacobi BiCGStab (momentum, up to three systems sharing one matrix).  Paper Sec. "Numerical
// schemes and linear solvers": CG for the symmetric pressure system, BiCGStab for momentum.
//
// Every dot product is reduced deterministically (fixed 256-cell tiles, the last tile to finish sums
// the tile partials in a fixed order).  The scalars live in device memory and every kernel checks
// the solver's "active" flag first, so iterations queued after convergence are no-ops and the
// iterate is exactly the one at which the stopping test first held; the host reads the flag only
// once per block of iterations.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "device.h"
#include "ops.h"

namespace difvm {


struct PcgCtl;

struct BiState {
  double tol;
  double bn[3], rho[3], rho1[3], alpha[3], omega[3], beta[3], res[3];
  int maxit, any;
  int iters[3], active[3], phase[3], status[3], zero_b[3];
};

struct KrylovWork {
  int nc = 0, ntile = 0;
  double *r = nullptr, *p = nullptr, *q = nullptr, *rh = nullptr, *v = nullptr, *y = nullptr, *s = nullptr,
         *z = nullptr, *t = nullptr;
  double* partials = nullptr;
  struct PcgCtl* pcg = nullptr;
  BiState* bi = nullptr;
  int* host_flag = nullptr;  // pinned
  void* host_state = nullptr;  // pinned, sizeof(BiState)
  int pcg_hint = 0, bi_hint = 0;  // iterations of the previous solve: sizes the first unpolled block
};

KrylovWork* krylov_work(difvm_mesh* m) { return m->krylov; }

static KrylovWork* make_work(difvm_mesh* m) {
  if (m->krylov) return m->krylov;
  KrylovWork* w = new KrylovWork();
  m->krylov = w;
  int nc = m->d.nc;
  w->nc = nc;
  w->ntile = grid_for(nc);
  size_t n3 = (size_t)nc * 3;
  w->r = dalloc<double>(n3); w->p = dalloc<double>(n3); w->q = dalloc<double>(n3); w->rh = dalloc<double>(n3);
  w->v = dalloc<double>(n3); w->y = dalloc<double>(n3); w->s = dalloc<double>(n3); w->z = dalloc<double>(n3);
  w->t = dalloc<double>(n3);
  w->partials = dalloc<double>((size_t)8 * w->ntile);  // >= 8 * ceil(nc/1024) for PCG
  w->pcg = static_cast<PcgCtl*>(dmalloc(128));
  w->bi = dalloc<BiState>(1);
  DIFVM_HIP(hipHostMalloc((void**)&w->host_flag, sizeof(int), hipHostMallocDefault));
  DIFVM_HIP(hipHostMalloc((void**)&w->host_state, sizeof(BiState), hipHostMallocDefault));
  return w;
}

void krylov_work_free(KrylovWork* w) {
  if (!w) return;
  for (double* a : {w->r, w->p, w->q, w->rh, w->v, w->y, w->s, w->z, w->t, w->partials}) dfree(a);
  dfree(w->pcg);
  dfree(w->bi);
  if (w->host_flag) (void)hipHostFree(w->host_flag);
  if (w->host_state) (void)hipHostFree(w->host_state);
  delete w;
}

// ---------------------------------------------------------------------------------------------
// matrix helpers
// ---------------------------------------------------------------------------------------------
struct SellView {
  int nc;
  const int32_t* __restrict__ slice_start;
  const int32_t* __restrict__ col;
  const double* __restrict__ val;
  const double* __restrict__ diag;
};

static SellView sview(const difvm_mesh* m, SellMatrix A) {
  return {m->d.nc, m->d.slice_start, m->d.slot_col, A.val, A.diag};
}

// (A x)_i for NC interleaved components; padding and boundary slots carry val = 0, col = i
template <int NC>
__device__ __forceinline__ void sell_row(const SellView& A, int i, const double* __restrict__ x, double (&acc)[NC]) {
  SlotRange R = slots_of(A.slice_start, i);
  double di = A.diag[i];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = di * x[(size_t)i * NC + c];
#pragma unroll 4
  for (int k = 0; k < R.width; ++k) {
    int at = R.base + k * SLICE;
    double a = A.val[at];
    int j = A.col[at];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += a * x[(size_t)j * NC + c];
  }
}

__global__ __launch_bounds__(BLOCK) void k_sell_from_ldu(int nc, int nfi, const int32_t* __restrict__ slice_start,
                                                         const int32_t* __restrict__ slot_face, const double* __restrict__ up,
                                                         const double* __restrict__ lo, double* __restrict__ val) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= nc) return;
  SlotRange R = slots_of(slice_start, i);
  for (int k = 0; k < R.width; ++k) {
    int at = R.base + k * SLICE;
    int sf = slot_face[at];
    double a = 0.0;
    if (sf != SLOT_PAD && sf < nfi) a = sf < 0 ? lo[-sf - 1] : up[sf];
    val[at] = a;
  }
}

template <int NC>
__global__ __launch_bounds__(BLOCK) void k_sell_spmv(SellView A, const double* __restrict__ x, double* __restrict__ y) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= A.nc) return;
  double acc[NC];
  sell_row<NC>(A, i, x, acc);
#pragma unroll
  for (int c = 0; c < NC; ++c) y[(size_t)i * NC + c] = acc[c];
}

void sell_from_ldu(const difvm_mesh* m, const double* upper, const double* lower, double* val) {
  const DMesh& d = m->d;
  // padding rows of the last slice are never read by row kernels; clear the whole array once so no
  // slot holds stale values
  DIFVM_HIP(hipMemsetAsync(val, 0, sizeof(double) * (size_t)d.nslot, stream_of(m)));
  k_sell_from_ldu<<<grid_for(d.nc), BLOCK, 0, stream_of(m)>>>(d.nc, d.nfi, d.slice_start, d.slot_face, upper,
                                                              lower ? lower : upper, val);
  DIFVM_HIP(hipGetLastError());
}

void sell_spmv(const difvm_mesh* m, int ncomp, SellMatrix A, const double* x, double* y) {
  SellView v = sview(m, A);
  if (ncomp == 1) k_sell_spmv<1><<<grid_for(v.nc), BLOCK, 0, stream_of(m)>>>(v, x, y);
  else k_sell_spmv<3><<<grid_for(v.nc), BLOCK, 0, stream_of(m)>>>(v, x, y);
  DIFVM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------------------------
// PCG: two kernels per iteration and no memory fences.
//
// Dot products are summed per 1024-cell tile into partial arrays; the NEXT kernel re-sums an array
// in a fixed order in every block (all blocks obtain the same bits), so no tile waits for another
// and no L2 write-back is needed.  The direction update p_k = z_{k-1} + beta p_{k-1} is fused into
// the product q = A p_k: each cell forms its own and its neighbours' p_k from the interleaved pair
// (z, p) of the previous iteration, one 16-byte gather per matrix slot.  (z, p) pairs are
// double-buffered by iteration parity, and so are the published scalars rho_k = r_k.z_k.
//   init1:  r = b - A x                               partials (b.b, r.r)
//   init2:  stopping test at k = 0; z0 = r/d          partials B = (r.r, r.z)
//   spmv_k: rho_{k-1} and the stopping test of iterate k-1 (from B), beta; p_k; q = A p_k
//                                                     partials A = (p.q); tile 0 publishes rho_{k-1}
//   upd_k:  alpha = rho_{k-1}/(p.q); x += alpha p; r -= alpha q; z = r/d   partials B
// Tile 0 records iterations / residual / status; kernels after the stop return at once.
// ---------------------------------------------------------------------------------------------
constexpr int PCG_TILE = 1024;             // cells per reduction partial
constexpr int PCG_CPT = PCG_TILE / BLOCK;  // cells per thread

struct PcgCtl {
  double tol, bn, res;
  double rho[2];  // rho_k at index k & 1, published by tile 0 of spmv_{k+1}
  int maxit, done, iters, status;
};

// one read of a flag per block, shared through LDS, so every wave of the block takes the same branch
// even while tile 0 of the same launch may be writing it
__device__ __forceinline__ bool block_flag(const int* flag) {
  __shared__ int f;
  if (threadIdx.x == 0) f = *flag;
  __syncthreads();
  return f != 0;
}

// fixed-order sum of G partials (NV arrays, value-major) -> identical result in every block
template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int G, double (&out)[NV]) {
  __shared__ double lds[NV][BLOCK / 64];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int q = threadIdx.x; q < G; q += BLOCK) s += part[(size_t)k * G + q];
    out[k] = s;
  }
  block_sum<NV>(out, lds);
}

template <int NV>
__device__ __forceinline__ void write_partial(double (&v)[NV], double* __restrict__ part, int G, int tile) {
  __shared__ double lds[NV][BLOCK / 64];
  block_sum<NV>(v, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) part[(size_t)k * G + tile] = v[k];
}

// slice start of the wave's 64 cells, read once per wave through the scalar unit
__device__ __forceinline__ SlotRange wave_slots(const int32_t* __restrict__ slice_start, int i) {
  int s = __builtin_amdgcn_readfirstlane(i >> 6);
  int b = slice_start[s];
  int e = slice_start[s + 1];
  return {b + (i & (SLICE - 1)), (e - b) >> 6};
}

__global__ __launch_bounds__(BLOCK) void k_pcg_init1(SellView A, const double* __restrict__ b, const double* __restrict__ x,
                                                     double* __restrict__ r, double* __restrict__ part) {
  int G = gridDim.x, tile = xcd_tile(blockIdx.x, G);
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int c = 0; c < PCG_CPT; ++c) {
    int i = tile * PCG_TILE + c * BLOCK + threadIdx.x;
    if (i < A.nc) {
      double ax[1];
      sell_row<1>(A, i, x, ax);
      double bi = b[i], ri = bi - ax[0];
      r[i] = ri;
      v[0] += bi * bi;
      v[1] += ri * ri;
    }
  }
  write_partial<2>(v, part, G, tile);
}

__global__ __launch_bounds__(BLOCK) void k_pcg_init2(SellView A, double* __restrict__ x, const double* __restrict__ r,
                                                     double2* __restrict__ zp0, const double* __restrict__ part_in,
                                                     double* __restrict__ partB, PcgCtl* ctl) {
  int G = gridDim.x, tile = xcd_tile(blockIdx.x, G);
  double s[2];
  sum_partials<2>(part_in, G, s);
  double bn = sqrt(s[0]), rn = sqrt(s[1]);
  bool zero_b = bn == 0.0;
  bool stop = zero_b || rn <= ctl->tol * bn;
  if (tile == 0 && threadIdx.x == 0) {
    ctl->bn = bn;
    ctl->res = zero_b ? 0.0 : rn / bn;
    ctl->iters = 0;
    ctl->status = 0;
    ctl->done = stop ? 1 : 0;
  }
  if (zero_b) {
#pragma unroll
    for (int c = 0; c < PCG_CPT; ++c) {
      int i = tile * PCG_TILE + c * BLOCK + threadIdx.x;
      if (i < A.nc) x[i] = 0.0;
    }
  }
  if (stop) return;
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int c = 0; c < PCG_CPT; ++c) {
    int i = tile * PCG_TILE + c * BLOCK + threadIdx.x;
    if (i < A.nc) {
      double ri = r[i], zi = ri / A.diag[i];
      zp0[i] = make_double2(zi, 0.0);  // p_0 = 0 so that p_1 = z_0 + 0 * p_0
      v[0] += ri * ri;
      v[1] += ri * zi;
    }
  }
  write_partial<2>(v, partB, G, tile);
}

// iteration k >= 1: stopping test of iterate k-1, then p_k and q = A p_k
__global__ __launch_bounds__(BLOCK) void k_pcg_spmv(SellView A, int k, const double2* __restrict__ zp_prev,
                                                    double2* __restrict__ zp_cur, double* __restrict__ q,
                                                    const double* __restrict__ partB, double* __restrict__ partA,
                                                    PcgCtl* ctl) {
  if (block_flag(&ctl->done)) return;
  int G = gridDim.x, tile = xcd_tile(blockIdx.x, G);
  double s2[2];
  sum_partials<2>(partB, G, s2);  // (r_{k-1}.r_{k-1}, r_{k-1}.z_{k-1})
  double rho = s2[1];
  if (tile == 0 && threadIdx.x == 0) ctl->rho[(k - 1) & 1] = rho;
  double beta = 0.0;
  if (k >= 2) {
    double rn = sqrt(s2[0]), bn = ctl->bn;
    bool conv = rn <= ctl->tol * bn;
    if (conv || k - 1 >= ctl->maxit) {
      if (tile == 0 && threadIdx.x == 0) {
        ctl->done = 1;
        ctl->iters = k - 1;
        ctl->res = rn / bn;
        ctl->status = conv ? 0 : DIFVM_WARN_NOT_CONVERGED;
      }
      return;
    }
    beta = rho / ctl->rho[k & 1];  // rho_{k-1} / rho_{k-2}
  } else if (ctl->maxit <= 0) {
    if (tile == 0 && threadIdx.x == 0) {
      ctl->done = 1;
      ctl->status = DIFVM_WARN_NOT_CONVERGED;
    }
    return;
  }
  double v[1] = {0.0};
#pragma unroll
  for (int c = 0; c < PCG_CPT; ++c) {
    int i = tile * PCG_TILE + c * BLOCK + threadIdx.x;
    if (i < A.nc) {
      double2 zpi = zp_prev[i];
      double pi = zpi.x + beta * zpi.y;
      SlotRange R = wave_slots(A.slice_start, i);
      double acc = A.diag[i] * pi;
#pragma unroll 4
      for (int s = 0; s < R.width; ++s) {
        int at = R.base + s * SLICE;
        double2 zpj = zp_prev[A.col[at]];
        acc += A.val[at] * (zpj.x + beta * zpj.y);
      }
      zp_cur[i].y = pi;
      q[i] = acc;
      v[0] += pi * acc;
    }
  }
  write_partial<1>(v, partA, G, tile);
}

// iteration k: alpha, x and r updates, z = r/d, partials of r.r and r.z (loads issued before the
// partial sum, as above)
__global__ __launch_bounds__(BLOCK) void k_pcg_update(SellView A, double* __restrict__ x, double* __restrict__ r,
                                                      double2* __restrict__ zp_cur, const double* __restrict__ q,
                                                      const double* __restrict__ partA, double* __restrict__ partB,
                                                      int k, PcgCtl* ctl) {
  if (block_flag(&ctl->done)) return;
  int G = gridDim.x, tile = xcd_tile(blockIdx.x, G);
  double xv[PCG_CPT], pv[PCG_CPT], rv[PCG_CPT], qv[PCG_CPT], dv[PCG_CPT];
#pragma unroll
  for (int c = 0; c < PCG_CPT; ++c) {
    int i = tile * PCG_TILE + c * BLOCK + threadIdx.x;
    if (i < A.nc) {
      xv[c] = x[i];
      pv[c] = zp_cur[i].y;
      rv[c] = r[i];
      qv[c] = q[i];
      dv[c] = A.diag[i];
    }
  }
  double pq[1];
  sum_partials<1>(partA, G, pq);
  double alpha = ctl->rho[(k - 1) & 1] / pq[0];
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int c = 0; c < PCG_CPT; ++c) {
    int i = tile * PCG_TILE + c * BLOCK + threadIdx.x;
    if (i < A.nc) {
      x[i] = xv[c] + alpha * pv[c];
      double ri = rv[c] - alpha * qv[c];
      double zi = ri / dv[c];
      r[i] = ri;
      zp_cur[i].x = zi;
      v[0] += ri * ri;
      v[1] += ri * zi;
    }
  }
  write_partial<2>(v, partB, G, tile);
}

static int poll_flag(difvm_mesh* m, KrylovWork* w, const int* dflag) {
  DIFVM_HIP(hipMemcpyAsync(w->host_flag, dflag, sizeof(int), hipMemcpyDeviceToHost, stream_of(m)));
  DIFVM_HIP(hipStreamSynchronize(stream_of(m)));
  return *w->host_flag;
}

SolveResult pcg(difvm_mesh* m, SellMatrix A, const double* b, double* x, double tol, int maxit) {
  KrylovWork* w = make_work(m);
  hipStream_t s = stream_of(m);
  SellView V = sview(m, A);
  int G = (V.nc + PCG_TILE - 1) / PCG_TILE;
  PcgCtl* ctl = w->pcg;
  PcgCtl init{};
  init.tol = tol;
  init.maxit = maxit;
  DIFVM_HIP(hipMemcpyAsync(ctl, &init, sizeof(PcgCtl), hipMemcpyHostToDevice, s));
  double* r = w->r;
  double* q = w->q;
  // (z, p) pairs, two parities: 2 * 2 * nc doubles in the p and v buffers (each 3 nc long)
  double2* ZP[2] = {reinterpret_cast<double2*>(w->p), reinterpret_cast<double2*>(w->v)};
  double* partA = w->partials;
  double* partB = w->partials + 2 * (size_t)G;
  double* part0 = w->partials + 4 * (size_t)G;
  k_pcg_init1<<<G, BLOCK, 0, s>>>(V, b, x, r, part0);
  k_pcg_init2<<<G, BLOCK, 0, s>>>(V, x, r, ZP[0], part0, partB, ctl);
  DIFVM_HIP(hipGetLastError());
  // First block sized from the previous solve (iterations are similar from step to step), then
  // short polled blocks; kernels queued after the stop return at once.  Iteration k's stopping
  // test runs at the start of iteration k+1, so the host always queues up to iteration maxit+1.
  int k = 1;
  int nb = std::max(4, w->pcg_hint - 2);
  while (true) {
    int last = std::min(k + nb - 1, maxit + 1);
    for (; k <= last; ++k) {
      {
        ProfScope ps(m, "pcg_spmv_dot");
        k_pcg_spmv<<<G, BLOCK, 0, s>>>(V, k, ZP[(k - 1) & 1], ZP[k & 1], q, partB, partA, ctl);
      }
      if (k > maxit) break;
      {
        ProfScope ps(m, "pcg_update_dot");
        k_pcg_update<<<G, BLOCK, 0, s>>>(V, x, r, ZP[k & 1], q, partA, partB, k, ctl);
      }
    }
    DIFVM_HIP(hipGetLastError());
    if (k > maxit || poll_flag(m, w, &ctl->done)) break;
    nb = 4;
  }
  PcgCtl out;
  DIFVM_HIP(hipMemcpyAsync(w->host_state, ctl, sizeof(PcgCtl), hipMemcpyDeviceToHost, s));
  DIFVM_HIP(hipStreamSynchronize(s));
  std::memcpy(&out, w->host_state, sizeof(PcgCtl));
  if (!out.done) out.status = DIFVM_WARN_NOT_CONVERGED;
  w->pcg_hint = out.iters;
  SolveResult R;
  R.iters[0] = out.iters;
  R.res[0] = out.res;
  R.status = out.status;
  return R;
}

// ---------------------------------------------------------------------------------------------
// BiCGStab kernels (NC systems sharing one matrix, interleaved vectors).  Each reduction kernel
// writes per-tile partials; a one-block finalize kernel sums them in a fixed order and advances the
// scalar recurrences in device memory (the kernel boundary orders everything, no fences).
// ---------------------------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void tile_partials(double (&v)[NV], double* __restrict__ part, int G, int tile) {
  __shared__ double lds[NV][BLOCK / 64];
  block_sum<NV>(v, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) part[(size_t)k * G + tile] = v[k];
}

#define TILE_INDEX() int tile = xcd_tile(blockIdx.x, gridDim.x); int i = tile * BLOCK + threadIdx.x; bool in = i < A.nc

enum BiStage { BI_INIT = 0, BI_ALPHA = 1, BI_S = 2, BI_OMEGA = 3, BI_X = 4 };

template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_fin(int stage, const double* __restrict__ part, int G, BiState* st) {
  if (stage != BI_INIT && !st->any) return;
  constexpr int NV = 2 * NC;
  __shared__ double lds[NV][BLOCK / 64];
  double tot[NV];
  int nv = (stage == BI_ALPHA || stage == BI_S) ? NC : NV;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    if (k < nv)
      for (int q = threadIdx.x; q < G; q += BLOCK) s += part[(size_t)k * G + q];
    tot[k] = s;
  }
  block_sum<NV>(tot, lds);
  if (threadIdx.x != 0) return;
  int any = 0;
  for (int c = 0; c < NC; ++c) {
    if (stage == BI_INIT) {
      double bn = sqrt(tot[c]), rn = sqrt(tot[NC + c]);
      st->bn[c] = bn;
      st->iters[c] = 0;
      st->status[c] = 0;
      st->phase[c] = 0;
      st->zero_b[c] = bn == 0.0;
      st->res[c] = bn == 0.0 ? 0.0 : rn / bn;
      st->active[c] = (bn == 0.0 || rn <= st->tol * bn) ? 0 : 1;
      st->rho[c] = st->alpha[c] = st->omega[c] = 1.0;
      st->rho1[c] = tot[NC + c];  // rhat = r, so rhat.r = r.r
      if (st->active[c] && st->maxit <= 0) {
        st->active[c] = 0;
        st->status[c] = DIFVM_WARN_NOT_CONVERGED;
      } else if (st->active[c] && st->rho1[c] == 0.0) {
        st->active[c] = 0;
        st->status[c] = DIFVM_WARN_BREAKDOWN;
      }
      if (st->active[c]) st->beta[c] = (st->rho1[c] / st->rho[c]) * (st->alpha[c] / st->omega[c]);
    } else if (!st->active[c]) {
      continue;
    } else if (stage == BI_ALPHA) {
      st->alpha[c] = st->rho1[c] / tot[c];
    } else if (stage == BI_S) {
      double sn = sqrt(tot[c]);
      if (sn <= st->tol * st->bn[c]) {
        st->phase[c] = 1;
        st->res[c] = sn / st->bn[c];
      }
    } else if (stage == BI_OMEGA) {
      if (!st->phase[c]) {
        if (tot[NC + c] == 0.0) {
          st->active[c] = 0;
          st->status[c] = DIFVM_WARN_BREAKDOWN;
        } else {
          st->omega[c] = tot[c] / tot[NC + c];
        }
      }
    } else {  // BI_X
      int it = st->iters[c] + 1;
      st->iters[c] = it;
      if (st->phase[c]) {
        st->active[c] = 0;
      } else {
        st->rho[c] = st->rho1[c];
        double rn = sqrt(tot[c]);
        st->res[c] = rn / st->bn[c];
        if (rn <= st->tol * st->bn[c]) {
          st->active[c] = 0;
        } else if (it >= st->maxit) {
          st->active[c] = 0;
          st->status[c] = DIFVM_WARN_NOT_CONVERGED;
        } else {
          st->rho1[c] = tot[NC + c];
          if (st->rho1[c] == 0.0) {
            st->active[c] = 0;
            st->status[c] = DIFVM_WARN_BREAKDOWN;
          } else {
            st->beta[c] = (st->rho1[c] / st->rho[c]) * (st->alpha[c] / st->omega[c]);
          }
        }
      }
    }
    any |= st->active[c];
  }
  st->any = any;
}

template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_init(SellView A, const double* __restrict__ b, const double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ rh, double* __restrict__ p,
                                                   double* __restrict__ v, double* __restrict__ part) {
  TILE_INDEX();
  double acc[2 * NC];
#pragma unroll
  for (int k = 0; k < 2 * NC; ++k) acc[k] = 0.0;
  if (in) {
    double ax[NC];
    sell_row<NC>(A, i, x, ax);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      size_t at = (size_t)i * NC + c;
      double bi = b[at], ri = bi - ax[c];
      r[at] = ri;
      rh[at] = ri;
      p[at] = 0.0;
      v[at] = 0.0;
      acc[c] = bi * bi;
      acc[NC + c] = ri * ri;
    }
  }
  tile_partials<2 * NC>(acc, part, gridDim.x, tile);
}

template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_zero(int nc, double* __restrict__ x, const BiState* st) {
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= nc) return;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (st->zero_b[c]) x[(size_t)i * NC + c] = 0.0;
}

// p = r + beta (p - omega v); y = p / d
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_dir(SellView A, const double* __restrict__ r, double* __restrict__ p,
                                                  const double* __restrict__ v, double* __restrict__ y, const BiState* st) {
  if (!st->any) return;
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= A.nc) return;
  double di = A.diag[i];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (!st->active[c]) continue;
    size_t at = (size_t)i * NC + c;
    double pi = r[at] + st->beta[c] * (p[at] - st->omega[c] * v[at]);
    p[at] = pi;
    y[at] = pi / di;
  }
}

// v = A y; partial rhat . v
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_v(SellView A, const double* __restrict__ y, double* __restrict__ v,
                                                const double* __restrict__ rh, double* __restrict__ part, const BiState* st) {
  if (!st->any) return;
  TILE_INDEX();
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  if (in) {
    double ay[NC];
    sell_row<NC>(A, i, y, ay);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!st->active[c]) continue;
      size_t at = (size_t)i * NC + c;
      v[at] = ay[c];
      acc[c] = rh[at] * ay[c];
    }
  }
  tile_partials<NC>(acc, part, gridDim.x, tile);
}

// s = r - alpha v; z = s / d; partial s.s
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_s(SellView A, const double* __restrict__ r, const double* __restrict__ v,
                                                double* __restrict__ s, double* __restrict__ z, double* __restrict__ part,
                                                const BiState* st) {
  if (!st->any) return;
  TILE_INDEX();
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  if (in) {
    double di = A.diag[i];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!st->active[c]) continue;
      size_t at = (size_t)i * NC + c;
      double si = r[at] - st->alpha[c] * v[at];
      s[at] = si;
      z[at] = si / di;
      acc[c] = si * si;
    }
  }
  tile_partials<NC>(acc, part, gridDim.x, tile);
}

// t = A z; partials t.s, t.t
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_t(SellView A, const double* __restrict__ z, const double* __restrict__ s,
                                                double* __restrict__ t, double* __restrict__ part, const BiState* st) {
  if (!st->any) return;
  TILE_INDEX();
  double acc[2 * NC];
#pragma unroll
  for (int k = 0; k < 2 * NC; ++k) acc[k] = 0.0;
  if (in) {
    double az[NC];
    sell_row<NC>(A, i, z, az);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!st->active[c] || st->phase[c]) continue;
      size_t at = (size_t)i * NC + c;
      t[at] = az[c];
      acc[c] = az[c] * s[at];
      acc[NC + c] = az[c] * az[c];
    }
  }
  tile_partials<2 * NC>(acc, part, gridDim.x, tile);
}

// x += alpha y (+ omega z); r = s - omega t; partials r.r, rhat.r
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_x(SellView A, double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ rh, const double* __restrict__ y,
                                                const double* __restrict__ z, const double* __restrict__ s,
                                                const double* __restrict__ t, double* __restrict__ part, const BiState* st) {
  if (!st->any) return;
  TILE_INDEX();
  double acc[2 * NC];
#pragma unroll
  for (int k = 0; k < 2 * NC; ++k) acc[k] = 0.0;
  if (in) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!st->active[c]) continue;
      size_t at = (size_t)i * NC + c;
      if (st->phase[c]) {
        x[at] += st->alpha[c] * y[at];
      } else {
        x[at] += st->alpha[c] * y[at] + st->omega[c] * z[at];
        double ri = s[at] - st->omega[c] * t[at];
        r[at] = ri;
        acc[c] = ri * ri;
        acc[NC + c] = rh[at] * ri;
      }
    }
  }
  tile_partials<2 * NC>(acc, part, gridDim.x, tile);
}

template <int NC>
static SolveResult bicgstab_nc(difvm_mesh* m, SellMatrix A, const double* b, double* x, double tol, int maxit) {
  KrylovWork* w = make_work(m);
  hipStream_t s = stream_of(m);
  SellView V = sview(m, A);
  int G = grid_for(V.nc);
  BiState init{};
  init.tol = tol;
  init.maxit = maxit;
  DIFVM_HIP(hipMemcpyAsync(w->bi, &init, sizeof(BiState), hipMemcpyHostToDevice, s));
  double* part = w->partials;
  k_bi_init<NC><<<G, BLOCK, 0, s>>>(V, b, x, w->r, w->rh, w->p, w->v, part);
  k_bi_fin<NC><<<1, BLOCK, 0, s>>>(BI_INIT, part, G, w->bi);
  k_bi_zero<NC><<<G, BLOCK, 0, s>>>(V.nc, x, w->bi);
  DIFVM_HIP(hipGetLastError());
  int done = 0;
  int nb = std::min(maxit, std::max(2, w->bi_hint - 1));
  while (nb > 0) {
    for (int k = 0; k < nb; ++k) {
      k_bi_dir<NC><<<G, BLOCK, 0, s>>>(V, w->r, w->p, w->v, w->y, w->bi);
      k_bi_v<NC><<<G, BLOCK, 0, s>>>(V, w->y, w->v, w->rh, part, w->bi);
      k_bi_fin<NC><<<1, BLOCK, 0, s>>>(BI_ALPHA, part, G, w->bi);
      k_bi_s<NC><<<G, BLOCK, 0, s>>>(V, w->r, w->v, w->s, w->z, part, w->bi);
      k_bi_fin<NC><<<1, BLOCK, 0, s>>>(BI_S, part, G, w->bi);
      k_bi_t<NC><<<G, BLOCK, 0, s>>>(V, w->z, w->s, w->t, part, w->bi);
      k_bi_fin<NC><<<1, BLOCK, 0, s>>>(BI_OMEGA, part, G, w->bi);
      k_bi_x<NC><<<G, BLOCK, 0, s>>>(V, x, w->r, w->rh, w->y, w->z, w->s, w->t, part, w->bi);
      k_bi_fin<NC><<<1, BLOCK, 0, s>>>(BI_X, part, G, w->bi);
    }
    DIFVM_HIP(hipGetLastError());
    done += nb;
    if (done >= maxit || !poll_flag(m, w, &w->bi->any)) break;
    nb = std::min(2, maxit - done);
  }
  BiState out;
  DIFVM_HIP(hipMemcpyAsync(w->host_state, w->bi, sizeof(BiState), hipMemcpyDeviceToHost, s));
  DIFVM_HIP(hipStreamSynchronize(s));
  std::memcpy(&out, w->host_state, sizeof(BiState));
  SolveResult R;
  w->bi_hint = 0;
  for (int c = 0; c < NC; ++c) w->bi_hint = std::max(w->bi_hint, out.iters[c]);
  for (int c = 0; c < NC; ++c) {
    R.iters[c] = out.iters[c];
    R.res[c] = out.res[c];
    R.status = std::max(R.status, out.active[c] ? (int)DIFVM_WARN_NOT_CONVERGED : out.status[c]);
  }
  return R;
}

SolveResult bicgstab(difvm_mesh* m, int ncomp, SellMatrix A, const double* b, double* x, double tol, int maxit) {
  if (ncomp == 1) return bicgstab_nc<1>(m, A, b, x, tol, maxit);
  return bicgstab_nc<3>(m, A, b, x, tol, maxit);
}

}  // namespace difvm
