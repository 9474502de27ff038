// Krylov solvers of libdifvm on the cell-slot matrix: Jacobi-preconditioned CG (pressure) and
// right-Jacobi BiCGStab (momentum, up to three systems sharing one matrix).  Paper Sec. "Numerical
// schemes and linear solvers": CG for the symmetric pressure system, BiCGStab for momentum.
//
// Every dot product is reduced deterministically (per-tile partials re-summed in a fixed order by the
// next kernel).  The scalars live in device memory and every kernel checks the solver's "done" flag
// first, so iterations queued after convergence are no-ops and the iterate is exactly the one at
// which the stopping test first held; the host reads the flag only once per block of iterations.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "amg_dev.h"
#include "device.h"
#include "krylov_util.h"
#include "ops.h"

namespace difvm {

// BiCGStab state of one segment (up to three systems sharing its matrix)
struct BiState {
  double tol;
  double bn[3], rho[3], rho1[3], alpha[3], omega[3], beta[3], res[3];
  int maxit, any;
  int iters[3], active[3], phase[3], status[3], zero_b[3];
};

struct KrylovWork {
  int nc = 0, ntile = 0;
  double *r = nullptr, *p = nullptr, *q = nullptr, *rh = nullptr, *v = nullptr, *s = nullptr, *z = nullptr,
         *t = nullptr;
  double* partials = nullptr;
  struct PcgCtl* pcg = nullptr;  // [nseg]
  BiState* bi = nullptr;         // [nseg]
  void* host_state[2] = {nullptr, nullptr};  // pinned mirrors of the solver states (two polls in flight)
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  const Ctx* ctx = nullptr;  // allocator of the buffers above
};

KrylovWork* krylov_work(difvm_mesh* m) { return m->krylov; }

void krylov_work_free(KrylovWork* w);

static KrylovWork* make_work(difvm_mesh* m) {
  if (m->krylov) return m->krylov;
  KrylovWork* w = new KrylovWork();
  try {
    int nc = m->d.nc;
    w->nc = nc;
    w->ntile = m->d.ntile;  // reduction tiles over all segments (at least ceil(nc / 1024))
    size_t n3 = (size_t)nc * 3;
    const Ctx& c = ctx_of(m);
    w->ctx = &c;
    w->r = dalloc<double>(c, n3); w->p = dalloc<double>(c, n3); w->q = dalloc<double>(c, n3);
    w->rh = dalloc<double>(c, n3); w->v = dalloc<double>(c, n3); w->s = dalloc<double>(c, n3);
    w->z = dalloc<double>(c, n3); w->t = dalloc<double>(c, n3);
    w->partials = dalloc<double>(c, (size_t)9 * w->ntile);  // up to 9 values per tile (PCG uses 6, BiCGStab 9)
    int nseg = m->d.nseg;
    w->pcg = static_cast<PcgCtl*>(dmalloc(c, sizeof(BiState) * nseg));  // PcgCtl is smaller (asserted below)
    w->bi = dalloc<BiState>(c, nseg);
    for (int q = 0; q < 2; ++q) {
      DIFVM_HIP(hipHostMalloc((void**)&w->host_state[q], sizeof(BiState) * nseg, hipHostMallocDefault));
      DIFVM_HIP(hipEventCreateWithFlags(&w->poll_ev[q], hipEventDisableTiming));
    }
  } catch (...) {
    krylov_work_free(w);
    throw;
  }
  m->krylov = w;
  return w;
}

void krylov_work_free(KrylovWork* w) {
  if (!w) return;
  if (w->ctx) {
    const Ctx& c = *w->ctx;
    for (double* a : {w->r, w->p, w->q, w->rh, w->v, w->s, w->z, w->t, w->partials}) dfree(c, a);
    dfree(c, w->pcg);
    dfree(c, w->bi);
  }
  for (int q = 0; q < 2; ++q) {
    if (w->host_state[q]) (void)hipHostFree(w->host_state[q]);
    if (w->poll_ev[q]) (void)hipEventDestroy(w->poll_ev[q]);
  }
  delete w;
}

// ---------------------------------------------------------------------------------------------
// matrix helpers (SellView, sell_row: krylov_util.h)
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_sell_from_ldu(int nc, int nfi, const int32_t* __restrict__ slice_start, int uw,
                                                         const int32_t* __restrict__ slot_face, const double* __restrict__ up,
                                                         const double* __restrict__ lo, double* __restrict__ val) {
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= nc) return;
  SlotRange R = slots_of(slice_start, uw, i);
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
  k_sell_from_ldu<<<grid_for(d.nc), BLOCK, 0, stream_of(m)>>>(d.nc, d.nfi, d.slice_start, d.uw, d.slot_face, upper,
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
// Partials of each kernel are re-summed (per segment, fixed order) at the start of the NEXT kernel
// in every block, so no tile waits for another and no L2 write-back is needed.  The direction update
// p_k = z_{k-1} + beta p_{k-1} is fused into the product q = A p_k: each cell forms its own and its
// neighbours' p_k from z and p_{k-1} (separate arrays, so every store writes whole cache lines);
// p and the published rho_k = r_k.z_k are double-buffered by parity.
//   init1:  r = b - A x                               partials (b.b, r.r)
//   init2:  stopping test at k = 0; z0 = r/d; p0 = 0  partials B = (r.r, r.z)
//   spmv_k: rho_{k-1} and the stopping test of iterate k-1 (from B), beta; p_k; q = A p_k
//                                                     partials A = (p.q); first tile publishes rho
//   upd_k:  alpha = rho_{k-1}/(p.q); x += alpha p; r -= alpha q; z = r/d   partials B
// The segment's first tile records iterations / residual / status; its kernels return at once
// after its stop.  The product runs 512 threads x 2 cells per 1024-cell tile, the update 256 x 4
// (measured best on gfx950 for these two memory patterns); the first four slots of a row are
// unrolled so their loads are in flight together.
// ---------------------------------------------------------------------------------------------
static_assert(sizeof(PcgCtl) <= sizeof(BiState), "PCG states share the BiState-sized allocation");

constexpr int PCG_SPMV_NT = 512;  // threads per block of the product kernel (TILE / NT cells each)

__global__ __launch_bounds__(BLOCK) void k_pcg_init1(SellView A, Tiles T, const double* __restrict__ b,
                                                     const double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ part) {
  TileIdx ti = tile_idx(T);
  double v[2] = {0.0, 0.0};
  FOR_TILE_CELLS(i) {
    double ax[1];
    sell_row<1>(A, i, x, ax);
    double bi = b[i], ri = bi - ax[0];
    r[i] = ri;
    v[0] += bi * bi;
    v[1] += ri * ri;
  }
  put_partial<2>(v, part, T.ntile, ti.t);
}

// JAC: Jacobi preconditioner (z = r/d here); otherwise z and the r.z partials come from the V-cycle
// that follows, and this kernel stores only the r.r partials
template <bool JAC>
__global__ __launch_bounds__(BLOCK) void k_pcg_init2(SellView A, Tiles T, double* __restrict__ x, const double* __restrict__ r,
                                                     double* __restrict__ z, double* __restrict__ p0,
                                                     const double* __restrict__ part_in, double* __restrict__ partB,
                                                     PcgCtl* ctls) {
  TileIdx ti = tile_idx(T);
  PcgCtl* ctl = ctls + ti.s;
  double s[2];
  sum_seg<2>(part_in, T, ti.s, s);
  double bn = sqrt(s[0]), rn = sqrt(s[1]);
  bool zero_b = bn == 0.0;
  bool stop = zero_b || rn <= ctl->tol * bn;
  if (ti.t == T.first[ti.s] && threadIdx.x == 0) {
    ctl->bn = bn;
    ctl->res = zero_b ? 0.0 : rn / bn;
    ctl->iters = 0;
    ctl->status = 0;
    ctl->done = stop ? 1 : 0;
  }
  if (zero_b) {
    FOR_TILE_CELLS(i) x[i] = 0.0;
  }
  if (stop) return;
  if constexpr (JAC) {
    double v[2] = {0.0, 0.0};
    FOR_TILE_CELLS(i) {
      double ri = r[i], zi = ri / A.diag[i];
      z[i] = zi;
      p0[i] = 0.0;  // p_1 = z_0 + 0 * p_0
      v[0] += ri * ri;
      v[1] += ri * zi;
    }
    put_partial<2>(v, partB, T.ntile, ti.t);
  } else {
    double v[1] = {0.0};
    FOR_TILE_CELLS(i) {
      double ri = r[i];
      p0[i] = 0.0;
      v[0] += ri * ri;
    }
    put_partial<1>(v, partB, T.ntile, ti.t);
  }
}

// (A (z + beta p))_i with the slot loads of a width-W row issued together
// OFF16: columns read as 16-bit offsets from the row (half the index bytes of the 32-bit columns)
template <int W, bool OFF16>
__device__ __forceinline__ double dir_row(const SellView& A, int i, int base, double acc, double beta,
                                          const double* __restrict__ z, const double* __restrict__ pp) {
  double a[W], zj[W], pj[W];
  int j[W];
#pragma unroll
  for (int sl = 0; sl < W; ++sl) {
    a[sl] = A.val[base + sl * SLICE];
    if constexpr (OFF16) j[sl] = i + A.off16[base + sl * SLICE];
    else j[sl] = A.col[base + sl * SLICE];
  }
#pragma unroll
  for (int sl = 0; sl < W; ++sl) {
    zj[sl] = z[j[sl]];
    pj[sl] = pp[j[sl]];
  }
#pragma unroll
  for (int sl = 0; sl < W; ++sl) acc += a[sl] * (zj[sl] + beta * pj[sl]);
  return acc;
}

// Tiles of this block: one tile per block when the grid has one block per tile (XCD-aware order),
// otherwise (a grid of G < ntile blocks, G a multiple of 8) block b walks tiles lo + b/8, lo + b/8 +
// G/8, ... of the contiguous eighth of the tiles that its XCD (b mod 8) owns.  Which block computes a
// tile does not change the tile's arithmetic or its partial.
struct TileWalk {
  int t, step, end;
};
__device__ __forceinline__ TileWalk tile_walk(int ntile) {
  int b = blockIdx.x, G = gridDim.x;
  if (G >= ntile) {
    int t = xcd_tile(b, G);
    return {t, 1, t + 1};
  }
  int x = b & 7, per = G >> 3;
  int lo = (int)((long long)ntile * x / 8), hi = (int)((long long)ntile * (x + 1) / 8);
  return {lo + (b >> 3), per, hi};
}

// iteration k >= 1: stopping test of iterate k-1, then p_k and q = A p_k
template <bool OFF16>
__global__ __launch_bounds__(PCG_SPMV_NT) void k_pcg_spmv(SellView A, Tiles T, int k, const double* __restrict__ z,
                                                          const double* __restrict__ p_prev, double* __restrict__ p_cur,
                                                          double* __restrict__ q, const double* __restrict__ partB,
                                                          double* __restrict__ partA, PcgCtl* ctls) {
  constexpr int NT = PCG_SPMV_NT, C = TILE / NT;
  TileWalk tw = tile_walk(T.ntile);
  int cur = -1;
  bool skip = true;
  double beta = 0.0;
  for (int t = tw.t; t < tw.end; t += tw.step) {
    const int s = T.seg[t], lo = T.lo[t], hi = T.hi[t];
    if (s != cur) {
      // first tile of segment s for this block: the segment's stopping test and beta.  Every load
      // that needs only s (the flag's included) is issued at once, then the partials', so the block
      // waits for two load latencies before its sum instead of five.
      cur = s;
      PcgCtl* ctl = ctls + s;
      const int f = T.first[s], n = T.count[s], maxit = ctl->maxit, done = ctl->done;
      const double tol = ctl->tol, bn = ctl->bn, rho_older = ctl->rho[k & 1];  // rho_{k-2}
      double s2[2];  // (r_{k-1}.r_{k-1}, r_{k-1}.z_{k-1})
      seg_thread_sum<2, NT>(partB, T.ntile, f, n, s2);
      // thread 0's read decides for the block: the segment's first tile may be setting the flag
      // during this launch
      skip = block_share(done);
      __shared__ double lds[2][NT / 64];
      block_sum<2, NT>(s2, lds);
      if (!skip) {
        bool lead = t == f && threadIdx.x == 0;  // the block holding the segment's first tile
        double rho = s2[1];
        if (lead) ctl->rho[(k - 1) & 1] = rho;
        beta = 0.0;
        if (k >= 2) {
          double rn = sqrt(s2[0]);
          bool conv = rn <= tol * bn;
          if (conv || k - 1 >= maxit) {
            if (lead) {
              ctl->done = 1;
              ctl->iters = k - 1;
              ctl->res = rn / bn;
              ctl->status = conv ? 0 : DIFVM_WARN_NOT_CONVERGED;
            }
            skip = true;
          } else {
            beta = rho / rho_older;  // rho_{k-1} / rho_{k-2}
          }
        } else if (maxit <= 0) {
          if (lead) {
            ctl->done = 1;
            ctl->status = DIFVM_WARN_NOT_CONVERGED;
          }
          skip = true;
        }
      }
    }
    if (skip) continue;
    double v[1] = {0.0};
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int i = lo + c * NT + threadIdx.x;
      if (i < hi) {
        double pi = z[i] + beta * p_prev[i];
        SlotRange R = slots_of(A, i);
        const int nrow = row_len(A, i, R);
        double acc = A.diag[i] * pi;
        walk_row<4>(nrow, [&](auto Wc, int k0) {
          acc = dir_row<decltype(Wc)::value, OFF16>(A, i, R.base + k0 * SLICE, acc, beta, z, p_prev);
        });
        p_cur[i] = pi;
        q[i] = acc;
        v[0] += pi * acc;
      }
    }
    put_partial<1, NT>(v, partA, T.ntile, t);
  }
}

static void launch_pcg_spmv(int G, hipStream_t s, const SellView& V, const Tiles& T, int k, const double* z,
                            const double* p_prev, double* p_cur, double* q, const double* partB, double* partA,
                            PcgCtl* ctls) {
  if (V.off16) k_pcg_spmv<true><<<G, PCG_SPMV_NT, 0, s>>>(V, T, k, z, p_prev, p_cur, q, partB, partA, ctls);
  else k_pcg_spmv<false><<<G, PCG_SPMV_NT, 0, s>>>(V, T, k, z, p_prev, p_cur, q, partB, partA, ctls);
}

// iteration k: alpha, x and r updates, z = r/d, partials of r.r and r.z (streaming loads issued
// before the partial sum so they overlap its latency)
template <bool JAC>
__global__ __launch_bounds__(BLOCK) void k_pcg_update(SellView A, Tiles T, double* __restrict__ x, double* __restrict__ r,
                                                      double* __restrict__ z, const double* __restrict__ p_cur,
                                                      const double* __restrict__ q, const double* __restrict__ partA,
                                                      double* __restrict__ partB, int k, PcgCtl* ctls) {
  TileIdx ti = tile_idx(T);
  PcgCtl* ctl = ctls + ti.s;
  // only earlier launches write the flag, so every wave reads the same value and the block needs
  // no barrier to agree on it
  if (ctl->done) return;
  const int f = T.first[ti.s], n = T.count[ti.s];
  const double rho = ctl->rho[(k - 1) & 1];
  double xv[CPT], pv[CPT], rv[CPT], qv[CPT], dv[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    int i = min(ti.lo + c * BLOCK + (int)threadIdx.x, ti.hi - 1);  // tiles are never empty
    xv[c] = x[i];
    pv[c] = p_cur[i];
    rv[c] = r[i];
    qv[c] = q[i];
    dv[c] = A.diag[i];
  }
  double pq[1];
  seg_thread_sum<1>(partA, T.ntile, f, n, pq);
  __shared__ double lds[1][BLOCK / 64];
  block_sum<1, BLOCK>(pq, lds);
  double alpha = rho / pq[0];
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    int i = ti.lo + c * BLOCK + threadIdx.x;
    if (i < ti.hi) {
      x[i] = xv[c] + alpha * pv[c];
      double ri = rv[c] - alpha * qv[c];
      r[i] = ri;
      v[0] += ri * ri;
      if constexpr (JAC) {
        double zi = ri / dv[c];
        z[i] = zi;
        v[1] += ri * zi;
      }
    }
  }
  if constexpr (JAC) {
    put_partial<2>(v, partB, T.ntile, ti.t);
  } else {
    double v1[1] = {v[0]};
    put_partial<1>(v1, partB, T.ntile, ti.t);
  }
}

// per-segment control state set on the device (no host buffer, so the launch can be captured)
__global__ void k_pcg_ctl_init(PcgCtl* ctls, int nseg, double tol, int maxit) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nseg) return;
  PcgCtl c{};
  c.tol = tol;
  c.maxit = maxit;
  ctls[g] = c;
}

// copies n doubles (solver states are made of doubles and ints, 8-byte multiples)
__global__ void k_copy_words(double* __restrict__ dst, const double* __restrict__ src, int n) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = src[q];
}
static void copy_state(void* dst, const void* src, size_t bytes, hipStream_t s) {
  int n = (int)(bytes / sizeof(double));
  k_copy_words<<<(n + 255) / 256, 256, 0, s>>>(static_cast<double*>(dst), static_cast<const double*>(src), n);
  DIFVM_HIP(hipGetLastError());
}

size_t pcg_state_bytes(const difvm_mesh* m) { return sizeof(PcgCtl) * m->d.nseg; }

// grid of the product kernel: one block per tile, or the tuned persistent grid (a multiple of 8)
int pcg_spmv_grid(const difvm_mesh* m) {
  int nt = m->d.ntile, g = m->tune[DIFVM_TUNE_PCG_GRID];
  if (g <= 0 || g >= nt) return nt;
  return std::max(8, g & ~7);
}

SolveResult pcg_result(const difvm_mesh* m, const void* host_state, bool* complete) {
  const PcgCtl* hs = static_cast<const PcgCtl*>(host_state);
  int nseg = m->d.nseg;
  SolveResult R;
  R.seg.resize(nseg);
  bool all = true;
  for (int g = 0; g < nseg; ++g) {
    const PcgCtl& c = hs[g];
    all = all && c.done;
    int st = c.done ? c.status : (int)DIFVM_WARN_NOT_CONVERGED;
    R.seg[g] = {{c.iters, 0, 0}, {c.res, 0, 0}, st};
    R.iters[0] = std::max(R.iters[0], c.iters);
    R.res[0] = std::max(R.res[0], c.res);
    R.status = std::max(R.status, st);
  }
  if (complete) *complete = all;
  return R;
}

// Polling without draining the queue: the host copies the per-segment states into one of two pinned
// buffers after a block of iterations and records an event, queues the next block, and only then
// waits for the earlier copy; iterations queued past a segment's stop are predicated no-ops, so the
// extra block changes nothing.
static void post_poll(difvm_mesh* m, KrylovWork* w, const void* dstate, size_t bytes, int slot) {
  hipStream_t s = stream_of(m);
  DIFVM_HIP(hipMemcpyAsync(w->host_state[slot], dstate, bytes, hipMemcpyDeviceToHost, s));
  DIFVM_HIP(hipEventRecord(w->poll_ev[slot], s));
}
static const void* wait_poll(KrylovWork* w, int slot) {
  DIFVM_HIP(hipEventSynchronize(w->poll_ev[slot]));
  return w->host_state[slot];
}

SolveResult pcg(difvm_mesh* m, SellMatrix A, const double* b, double* x, double tol, int maxit, const QueueOnly* qo,
                const AmgDev* amg, int* hint) {
  KrylovWork* w = make_work(m);
  hipStream_t s = stream_of(m);
  SellView V = sview(m, A);
  Tiles T = tiles_of(m);
  int G = T.ntile, nseg = m->d.nseg;
  const size_t prof_mark = ctx_of(m).prof.pending.size();  // timed launches of this solve start here
  k_pcg_ctl_init<<<(nseg + 63) / 64, 64, 0, s>>>(w->pcg, nseg, tol, maxit);
  const int GS = pcg_spmv_grid(m);
  double* r = w->r;
  double* q = w->q;
  double* z = w->z;
  double* Pk[2] = {w->p, w->v};  // p_k at parity k & 1
  double* partA = w->partials;
  double* partB = w->partials + 2 * (size_t)G;
  double* part0 = w->partials + 4 * (size_t)G;
  // z = M^-1 r: Jacobi inside the init / update kernels, or one V-cycle after them (which also stores
  // the r.z partials)
  // (the V-cycle's kernels skip their work once every segment has stopped; while some segment runs
  // on they compute for all, which changes nothing a stopped segment reads)
  auto precondition = [&](int kk) {
    if (!amg) return;
    ProfScope ps(m, "pcg_amg_vcycle", kk);
    amg_vcycle(amg, A, r, z, partB + G, w->pcg);
  };
  k_pcg_init1<<<G, BLOCK, 0, s>>>(V, T, b, x, r, part0);
  if (amg) k_pcg_init2<false><<<G, BLOCK, 0, s>>>(V, T, x, r, z, Pk[0], part0, partB, w->pcg);
  else k_pcg_init2<true><<<G, BLOCK, 0, s>>>(V, T, x, r, z, Pk[0], part0, partB, w->pcg);
  DIFVM_HIP(hipGetLastError());
  precondition(0);
  auto update = [&](int kk) {
    {
      ProfScope ps(m, "pcg_update_dot", kk);
      if (amg) k_pcg_update<false><<<G, BLOCK, 0, s>>>(V, T, x, r, z, Pk[kk & 1], q, partA, partB, kk, w->pcg);
      else k_pcg_update<true><<<G, BLOCK, 0, s>>>(V, T, x, r, z, Pk[kk & 1], q, partA, partB, kk, w->pcg);
    }
    precondition(kk);
  };
  if (qo) {
    // queue-only: iterations 1..K and the stopping test of iterate K, no read-back
    int K = std::min(qo->budget, maxit);
    for (int kk = 1; kk <= K + 1; ++kk) {
      {
        ProfScope ps(m, "pcg_spmv_dot", kk);
        launch_pcg_spmv(GS, s, V, T, kk, z, Pk[(kk - 1) & 1], Pk[kk & 1], q, partB, partA, w->pcg);
      }
      if (kk <= K) update(kk);
    }
    DIFVM_HIP(hipGetLastError());
    copy_state(qo->state_out, w->pcg, pcg_state_bytes(m), s);
    return SolveResult{};
  }
  // First block sized from the previous solve, then blocks of one iteration, each queued before the
  // host waits for the state copied after the block before it (an iteration's GPU time covers the
  // host's queueing of the next block); iterations queued past the stop are idle launches, one or two
  // per solve.  Iteration k's stopping test runs at the start of iteration k+1, so the host
  // queues up to iteration maxit+1.
  int k = 1;  // next iteration to queue
  auto queue_block = [&](int nb) {
    for (int n = 0; n < nb && k <= maxit + 1; ++n, ++k) {
      {
        ProfScope ps(m, "pcg_spmv_dot", k);
        launch_pcg_spmv(GS, s, V, T, k, z, Pk[(k - 1) & 1], Pk[k & 1], q, partB, partA, w->pcg);
      }
      if (k <= maxit) update(k);
    }
    DIFVM_HIP(hipGetLastError());
  };
  const size_t bytes = pcg_state_bytes(m);
  queue_block(std::max(4, (hint ? *hint : 0) - 2));
  int slot = 0;
  post_poll(m, w, w->pcg, bytes, slot);
  const PcgCtl* hs = nullptr;
  while (true) {
    bool more = k <= maxit + 1;
    if (more) {
      queue_block(1);
      post_poll(m, w, w->pcg, bytes, slot ^ 1);
    }
    hs = static_cast<const PcgCtl*>(wait_poll(w, slot));
    bool all = true;
    for (int g = 0; g < nseg; ++g) all = all && hs[g].done;
    if (all || !more) break;
    slot ^= 1;
  }
  SolveResult R = pcg_result(m, hs, nullptr);
  // iteration k's kernels ran while some segment had not stopped, i.e. for k <= the largest count
  prof_idle_after(ctx_of(m), prof_mark, R.iters[0]);  // iters[0]: the largest over the segments
  if (hint) *hint = R.iters[0];
  return R;
}

// ---------------------------------------------------------------------------------------------
// BiCGStab kernels (NC systems sharing one matrix per segment, interleaved vectors).  Each reduction
// kernel writes per-tile partials; a finalize kernel (one block per segment) sums them in a fixed
// order and advances the segment's scalar recurrences in device memory.
// ---------------------------------------------------------------------------------------------
enum BiStage { BI_INIT = 0, BI_ALPHA = 1, BI_SO = 2, BI_X = 3 };

// NV partial arrays: NC for BI_ALPHA, 3 NC for BI_SO (t.s, t.t, s.s), 2 NC otherwise
template <int NC, int NV>
__global__ __launch_bounds__(BLOCK) void k_bi_fin(int stage, const double* __restrict__ part, Tiles T, BiState* sts) {
  BiState* st = sts + blockIdx.x;
  // the segment's state and tile range loaded together, before the partials (thread 0 works on the
  // copy and stores it back whole; no other block touches this segment's state).  No early return
  // for a stopped segment, which would hold the other loads back behind the flag's: with no active
  // component the update below changes nothing.
  BiState S = *st;
  const int f = T.first[blockIdx.x], n = T.count[blockIdx.x];
  double tot[NV];
  seg_thread_sum<NV>(part, T.ntile, f, n, tot);
  __shared__ double lds[NV][BLOCK / 64];
  block_sum<NV>(tot, lds);
  if (threadIdx.x != 0) return;
  int any = 0;
  for (int c = 0; c < NC; ++c) {
    if (stage == BI_INIT) {
      double bn = sqrt(tot[c]), rn = sqrt(tot[NC + c]);
      S.bn[c] = bn;
      S.iters[c] = 0;
      S.status[c] = 0;
      S.phase[c] = 0;
      S.zero_b[c] = bn == 0.0;
      S.res[c] = bn == 0.0 ? 0.0 : rn / bn;
      S.active[c] = (bn == 0.0 || rn <= S.tol * bn) ? 0 : 1;
      S.rho[c] = S.alpha[c] = S.omega[c] = 1.0;
      S.rho1[c] = tot[NC + c];  // rhat = r, so rhat.r = r.r
      if (S.active[c] && S.maxit <= 0) {
        S.active[c] = 0;
        S.status[c] = DIFVM_WARN_NOT_CONVERGED;
      } else if (S.active[c] && S.rho1[c] == 0.0) {
        S.active[c] = 0;
        S.status[c] = DIFVM_WARN_BREAKDOWN;
      }
      if (S.active[c]) S.beta[c] = (S.rho1[c] / S.rho[c]) * (S.alpha[c] / S.omega[c]);
    } else if (!S.active[c]) {
      continue;
    } else if (stage == BI_ALPHA) {
      S.alpha[c] = S.rho1[c] / tot[c];
    } else if (stage == BI_SO) {
      // the test on |s| first (the iteration ends with x += alpha y if it passes), then omega
      double sn = sqrt(tot[(2 * NC + c) % NV]);  // NV = 3 NC in this stage
      if (sn <= S.tol * S.bn[c]) {
        S.phase[c] = 1;
        S.res[c] = sn / S.bn[c];
      } else if (tot[NC + c] == 0.0) {
        S.active[c] = 0;
        S.status[c] = DIFVM_WARN_BREAKDOWN;
      } else {
        S.omega[c] = tot[c] / tot[NC + c];
      }
    } else {  // BI_X
      int it = S.iters[c] + 1;
      S.iters[c] = it;
      if (S.phase[c]) {
        S.active[c] = 0;
      } else {
        S.rho[c] = S.rho1[c];
        double rn = sqrt(tot[c]);
        S.res[c] = rn / S.bn[c];
        if (rn <= S.tol * S.bn[c]) {
          S.active[c] = 0;
        } else if (it >= S.maxit) {
          S.active[c] = 0;
          S.status[c] = DIFVM_WARN_NOT_CONVERGED;
        } else {
          S.rho1[c] = tot[NC + c];
          if (S.rho1[c] == 0.0) {
            S.active[c] = 0;
            S.status[c] = DIFVM_WARN_BREAKDOWN;
          } else {
            S.beta[c] = (S.rho1[c] / S.rho[c]) * (S.alpha[c] / S.omega[c]);
          }
        }
      }
    }
    any |= S.active[c];
  }
  S.any = any;
  *st = S;
}

// r = b - A x, rhat = r, partials b.b and r.r (p and v start at zero: the first direction pass
// writes p = r without reading them)
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_init(SellView A, Tiles T, const double* __restrict__ b,
                                                   const double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ rh, double* __restrict__ part) {
  TileIdx ti = tile_idx(T);
  double acc[2 * NC];
#pragma unroll
  for (int k = 0; k < 2 * NC; ++k) acc[k] = 0.0;
  FOR_TILE_CELLS(i) {
    double ax[NC];
    sell_row<NC>(A, i, x, ax);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      size_t at = (size_t)i * NC + c;
      double bi = b[at], ri = bi - ax[c];
      r[at] = ri;
      rh[at] = ri;
      acc[c] += bi * bi;
      acc[NC + c] += ri * ri;
    }
  }
  put_partial<2 * NC>(acc, part, T.ntile, ti.t);
}

template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_zero(Tiles T, double* __restrict__ x, const BiState* sts) {
  TileIdx ti = tile_idx(T);
  const BiState* st = sts + ti.s;
  FOR_TILE_CELLS(i) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (st->zero_b[c]) x[(size_t)i * NC + c] = 0.0;
  }
}

// (A f)_i for NC interleaved components, f(j, c) giving the operand of cell j; padding and boundary
// slots carry val = 0 and col = i
template <int NC, class F>
__device__ __forceinline__ void sell_row_f(const SellView& A, int i, F&& f, double (&acc)[NC]) {
  SlotRange R = slots_of(A, i);
  double di = A.diag[i];
  const bool off16 = A.off16 != nullptr;  // the same for every thread: a uniform branch
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = di * f(i, c);
#pragma unroll 4
  for (int k = 0; k < R.width; ++k) {
    int at = R.base + k * SLICE;
    double a = A.val[at];
    int j = off16 ? i + A.off16[at] : A.col[at];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += a * f(j, c);
  }
}

// The right-preconditioned vectors y = p / d and z = s / d are formed where they are used, not stored.
// p = r + beta (p - omega v); the first iteration's p = r (p and v are zero then and not read)
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_dir(SellView A, Tiles T, const double* __restrict__ r, double* __restrict__ p,
                                                  const double* __restrict__ v, const BiState* sts, int first) {
  TileIdx ti = tile_idx(T);
  const BiState* st = sts + ti.s;
  if (!st->any) return;
  // one thread per value of the tile's rows (consecutive lanes, consecutive doubles)
  const int e1 = NC * ti.hi;
#pragma unroll
  for (int q = 0; q < NC * CPT; ++q) {
    int e = NC * ti.lo + q * BLOCK + (int)threadIdx.x;
    if (e >= e1) break;
    int c = e % NC;
    if (!st->active[c]) continue;
    if (first) p[e] = r[e];
    else p[e] = r[e] + st->beta[c] * (p[e] - st->omega[c] * v[e]);
  }
}

// v = A y, y = p / d; partial rhat . v
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_v(SellView A, Tiles T, const double* __restrict__ p, double* __restrict__ v,
                                                const double* __restrict__ rh, double* __restrict__ part, const BiState* sts) {
  TileIdx ti = tile_idx(T);
  const BiState* st = sts + ti.s;
  if (!st->any) return;
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  // (staging these stores through LDS measured slower here: the rounds' barriers hold back the
  // gathers of the waves that could run ahead)
  FOR_TILE_CELLS(i) {
    double rhi[NC], ay[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) rhi[c] = rh[(size_t)i * NC + c];  // in flight with the row's loads
    sell_row_f<NC>(A, i, [&](int j, int c) { return p[(size_t)j * NC + c] / A.diag[j]; }, ay);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!st->active[c]) continue;
      size_t at = (size_t)i * NC + c;
      v[at] = ay[c];
      acc[c] += rhi[c] * ay[c];
    }
  }
  put_partial<NC>(acc, part, T.ntile, ti.t);
}

// s = r - alpha v, one thread per value of the tile's rows (as k_bi_dir)
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_s(Tiles T, const double* __restrict__ r, const double* __restrict__ v,
                                                double* __restrict__ s, const BiState* sts) {
  TileIdx ti = tile_idx(T);
  const BiState* st = sts + ti.s;
  if (!st->any) return;
  const int e1 = NC * ti.hi;
#pragma unroll
  for (int q = 0; q < NC * CPT; ++q) {
    int e = NC * ti.lo + q * BLOCK + (int)threadIdx.x;
    if (e >= e1) break;
    int c = e % NC;
    if (!st->active[c]) continue;
    s[e] = r[e] - st->alpha[c] * v[e];
  }
}

// t = A z with z = s / d (s gathered from the pass above); partials t.s, t.t, s.s
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_t(SellView A, Tiles T, const double* __restrict__ s,
                                                double* __restrict__ t, double* __restrict__ part, const BiState* sts) {
  TileIdx ti = tile_idx(T);
  const BiState* st = sts + ti.s;
  if (!st->any) return;
  double acc[3 * NC];
#pragma unroll
  for (int k = 0; k < 3 * NC; ++k) acc[k] = 0.0;
  FOR_TILE_CELLS(i) {
    double az[NC];
    sell_row_f<NC>(A, i, [&](int j, int c) { return s[(size_t)j * NC + c] / A.diag[j]; }, az);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (!st->active[c]) continue;
      size_t at = (size_t)i * NC + c;
      double si = s[at];
      t[at] = az[c];
      acc[c] += az[c] * si;
      acc[NC + c] += az[c] * az[c];
      acc[2 * NC + c] += si * si;
    }
  }
  put_partial<3 * NC>(acc, part, T.ntile, ti.t);
}

// x += alpha y (+ omega z); r = s - omega t; partials r.r, rhat.r
template <int NC>
__global__ __launch_bounds__(BLOCK) void k_bi_x(SellView A, Tiles T, double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ rh, const double* __restrict__ p,
                                                const double* __restrict__ s, const double* __restrict__ t,
                                                double* __restrict__ part, const BiState* sts) {
  TileIdx ti = tile_idx(T);
  const BiState* st = sts + ti.s;
  if (!st->any) return;
  double acc[2 * NC];
#pragma unroll
  for (int k = 0; k < 2 * NC; ++k) acc[k] = 0.0;
  bool keep_x[NC], keep_r[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    keep_x[c] = st->active[c] != 0;
    keep_r[c] = keep_x[c] && !st->phase[c];
  }
  __shared__ double lds[NC * BLOCK];
  FOR_TILE_ROUNDS(base, i) {
    double xv[NC] = {}, rv[NC] = {};
    if (i < ti.hi) {
      double di = A.diag[i];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (!keep_x[c]) continue;
        size_t at = (size_t)i * NC + c;
        double yi = p[at] / di;
        if (!keep_r[c]) {
          xv[c] = x[at] + st->alpha[c] * yi;
        } else {
          double si = s[at];
          xv[c] = x[at] + (st->alpha[c] * yi + st->omega[c] * (si / di));
          double ri = si - st->omega[c] * t[at];
          rv[c] = ri;
          acc[c] += ri * ri;
          acc[NC + c] += rh[at] * ri;
        }
      }
    }
    if constexpr (NC == 1) {
      if (i < ti.hi && keep_x[0]) x[i] = xv[0];
      if (i < ti.hi && keep_r[0]) r[i] = rv[0];
    } else {
      store_rows_if<NC>(x, base, ti.hi, xv, keep_x, lds);
      store_rows_if<NC>(r, base, ti.hi, rv, keep_r, lds);
    }
  }
  put_partial<2 * NC>(acc, part, T.ntile, ti.t);
}

__global__ void k_bi_state_init(BiState* sts, int nseg, double tol, int maxit) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nseg) return;
  BiState st{};
  st.tol = tol;
  st.maxit = maxit;
  sts[g] = st;
}

size_t bicgstab_state_bytes(const difvm_mesh* m) { return sizeof(BiState) * m->d.nseg; }

SolveResult bicgstab_result(const difvm_mesh* m, int ncomp, const void* host_state, bool* complete) {
  const BiState* hs = static_cast<const BiState*>(host_state);
  int nseg = m->d.nseg;
  SolveResult R;
  R.seg.resize(nseg);
  bool all = true;
  for (int g = 0; g < nseg; ++g) {
    const BiState& st = hs[g];
    all = all && !st.any;
    SegResult& sr = R.seg[g];
    sr.status = 0;
    for (int c = 0; c < ncomp; ++c) {
      sr.iters[c] = st.iters[c];
      sr.res[c] = st.res[c];
      sr.status = std::max(sr.status, st.active[c] ? (int)DIFVM_WARN_NOT_CONVERGED : st.status[c]);
      R.iters[c] = std::max(R.iters[c], st.iters[c]);
      R.res[c] = std::max(R.res[c], st.res[c]);
    }
    R.status = std::max(R.status, sr.status);
  }
  if (complete) *complete = all;
  return R;
}

template <int NC>
static SolveResult bicgstab_nc(difvm_mesh* m, SellMatrix A, const double* b, double* x, double tol, int maxit,
                               const QueueOnly* qo, int* hint) {
  KrylovWork* w = make_work(m);
  hipStream_t s = stream_of(m);
  SellView V = sview(m, A);
  Tiles T = tiles_of(m);
  int G = T.ntile, nseg = m->d.nseg;
  k_bi_state_init<<<(nseg + 63) / 64, 64, 0, s>>>(w->bi, nseg, tol, maxit);
  double* part = w->partials;
  k_bi_init<NC><<<G, BLOCK, 0, s>>>(V, T, b, x, w->r, w->rh, part);
  k_bi_fin<NC, 2 * NC><<<nseg, BLOCK, 0, s>>>(BI_INIT, part, T, w->bi);
  k_bi_zero<NC><<<G, BLOCK, 0, s>>>(T, x, w->bi);
  DIFVM_HIP(hipGetLastError());
  int done = 0;  // iterations queued
  auto queue_iters = [&](int nb) {
    for (int it = 0; it < nb; ++it) {
      k_bi_dir<NC><<<G, BLOCK, 0, s>>>(V, T, w->r, w->p, w->v, w->bi, done + it == 0 ? 1 : 0);
      k_bi_v<NC><<<G, BLOCK, 0, s>>>(V, T, w->p, w->v, w->rh, part, w->bi);
      k_bi_fin<NC, NC><<<nseg, BLOCK, 0, s>>>(BI_ALPHA, part, T, w->bi);
      k_bi_s<NC><<<G, BLOCK, 0, s>>>(T, w->r, w->v, w->s, w->bi);
      k_bi_t<NC><<<G, BLOCK, 0, s>>>(V, T, w->s, w->t, part, w->bi);
      k_bi_fin<NC, 3 * NC><<<nseg, BLOCK, 0, s>>>(BI_SO, part, T, w->bi);
      k_bi_x<NC><<<G, BLOCK, 0, s>>>(V, T, x, w->r, w->rh, w->p, w->s, w->t, part, w->bi);
      k_bi_fin<NC, 2 * NC><<<nseg, BLOCK, 0, s>>>(BI_X, part, T, w->bi);
    }
    done += nb;
    DIFVM_HIP(hipGetLastError());
  };
  if (qo) {
    queue_iters(std::min(qo->budget, maxit));
    copy_state(qo->state_out, w->bi, bicgstab_state_bytes(m), s);
    return SolveResult{};
  }
  const size_t bytes = bicgstab_state_bytes(m);
  queue_iters(std::min(maxit, std::max(2, (hint ? *hint : 0) - 1)));
  int slot = 0;
  post_poll(m, w, w->bi, bytes, slot);
  const BiState* hs = nullptr;
  while (true) {
    bool more = done < maxit;
    if (more) {
      queue_iters(std::min(1, maxit - done));
      post_poll(m, w, w->bi, bytes, slot ^ 1);
    }
    hs = static_cast<const BiState*>(wait_poll(w, slot));
    bool any = false;
    for (int g = 0; g < nseg; ++g) any = any || hs[g].any;
    if (!any || !more) break;
    slot ^= 1;
  }
  SolveResult R = bicgstab_result(m, NC, hs, nullptr);
  if (hint) *hint = std::max(R.iters[0], std::max(R.iters[1], R.iters[2]));
  return R;
}

SolveResult bicgstab(difvm_mesh* m, int ncomp, SellMatrix A, const double* b, double* x, double tol, int maxit,
                     const QueueOnly* qo, int* hint) {
  if (ncomp == 1) return bicgstab_nc<1>(m, A, b, x, tol, maxit, qo, hint);
  return bicgstab_nc<3>(m, A, b, x, tol, maxit, qo, hint);
}

// ---------------------------------------------------------------------------------------------
// timing of the product kernel for the autotuner: `reps` launches at iteration 2 on scratch data
// (matrix values, vectors and partials set to constants, a control state that never stops), so no
// solve state is involved; returns seconds per launch
// ---------------------------------------------------------------------------------------------
__global__ void k_fill_const(double* __restrict__ a, size_t n, double v) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) a[q] = v;
}
__global__ void k_tune_ctl(PcgCtl* ctls, int nseg) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nseg) return;
  PcgCtl c{};
  c.tol = 0.0;
  c.bn = 1.0;
  c.rho[0] = c.rho[1] = 1.0;
  c.maxit = 1 << 30;
  ctls[g] = c;
}

double time_pcg_spmv(difvm_mesh* m, int grid, int reps, hipEvent_t e0, hipEvent_t e1) {
  KrylovWork* w = make_work(m);
  hipStream_t s = stream_of(m);
  const DMesh& d = m->d;
  const Ctx& cx = ctx_of(m);
  double* val = dalloc<double>(cx, d.nslot);
  double* diag = nullptr;
  PcgCtl* ctl = nullptr;
  double t = 0.0;
  try {
    diag = dalloc<double>(cx, d.nc);
    ctl = static_cast<PcgCtl*>(dmalloc(cx, sizeof(PcgCtl) * d.nseg));
    auto fill = [&](double* a, size_t n, double v) {
      k_fill_const<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, n, v);
    };
    fill(val, d.nslot, -0.25);
    fill(diag, d.nc, 4.0);
    fill(w->z, d.nc, 1.0);
    fill(w->p, d.nc, 1.0);
    fill(w->partials, (size_t)8 * w->ntile, 1.0);
    k_tune_ctl<<<(d.nseg + 63) / 64, 64, 0, s>>>(ctl, d.nseg);
    DIFVM_HIP(hipGetLastError());
    int old = m->tune[DIFVM_TUNE_PCG_GRID];
    m->tune[DIFVM_TUNE_PCG_GRID] = grid;
    int GS = pcg_spmv_grid(m);
    m->tune[DIFVM_TUNE_PCG_GRID] = old;
    SellView V = sview(m, SellMatrix{diag, val});  // the same column form the solves read
    Tiles T = tiles_of(m);
    double* partA = w->partials;
    double* partB = w->partials + 2 * (size_t)T.ntile;
    launch_pcg_spmv(GS, s, V, T, 2, w->z, w->p, w->v, w->q, partB, partA, ctl);
    DIFVM_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r)
      launch_pcg_spmv(GS, s, V, T, 2, w->z, w->p, w->v, w->q, partB, partA, ctl);
    DIFVM_HIP(hipEventRecord(e1, s));
    DIFVM_HIP(hipGetLastError());
    DIFVM_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    DIFVM_HIP(hipEventElapsedTime(&ms, e0, e1));
    t = ms * 1e-3 / reps;
  } catch (...) {
    (void)hipStreamSynchronize(s);
    dfree(cx, val);
    dfree(cx, diag);
    dfree(cx, ctl);
    throw;
  }
  dfree(cx, val);
  dfree(cx, diag);
  dfree(cx, ctl);
  return t;
}

}  // namespace difvm
