// Device side of the smoothed-aggregation AMG preconditioner for the pressure CG.
//
// One V-cycle, z = M^-1 r, from level 0 (the cell-slot matrix K of the mesh, internal order) down to
// a coarsest level solved with its dense inverse:
//   down, level l:  x_l = w D_l^-1 b_l (one damped-Jacobi sweep from zero),  res_l = b_l - A_l x_l,
//                   b_{l+1} = R_l res_l                         (b_0 = r)
//   coarsest:       x_L = A_L^-1 b_L
//   up, level l:    t_l = x_l + P_l x_{l+1},  x_l = t_l + w D_l^-1 (b_l - A_l t_l)   (z = x_0)
// with w = 2/3.  Pre- and post-smoothing are the same symmetric sweep and R_l = P_l^T, so M^-1 is
// symmetric; it is positive definite since w rho(D^-1 A) < 2.  x_l = w D^-1 b_l is recomputed where
// needed rather than stored.  Each stage is one kernel: row kernels on the cell-slot layout for
// level 0, CSR kernels with SW lanes per row (rows summed by a fixed shuffle tree) on coarser levels,
// so every result is deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "amg_dev.h"
#include "krylov_util.h"

namespace difvm {

namespace {
constexpr double OMEGA = 2.0 / 3.0;

struct DevCsr {
  int n = 0, nnz = 0, sw = 1;  // sw: lanes per row in the CSR kernels
  int32_t *ptr = nullptr, *col = nullptr;
  double *val = nullptr, *diag = nullptr;
};
}  // namespace

struct AmgDev {
  difvm_mesh* mesh = nullptr;
  int L = 0;                     // coarse levels 1..L (level L is the coarsest)
  std::vector<DevCsr> A;         // A[l], l = 1..L (A[0] unused: level 0 is K)
  std::vector<DevCsr> P, R;      // P[l]: rows of level l, columns of l+1; R[l]: rows of level l+1
  std::vector<double*> b, res, t, x;  // per level (index 0: res, t only)
  double* cinv = nullptr;        // dense inverse of A_L, row-major
  std::vector<int> rows;
  std::vector<void*> allocs;
  // Eager solves replay the V-cycle as one captured graph (one host submission instead of one per
  // kernel; the cycle is launch-bound below the finest levels).  It is captured on a private stream
  // for one set of arguments and recaptured when they change.
  mutable hipStream_t cap = nullptr;
  mutable hipGraphExec_t vexec = nullptr;
  mutable const void* vkey[6] = {};
};

namespace {

template <class T>
T* up(AmgDev* a, const std::vector<T>& v, hipStream_t s) {
  T* p = dalloc<T>(v.size());
  a->allocs.push_back(p);
  upload(p, v, s);
  return p;
}
double* work(AmgDev* a, size_t n) {
  double* p = dalloc<double>(n);
  a->allocs.push_back(p);
  return p;
}

int lanes_for(int n, size_t nnz) {
  double avg = n ? (double)nnz / n : 0.0;
  int sw = 1;
  while (sw < 64 && sw * 2 <= avg) sw *= 2;
  return sw;
}

DevCsr upload_csr(AmgDev* a, const AmgCsr& M, bool with_diag, hipStream_t s) {
  DevCsr d;
  d.n = M.n;
  d.nnz = (int)M.col.size();
  d.sw = lanes_for(M.n, M.col.size());
  d.ptr = up(a, M.ptr, s);
  d.col = up(a, M.col, s);
  d.val = up(a, M.val, s);
  if (with_diag) d.diag = up(a, M.diag, s);
  return d;
}

// ---- kernels ------------------------------------------------------------------------------------
// Every segment's CG stopped: the V-cycle of an iteration queued past the stop has nothing to do.
// One thread reads the flags and the block shares the answer, so whole blocks return together.
struct StopFlags {
  const PcgCtl* ctl;  // nullptr: never stopped
  int nseg;
};
__device__ __forceinline__ bool stopped(const StopFlags& st) {
  if (!st.ctl) return false;
  __shared__ int f;
  __syncthreads();
  if (threadIdx.x == 0) {
    int all = 1;
    for (int g = 0; g < st.nseg && all; ++g) all = st.ctl[g].done;
    f = all;
  }
  __syncthreads();
  return f != 0;
}

// column of slot `at` in row i (16-bit offsets when the mesh has them)
template <bool OFF16>
__device__ __forceinline__ int slot_col_of(const SellView& K, int i, int at) {
  if constexpr (OFF16) return i + K.off16[at];
  else return K.col[at];
}

// level 0, down: res = r - K (w D^-1 r)
template <bool OFF16>
__global__ __launch_bounds__(BLOCK) void k_amg_fine_pre(SellView K, const double* __restrict__ r,
                                                        double* __restrict__ res, StopFlags ctl) {
  if (stopped(ctl)) return;
  int i = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (i >= K.nc) return;
  SlotRange R = slots_of(K.slice_start, i);
  double acc = 0.0;
#pragma unroll 4
  for (int k = 0; k < R.width; ++k) {
    int at = R.base + k * SLICE;
    int j = slot_col_of<OFF16>(K, i, at);
    acc += K.val[at] * (r[j] / K.diag[j]);
  }
  double ri = r[i];
  res[i] = ri - OMEGA * ri - OMEGA * acc;
}

// SW lanes per row: partial sums of the row's entries, then a fixed xor-shuffle tree
template <int SW>
__device__ __forceinline__ double lane_sum(double s) {
#pragma unroll
  for (int off = SW / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, SW);
  return s;
}

// out = R x (rows of the coarser level)
template <int SW>
__global__ __launch_bounds__(BLOCK) void k_amg_restrict(int n, const int32_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ col, const double* __restrict__ val,
                                                        const double* __restrict__ xin, double* __restrict__ out,
                                                        StopFlags ctl) {
  if (stopped(ctl)) return;
  int g = blockIdx.x * BLOCK + threadIdx.x;
  int row = g / SW, lane = g % SW;
  double s = 0.0;
  if (row < n)
    for (int q = ptr[row] + lane; q < ptr[row + 1]; q += SW) s += val[q] * xin[col[q]];
  s = lane_sum<SW>(s);
  if (row < n && lane == 0) out[row] = s;
}

// coarse level, down: res = b - A (w D^-1 b)
template <int SW>
__global__ __launch_bounds__(BLOCK) void k_amg_pre(int n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, const double* __restrict__ diag,
                                                   const double* __restrict__ b, double* __restrict__ res,
                                                   StopFlags ctl) {
  if (stopped(ctl)) return;
  int g = blockIdx.x * BLOCK + threadIdx.x;
  int row = g / SW, lane = g % SW;
  double s = 0.0;
  if (row < n)
    for (int q = ptr[row] + lane; q < ptr[row + 1]; q += SW) {
      int j = col[q];
      s += val[q] * (b[j] / diag[j]);
    }
  s = lane_sum<SW>(s);
  if (row < n && lane == 0) {
    double bi = b[row];
    res[row] = bi - OMEGA * bi - OMEGA * s;
  }
}

// coarse level, up: x = t + w D^-1 (b - A t)
template <int SW>
__global__ __launch_bounds__(BLOCK) void k_amg_post(int n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                    const double* __restrict__ val, const double* __restrict__ diag,
                                                    const double* __restrict__ b, const double* __restrict__ t,
                                                    double* __restrict__ x, StopFlags ctl) {
  if (stopped(ctl)) return;
  int g = blockIdx.x * BLOCK + threadIdx.x;
  int row = g / SW, lane = g % SW;
  double s = 0.0;
  if (row < n)
    for (int q = ptr[row] + lane; q < ptr[row + 1]; q += SW) s += val[q] * t[col[q]];
  s = lane_sum<SW>(s);
  if (row < n && lane == 0) {
    double d = diag[row], ti = t[row];
    x[row] = ti + OMEGA * (b[row] - d * ti - s) / d;
  }
}

// up: t = w D^-1 b + P xc (one thread per row of the finer level)
__global__ __launch_bounds__(BLOCK) void k_amg_prolong(int n, const int32_t* __restrict__ ptr,
                                                       const int32_t* __restrict__ col, const double* __restrict__ val,
                                                       const double* __restrict__ diag, const double* __restrict__ b,
                                                       const double* __restrict__ xc, double* __restrict__ t,
                                                       StopFlags ctl) {
  if (stopped(ctl)) return;
  int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = ptr[i]; q < ptr[i + 1]; ++q) s += val[q] * xc[col[q]];
  t[i] = OMEGA * b[i] / diag[i] + s;
}

// coarsest: x = A_L^-1 b (dense, one thread per row, one block)
__global__ __launch_bounds__(1024) void k_amg_coarsest(int n, const double* __restrict__ inv,
                                                       const double* __restrict__ b, double* __restrict__ x,
                                                       StopFlags ctl) {
  if (stopped(ctl)) return;
  int i = threadIdx.x;
  if (i >= n) return;
  const double* row = inv + (size_t)i * n;
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += row[j] * b[j];
  x[i] = s;
}

// level 0, up: z = t + w D^-1 (r - K t), with per-tile partials of r.z
template <bool OFF16>
__global__ __launch_bounds__(BLOCK) void k_amg_fine_post(SellView K, Tiles T, const double* __restrict__ r,
                                                         const double* __restrict__ t, double* __restrict__ z,
                                                         double* __restrict__ part, StopFlags ctl) {
  TileIdx ti = tile_idx(T);
  if (stopped(ctl)) return;
  double v[1] = {0.0};
  FOR_TILE_CELLS(i) {
    SlotRange R = slots_of(K.slice_start, i);
    double di = K.diag[i], ti = t[i];
    double kt = di * ti;
#pragma unroll 4
    for (int k = 0; k < R.width; ++k) {
      int at = R.base + k * SLICE;
      kt += K.val[at] * t[slot_col_of<OFF16>(K, i, at)];
    }
    double ri = r[i];
    double zi = ti + OMEGA * (ri - kt) / di;
    z[i] = zi;
    v[0] += ri * zi;
  }
  if (part) put_partial<1>(v, part, T.ntile, ti.t);
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
    a->P.resize(L_);
    a->R.resize(L_);
    a->b.assign(L_ + 1, nullptr);
    a->res.assign(L_ + 1, nullptr);
    a->t.assign(L_ + 1, nullptr);
    a->x.assign(L_ + 1, nullptr);
    a->rows.push_back(d.nc);
    for (int l = 0; l < L_; ++l) {
      a->P[l] = upload_csr(a, H.levels[l].P, false, s);
      a->R[l] = upload_csr(a, H.levels[l].R, false, s);
      a->A[l + 1] = upload_csr(a, H.coarse[l], true, s);
      a->rows.push_back(H.coarse[l].n);
    }
    for (int l = 0; l <= L_; ++l) {
      size_t n = a->rows[l];
      a->res[l] = work(a, n);
      a->t[l] = work(a, n);
      if (l > 0) {
        a->b[l] = work(a, n);
        a->x[l] = work(a, n);
      }
    }
    DIFVM_CHECK(H.n_coarsest <= 1024, DIFVM_ERR_UNSUPPORTED, "coarsest AMG level too large");
    a->cinv = up(a, H.coarsest_inv, s);
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
  if (a->vexec) (void)hipGraphExecDestroy(a->vexec);
  if (a->cap) (void)hipStreamDestroy(a->cap);
  for (void* p : a->allocs) dfree(p);
  delete a;
}

int amg_levels(const AmgDev* a, int* rows, int cap) {
  int n = (int)a->rows.size();
  for (int l = 0; l < n && l < cap; ++l) rows[l] = a->rows[l];
  return n;
}

static void launch_vcycle(const AmgDev* a, hipStream_t s, SellMatrix Km, const double* r, double* z, double* part,
                          StopFlags ctl) {
  difvm_mesh* m = a->mesh;
  SellView K = sview(m, Km);
  const int L = a->L, nc = m->d.nc;
  // down
  if (K.off16) k_amg_fine_pre<true><<<grid_for(nc), BLOCK, 0, s>>>(K, r, a->res[0], ctl);
  else k_amg_fine_pre<false><<<grid_for(nc), BLOCK, 0, s>>>(K, r, a->res[0], ctl);
  {
    const DevCsr& R = a->R[0];
    DIFVM_AMG_DISPATCH(k_amg_restrict, R.sw, R.n, s, R.n, R.ptr, R.col, R.val, a->res[0], a->b[1], ctl);
  }
  for (int l = 1; l < L; ++l) {
    const DevCsr& A = a->A[l];
    DIFVM_AMG_DISPATCH(k_amg_pre, A.sw, A.n, s, A.n, A.ptr, A.col, A.val, A.diag, a->b[l], a->res[l], ctl);
    const DevCsr& R = a->R[l];
    DIFVM_AMG_DISPATCH(k_amg_restrict, R.sw, R.n, s, R.n, R.ptr, R.col, R.val, a->res[l], a->b[l + 1], ctl);
  }
  k_amg_coarsest<<<1, 1024, 0, s>>>(a->rows[L], a->cinv, a->b[L], a->x[L], ctl);
  // up
  for (int l = L - 1; l >= 1; --l) {
    const DevCsr& P = a->P[l];
    const DevCsr& A = a->A[l];
    k_amg_prolong<<<grid_for(P.n), BLOCK, 0, s>>>(P.n, P.ptr, P.col, P.val, A.diag, a->b[l], a->x[l + 1], a->t[l], ctl);
    DIFVM_AMG_DISPATCH(k_amg_post, A.sw, A.n, s, A.n, A.ptr, A.col, A.val, A.diag, a->b[l], a->t[l], a->x[l], ctl);
  }
  {
    const DevCsr& P = a->P[0];
    k_amg_prolong<<<grid_for(P.n), BLOCK, 0, s>>>(P.n, P.ptr, P.col, P.val, Km.diag, r, a->x[1], a->t[0], ctl);
  }
  Tiles T = tiles_of(m);
  if (K.off16) k_amg_fine_post<true><<<T.ntile, BLOCK, 0, s>>>(K, T, r, a->t[0], z, part, ctl);
  else k_amg_fine_post<false><<<T.ntile, BLOCK, 0, s>>>(K, T, r, a->t[0], z, part, ctl);
  DIFVM_HIP(hipGetLastError());
}

void amg_vcycle(const AmgDev* a, SellMatrix Km, const double* r, double* z, double* part, const PcgCtl* ctls) {
  difvm_mesh* m = a->mesh;
  Ctx& c = ctx_of(m);
  StopFlags ctl{ctls, m->d.nseg};
  if (c.capturing) {  // inside a captured step: the kernels join that graph
    launch_vcycle(a, c.stream, Km, r, z, part, ctl);
    return;
  }
  const void* key[6] = {Km.diag, Km.val, r, z, part, ctls};
  if (!a->vexec || !std::equal(key, key + 6, a->vkey)) {
    if (a->vexec) {
      DIFVM_HIP(hipStreamSynchronize(c.stream));  // a replay of the old graph may still be queued
      DIFVM_HIP(hipGraphExecDestroy(a->vexec));
      a->vexec = nullptr;
    }
    if (!a->cap) DIFVM_HIP(hipStreamCreateWithFlags(&a->cap, hipStreamNonBlocking));
    DIFVM_HIP(hipStreamBeginCapture(a->cap, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      launch_vcycle(a, a->cap, Km, r, z, part, ctl);
    } catch (...) {
      (void)hipStreamEndCapture(a->cap, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    DIFVM_HIP(hipStreamEndCapture(a->cap, &g));
    hipError_t e = hipGraphInstantiate(&a->vexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    DIFVM_HIP(e);
    std::copy(key, key + 6, a->vkey);
  }
  DIFVM_HIP(hipGraphLaunch(a->vexec, c.stream));
}

}  // namespace difvm
