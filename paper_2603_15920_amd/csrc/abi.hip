// C entry points of libdifvm (declared in include/difvm.h): argument checks, object lifetimes and
// dispatch to the kernels.  No exception crosses this boundary.
#include <cstring>
#include <mutex>
#include <string>

#include "abi_util.h"
#include "amg_dev.h"
#include "ops.h"

namespace difvm {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

void* dmalloc(const Ctx& c, size_t bytes) {
  bytes = bytes ? bytes : 1;
  if (c.alloc.alloc) {
    void* p = c.alloc.alloc(bytes, c.stream, c.alloc.user);
    if (!p) throw Error{DIFVM_ERR_OOM, "the context's allocator returned NULL for " + std::to_string(bytes) + " bytes"};
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) throw Error{DIFVM_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
  return p;
}
void dfree(const Ctx& c, void* p) {
  if (!p) return;
  if (c.alloc.free) c.alloc.free(p, c.stream, c.alloc.user);
  else (void)hipFree(p);
}

static hipEvent_t pool_event(Profiler& P) {
  if (!P.pool.empty()) {
    hipEvent_t e = P.pool.back();
    P.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  // timing-only events: no system-scope fence (cache write-back) around the timed launch
  DIFVM_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return e;
}

static int prof_id(Profiler& P, const std::string& name) {
  for (size_t k = 0; k < P.names.size(); ++k)
    if (P.names[k] == name) return (int)k;
  P.names.push_back(name);
  P.total_ms.push_back(0.0);
  P.launches.push_back(0);
  P.seen.push_back(0);
  return (int)P.names.size() - 1;
}

int prof_begin(Ctx& c, const char* name, long iter) {
  Profiler& P = c.prof;
  if (c.capturing) return -1;
  const bool phase = std::strncmp(name, "step: ", 6) == 0;  // phases: every time, kernels: every stride-th
  if (phase ? !P.phases : !P.on) return -1;
  int id = prof_id(P, name);
  if (!phase && P.seen[id]++ % P.stride != 0) return -1;
  Profiler::Rec r{id, pool_event(P), pool_event(P), iter};
  DIFVM_HIP(hipEventRecord(r.a, c.stream));
  P.pending.push_back(r);
  return (int)P.pending.size() - 1;
}

void prof_end(Ctx& c, int handle) {
  if (handle < 0) return;
  (void)hipEventRecord(c.prof.pending[handle].b, c.stream);
}

void prof_idle_after(Ctx& c, size_t from, long last) {
  Profiler& P = c.prof;
  for (size_t k = from; k < P.pending.size(); ++k) {
    Profiler::Rec& r = P.pending[k];
    if (r.iter > last) r.id = prof_id(P, P.names[r.id] + " (idle)");
  }
}

static void prof_collect(Ctx& c) {
  Profiler& P = c.prof;
  if (P.pending.empty()) return;
  DIFVM_HIP(hipStreamSynchronize(c.stream));
  for (auto& r : P.pending) {
    float ms = 0.f;
    DIFVM_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    P.total_ms[r.id] += ms;
    P.launches[r.id] += 1;
    P.pool.push_back(r.a);
    P.pool.push_back(r.b);
  }
  P.pending.clear();
}

// PISO functions (piso.hip)
void piso_create(difvm_mesh* m, const difvm_piso_params* prm, difvm_piso** out);
void piso_set_boundary(difvm_piso* P, const double* Ub, const double* pb);
void piso_set_windkessel(difvm_piso* P, int id, double Rp, double C, double Rd, double pc);
void piso_set_viscosity(difvm_piso* P, int nseg, const double* nu_seg);
void piso_release(difvm_piso* P);
void piso_set_graph(difvm_piso* P, int enable, int extra);
SolveResult piso_transport_scalar(difvm_piso* P, double D, int table, const double* cb_user, double* c_user);
void piso_graph_info(const difvm_piso* P, long long* replays, long long* redos, long long* captures);
void piso_segment_stats(const difvm_piso* P, int nseg, difvm_step_stats* out);
void piso_set_state(difvm_piso* P, const double* U, const double* p, const double* phi);
void piso_get_state(difvm_piso* P, double* U, double* p, double* phi, double* pc_host);
int piso_step(difvm_piso* P, int nsteps, difvm_step_stats* stats);
int piso_step_trace(difvm_piso* P, double* Ustar_user, double* p_user, difvm_step_stats* stats);
void piso_precond_info(const difvm_piso* P, int32_t* n_levels, int32_t* rows, int32_t cap, double* vcycle_bytes);
void piso_rebuild_preconditioner(difvm_piso* P);

static void check_mesh(const difvm_mesh* m) { DIFVM_CHECK(m != nullptr, DIFVM_ERR_INVALID_ARG, "mesh is NULL"); }
// solvers reduce over every cell of the mesh: a partition part (ghost rows included, no exchange
// inside the iteration) is refused
static void check_whole(const difvm_mesh* m) {
  DIFVM_CHECK(m->part_n_owned < 0, DIFVM_ERR_UNSUPPORTED,
              "solves and PISO steps run on a whole mesh, not on a partition part");
}
static void check_dtype(int dtype) {
  DIFVM_CHECK(dtype == DIFVM_F64 || dtype == DIFVM_F32, DIFVM_ERR_INVALID_ARG, "dtype must be DIFVM_F64 or DIFVM_F32");
}
static void check_ncomp(int ncomp) { DIFVM_CHECK(ncomp == 1 || ncomp == 3, DIFVM_ERR_INVALID_ARG, "ncomp must be 1 or 3"); }
static void check_bc(int bc) { DIFVM_CHECK(bc >= 0 && bc < N_TABLES, DIFVM_ERR_INVALID_ARG, "unknown boundary table"); }
static void check_ptr(const void* p, const char* what) {
  DIFVM_CHECK(p != nullptr, DIFVM_ERR_INVALID_ARG, std::string(what) + " is NULL");
}

template <class T>
static T* up_vec(difvm_mesh* m, const std::vector<T>& v) {
  T* p = dalloc<T>(ctx_of(m), v.size());
  m->allocs.push_back(p);
  upload(p, v, stream_of(m));
  return p;
}

static void upload_mesh(difvm_mesh* m) {
  HostLayout& L = m->host;
  DMesh& d = m->d;
  std::memset(&d, 0, sizeof(d));
  d.nc = L.nc; d.nfi = L.nfi; d.nfb = L.nfb; d.nslice = L.nslice; d.nslot = L.nslot; d.n_wk = L.n_wk;
  d.has_fixed_p = L.has_fixed_p;
  int nfi = L.nfi, nfb = L.nfb;
  std::vector<double4> gS(nfi), gK(nfi), bg(nfb);
  std::vector<float4> gS32(nfi), gK32(nfi), bg32(nfb);
  std::vector<float> w32(nfi), V32(L.nc);
  for (int f = 0; f < nfi; ++f) {
    gS[f] = make_double4(L.S[3 * f], L.S[3 * f + 1], L.S[3 * f + 2], L.w[f]);
    gK[f] = make_double4(L.k[3 * f], L.k[3 * f + 1], L.k[3 * f + 2], L.delta[f]);
    gS32[f] = make_float4((float)gS[f].x, (float)gS[f].y, (float)gS[f].z, (float)gS[f].w);
    gK32[f] = make_float4((float)gK[f].x, (float)gK[f].y, (float)gK[f].z, (float)gK[f].w);
    w32[f] = (float)L.w[f];
  }
  for (int b = 0; b < nfb; ++b) {
    int f = nfi + b;
    bg[b] = make_double4(L.S[3 * f], L.S[3 * f + 1], L.S[3 * f + 2], L.delta[f]);
    bg32[b] = make_float4((float)bg[b].x, (float)bg[b].y, (float)bg[b].z, (float)bg[b].w);
  }
  for (int i = 0; i < L.nc; ++i) V32[i] = (float)L.V[i];
  std::vector<int8_t> codes((size_t)N_TABLES * nfb);
  for (int t = 0; t < N_TABLES; ++t) std::copy(L.bcode[t].begin(), L.bcode[t].end(), codes.begin() + (size_t)t * nfb);
  d.own = up_vec(m, L.owner);
  d.nbr = up_vec(m, L.neighbour);
  d.geomS = up_vec(m, gS);
  d.geomK = up_vec(m, gK);
  d.w = up_vec(m, L.w);
  d.geomS32 = up_vec(m, gS32);
  d.geomK32 = up_vec(m, gK32);
  d.w32 = up_vec(m, w32);
  d.bown = up_vec(m, L.bowner);
  d.bgeom = up_vec(m, bg);
  d.bgeom32 = up_vec(m, bg32);
  d.bcode = up_vec(m, codes);
  d.wk_start = up_vec(m, L.wk_start);
  d.wk_faces = up_vec(m, L.wk_faces);
  d.V = up_vec(m, L.V);
  d.V32 = up_vec(m, V32);
  d.slice_start = up_vec(m, L.slice_start);
  d.slot_face = up_vec(m, L.slot_face);
  d.slot_col = up_vec(m, L.slot_col);
  // the PCG product reads columns as 16-bit offsets from the row when RCM keeps them that close
  // (declared here, like every host array uploaded below, so that it outlives the asynchronous
  // copies until the synchronisation at the end)
  std::vector<int16_t> off(L.slot_col.size(), 0);
  {
    bool fits = true;
    for (int sl = 0; sl < L.nslice && fits; ++sl)
      for (int at = L.slice_start[sl]; at < L.slice_start[sl + 1]; ++at) {
        int row = sl * SLICE + (at - L.slice_start[sl]) % SLICE;
        int o = L.slot_col[at] - row;
        if (row >= L.nc) continue;  // padding rows of the last slice are never read
        if (o < INT16_MIN || o > INT16_MAX) {
          fits = false;
          break;
        }
        off[at] = (int16_t)o;
      }
    d.slot_off16 = fits ? up_vec(m, off) : nullptr;
  }
  d.cell_nslot = up_vec(m, L.cell_nslot);
  // uniform rows: every cell has the same slot count (then slice s starts at slot s * 64 * uw)
  d.uw = 0;
  if (L.nc > 0 && L.cell_nslot[0] > 0 && L.cell_nslot[0] < 255) {
    int c = L.cell_nslot[0];
    bool same = true;
    for (int i = 1; i < L.nc && same; ++i) same = L.cell_nslot[i] == c;
    for (int sl = 0; sl <= L.nslice && same; ++sl) same = L.slice_start[sl] == sl * SLICE * c;
    if (same) d.uw = c;
  }
  d.face_slot_own = up_vec(m, L.face_slot_own);
  d.face_slot_nbr = up_vec(m, L.face_slot_nbr);
  d.nseg = L.nseg;
  d.ntile = (int)L.tile_lo.size();
  d.cell_seg = up_vec(m, L.cell_seg);
  d.tile_lo = up_vec(m, L.tile_lo);
  d.tile_hi = up_vec(m, L.tile_hi);
  d.tile_seg = up_vec(m, L.tile_seg);
  d.seg_tile_first = up_vec(m, L.seg_tile_first);
  d.seg_tile_n = up_vec(m, L.seg_tile_n);
  d.cell_perm = up_vec(m, L.cell_perm);
  d.face_perm = up_vec(m, L.face_perm);
  d.bface_perm = up_vec(m, L.bface_perm);
  d.face_flip = up_vec(m, L.face_flip);
  std::vector<double4> rO(nfi), rN(nfi);
  for (int f = 0; f < nfi; ++f) {
    const double* xf = &L.Cf[3 * f];
    const double* xO = &L.C[3 * L.owner[f]];
    const double* xN = &L.C[3 * L.neighbour[f]];
    rO[f] = make_double4(xf[0] - xO[0], xf[1] - xO[1], xf[2] - xO[2], 0.0);
    rN[f] = make_double4(xf[0] - xN[0], xf[1] - xN[1], xf[2] - xN[2], 0.0);
  }
  d.face_rO = up_vec(m, rO);
  d.face_rN = up_vec(m, rN);
  DIFVM_HIP(hipStreamSynchronize(stream_of(m)));
}

static void ctx_release(difvm_ctx* ctx) {
  if (!ctx || --ctx->refs > 0) return;
  (void)hipStreamSynchronize(ctx->c.stream);
  for (auto& r : ctx->c.prof.pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->c.prof.pool) (void)hipEventDestroy(e);
  delete ctx;
}

static void free_mesh(difvm_mesh* m) {
  if (!m) return;
  if (m->ctx) (void)hipStreamSynchronize(stream_of(m));
  krylov_work_free(m->krylov);
  for (void* a : m->allocs) dfree(ctx_of(m), a);
  difvm_ctx* ctx = m->ctx;
  delete m;
  ctx_release(ctx);
}

double* mesh_scratch(difvm_mesh* m, int slot, size_t n) {
  if (!m->scratch[slot]) {
    m->scratch[slot] = dalloc<double>(ctx_of(m), n);
    m->allocs.push_back(m->scratch[slot]);
  }
  return m->scratch[slot];
}

void mesh_release(difvm_mesh* m) {
  if (m && --m->refs == 0) free_mesh(m);
}

// ---------------------------------------------------------------------------------------------
// Fixed scratch of difvm_ldu_assemble_momentum_noalloc: the velocity gradient (9 doubles per cell)
// of at most DIFVM_NOALLOC_MAX_CELLS cells, in a device array every GPU holds while the library is
// loaded.  Host code never uses the array's name as an address: difvm_ctx_create takes the array's
// device address on its device (hipGetSymbolAddress, once per device, that device current).
// ---------------------------------------------------------------------------------------------
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) double scratch[9 * (size_t)DIFVM_NOALLOC_MAX_CELLS];
static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

static void noalloc_init(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return;  // the entry point refuses such devices
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return;
  void* p = nullptr;
  DIFVM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  DIFVM_CHECK(p != nullptr, DIFVM_ERR_HIP, "hipGetSymbolAddress returned NULL for the fixed scratch");
  g_noalloc_ptr[device] = static_cast<double*>(p);
}

static double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  return (device >= 0 && device < NOALLOC_MAX_DEVICES) ? g_noalloc_ptr[device] : nullptr;
}

}  // namespace difvm

using namespace difvm;

struct difvm_partition {
  HostLayout G;                 // the whole mesh, renumbered, with its cell-slot layout
  std::vector<PartMaps> parts;
};

extern "C" {

int difvm_abi_version(void) { return DIFVM_ABI_VERSION; }
const char* difvm_last_error(void) { return g_last_error.c_str(); }

difvm_status difvm_ctx_create(int device, void* hip_stream, difvm_ctx** out) {
  DIFVM_API_BEGIN
  check_ptr(out, "out");
  int n = 0;
  DIFVM_HIP(hipGetDeviceCount(&n));
  DIFVM_CHECK(device >= 0 && device < n, DIFVM_ERR_INVALID_ARG, "device ordinal out of range");
  DIFVM_HIP(hipSetDevice(device));
  noalloc_init(device);  // device address of the fixed scratch on this device (once per device)
  difvm_ctx* c = new difvm_ctx();
  c->c.device = device;
  c->c.stream = static_cast<hipStream_t>(hip_stream);
  *out = c;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_ctx_set_stream(difvm_ctx* ctx, void* hip_stream) {
  DIFVM_API_BEGIN
  check_ptr(ctx, "ctx");
  ctx->c.stream = static_cast<hipStream_t>(hip_stream);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_ctx_set_allocator(difvm_ctx* ctx, void* (*alloc)(size_t, void*, void*),
                                     void (*free_fn)(void*, void*, void*), void* user) {
  DIFVM_API_BEGIN
  check_ptr(ctx, "ctx");
  DIFVM_CHECK((alloc == nullptr) == (free_fn == nullptr), DIFVM_ERR_INVALID_ARG,
              "alloc and free must both be set or both be NULL");
  // every block must go back to the allocator that made it: no object may hold memory yet
  DIFVM_CHECK(ctx->refs == 1, DIFVM_ERR_INVALID_ARG, "the allocator can only change while no object uses the context");
  ctx->c.alloc = Allocator{alloc, free_fn, alloc ? user : nullptr};
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_ctx_destroy(difvm_ctx* ctx) {
  ctx_release(ctx);
  return DIFVM_OK;
}

difvm_status difvm_ctx_profile(difvm_ctx* ctx, int enable) {
  DIFVM_API_BEGIN
  check_ptr(ctx, "ctx");
  DIFVM_CHECK(enable >= 0, DIFVM_ERR_INVALID_ARG, "enable must be >= 0");
  if (!enable) prof_collect(ctx->c);
  Profiler& P = ctx->c.prof;
  P.on = enable != 0;
  if (enable) {
    P.stride = enable;
    std::fill(P.seen.begin(), P.seen.end(), 0L);
  }
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_ctx_profile_phases(difvm_ctx* ctx, int enable) {
  DIFVM_API_BEGIN
  check_ptr(ctx, "ctx");
  if (!enable) prof_collect(ctx->c);
  ctx->c.prof.phases = enable != 0;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_ctx_profile_read(difvm_ctx* ctx, difvm_kernel_time* out, int32_t max_out, int32_t* n_out) {
  DIFVM_API_BEGIN
  check_ptr(ctx, "ctx");
  check_ptr(n_out, "n_out");
  Profiler& P = ctx->c.prof;
  prof_collect(ctx->c);
  int n = (int)P.names.size();
  *n_out = n;
  for (int k = 0; k < n && k < max_out && out; ++k) {
    std::memset(out[k].name, 0, sizeof(out[k].name));
    std::strncpy(out[k].name, P.names[k].c_str(), sizeof(out[k].name) - 1);
    out[k].launches = (int32_t)P.launches[k];
    out[k].total_ms = P.total_ms[k];
  }
  std::fill(P.total_ms.begin(), P.total_ms.end(), 0.0);
  std::fill(P.launches.begin(), P.launches.end(), 0L);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_mesh_renumber_host(const difvm_mesh_desc* desc, uint32_t flags, int32_t* cell_perm, int32_t* face_perm,
                                      uint8_t* face_flip, int32_t* owner, int32_t* neighbour, int32_t* own_start,
                                      int32_t* losort, int32_t* losort_start, int32_t* bface_perm, int32_t* bowner,
                                      double* S, double* w, double* delta, double* k) {
  DIFVM_API_BEGIN
  HostLayout L;
  build_layout(desc, flags, L, false);
  auto put = [](auto* dst, const auto& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), sizeof(v[0]) * v.size());
  };
  put(cell_perm, L.cell_perm); put(face_perm, L.face_perm); put(face_flip, L.face_flip); put(owner, L.owner);
  put(neighbour, L.neighbour); put(own_start, L.own_start); put(losort, L.losort); put(losort_start, L.losort_start);
  put(bface_perm, L.bface_perm); put(bowner, L.bowner); put(S, L.S); put(w, L.w); put(delta, L.delta); put(k, L.k);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_mesh_create(difvm_ctx* ctx, const difvm_mesh_desc* desc, uint32_t flags, difvm_mesh** out) {
  return difvm_mesh_create_segments(ctx, desc, flags, 1, nullptr, out);
}

difvm_status difvm_mesh_create_segments(difvm_ctx* ctx, const difvm_mesh_desc* desc, uint32_t flags, int32_t n_seg,
                                        const int32_t* seg_cell_start, difvm_mesh** out) {
  DIFVM_API_BEGIN
  difvm_mesh* m = nullptr;
  check_ptr(ctx, "ctx");
  check_ptr(out, "out");
  DIFVM_CHECK(n_seg >= 1, DIFVM_ERR_INVALID_ARG, "n_seg must be >= 1");
  DIFVM_CHECK(n_seg == 1 || seg_cell_start, DIFVM_ERR_INVALID_ARG, "seg_cell_start is NULL");
  DIFVM_HIP(hipSetDevice(ctx->c.device));
  m = new difvm_mesh();
  m->ctx = ctx;
  ctx->refs++;  // released by free_mesh, also on the failure path below
  try {
    build_layout(desc, flags, m->host, true, n_seg, seg_cell_start);
    upload_mesh(m);
  } catch (...) {
    free_mesh(m);
    throw;
  }
  *out = m;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_partition_create(const difvm_mesh_desc* desc, uint32_t flags, int32_t n_parts,
                                    difvm_partition** out) {
  DIFVM_API_BEGIN
  check_ptr(out, "out");
  difvm_partition* P = new difvm_partition();
  try {
    build_layout(desc, flags, P->G, true);
    build_partition(P->G, n_parts, P->parts);
  } catch (...) {
    delete P;
    throw;
  }
  *out = P;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_partition_destroy(difvm_partition* P) {
  delete P;
  return DIFVM_OK;
}

static const PartMaps& part_maps(const difvm_partition* P, int32_t part) {
  DIFVM_CHECK(P != nullptr, DIFVM_ERR_INVALID_ARG, "partition is NULL");
  DIFVM_CHECK(part >= 0 && part < (int32_t)P->parts.size(), DIFVM_ERR_INVALID_ARG, "part out of range");
  return P->parts[part];
}

difvm_status difvm_partition_info(const difvm_partition* P, int32_t part, difvm_part_info* info) {
  DIFVM_API_BEGIN
  const PartMaps& M = part_maps(P, part);
  check_ptr(info, "info");
  info->n_parts = (int32_t)P->parts.size();
  info->cell_lo = M.lo;
  info->cell_hi = M.hi;
  info->n_owned = M.n_owned;
  info->n_ghost = M.n_ghost;
  info->n_internal_faces = (int32_t)M.face_global.size();
  info->n_boundary_faces = (int32_t)M.bface_global.size();
  info->n_send = (int32_t)M.send_cells.size();
  int nb = 0;
  for (size_t q = 0; q + 1 < M.recv_start.size(); ++q)
    nb += (M.recv_start[q + 1] > M.recv_start[q] || M.send_start[q + 1] > M.send_start[q]) ? 1 : 0;
  info->n_neighbours = nb;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_partition_maps(const difvm_partition* P, int32_t part, int32_t* cell_global, int32_t* face_global,
                                  int32_t* bface_global, int32_t* recv_start, int32_t* send_start, int32_t* send_cells) {
  DIFVM_API_BEGIN
  const PartMaps& M = part_maps(P, part);
  auto put = [](int32_t* dst, const std::vector<int32_t>& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), sizeof(int32_t) * v.size());
  };
  put(cell_global, M.cell_global); put(face_global, M.face_global); put(bface_global, M.bface_global);
  put(recv_start, M.recv_start); put(send_start, M.send_start); put(send_cells, M.send_cells);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_mesh_create_part(difvm_ctx* ctx, const difvm_partition* P, int32_t part, difvm_mesh** out) {
  DIFVM_API_BEGIN
  const PartMaps& M = part_maps(P, part);
  check_ptr(ctx, "ctx");
  check_ptr(out, "out");
  DIFVM_HIP(hipSetDevice(ctx->c.device));
  difvm_mesh* m = new difvm_mesh();
  m->ctx = ctx;
  ctx->refs++;  // released by free_mesh, also on the failure path below
  try {
    build_part_layout(P->G, M, m->host);
    upload_mesh(m);
    m->part_n_owned = M.n_owned;
    m->part_n_ghost = M.n_ghost;
    m->part_n_send = (int)M.send_cells.size();
    m->part_send = up_vec(m, M.send_cells);
    DIFVM_HIP(hipStreamSynchronize(stream_of(m)));
  } catch (...) {
    free_mesh(m);
    throw;
  }
  *out = m;
  DIFVM_API_END
  return DIFVM_OK;
}

static void check_part(const difvm_mesh* m) {
  check_mesh(m);
  DIFVM_CHECK(m->part_n_owned >= 0, DIFVM_ERR_INVALID_ARG, "the mesh is not a partition part");
}

difvm_status difvm_halo_pack(const difvm_mesh* m, int dtype, int ncomp, const void* x, void* send_buf) {
  DIFVM_API_BEGIN
  check_part(m); check_dtype(dtype);
  DIFVM_CHECK(ncomp >= 1 && ncomp <= 9, DIFVM_ERR_INVALID_ARG, "ncomp must be in 1..9");
  if (m->part_n_send) { check_ptr(x, "x"); check_ptr(send_buf, "send_buf"); }
  op_halo_pack(m, dtype, ncomp, x, send_buf);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_halo_unpack(const difvm_mesh* m, int dtype, int ncomp, const void* recv_buf, void* x) {
  DIFVM_API_BEGIN
  check_part(m); check_dtype(dtype);
  DIFVM_CHECK(ncomp >= 1 && ncomp <= 9, DIFVM_ERR_INVALID_ARG, "ncomp must be in 1..9");
  if (m->part_n_ghost) { check_ptr(x, "x"); check_ptr(recv_buf, "recv_buf"); }
  op_halo_unpack(m, dtype, ncomp, recv_buf, x);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_mesh_get_info(const difvm_mesh* m, difvm_mesh_info* info) {
  DIFVM_API_BEGIN
  check_mesh(m);
  check_ptr(info, "info");
  const HostLayout& L = m->host;
  info->n_cells = L.nc;
  info->n_internal_faces = L.nfi;
  info->n_boundary_faces = L.nfb;
  info->n_patches = L.npatch;
  info->n_slices = L.nslice;
  info->n_slots = L.nslot;
  info->bandwidth_in = L.bandwidth_in;
  info->bandwidth_out = L.bandwidth_out;
  info->n_windkessel = L.n_wk;
  info->has_fixed_p = L.has_fixed_p ? 1 : 0;
  info->n_segments = L.nseg;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_mesh_destroy(difvm_mesh* m) {
  DIFVM_API_BEGIN
  mesh_release(m);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_permute(const difvm_mesh* m, int dtype, int ncomp, int kind, int dir, const void* src, void* dst) {
  DIFVM_API_BEGIN
  check_mesh(m); check_dtype(dtype);
  DIFVM_CHECK(ncomp >= 1 && ncomp <= 9, DIFVM_ERR_INVALID_ARG, "ncomp must be in 1..9");
  DIFVM_CHECK(kind >= DIFVM_KIND_CELL && kind <= DIFVM_KIND_BFACE, DIFVM_ERR_INVALID_ARG, "unknown kind");
  DIFVM_CHECK(dir == DIFVM_TO_INTERNAL || dir == DIFVM_FROM_INTERNAL, DIFVM_ERR_INVALID_ARG, "unknown direction");
  check_ptr(src, "src"); check_ptr(dst, "dst");
  DIFVM_CHECK(src != dst, DIFVM_ERR_INVALID_ARG, "src and dst must differ");
  permute(m, dtype, ncomp, kind, dir, src, dst);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_op_interp(const difvm_mesh* m, int dtype, int ncomp, int bc, const void* phi, const void* phi_b,
                             void* phi_f) {
  DIFVM_API_BEGIN
  check_mesh(m); check_dtype(dtype); check_ncomp(ncomp); check_bc(bc);
  check_ptr(phi, "phi"); check_ptr(phi_f, "phi_f");
  DIFVM_CHECK(phi_b || bc == DIFVM_BC_ALL_ZEROGRAD || m->d.nfb == 0, DIFVM_ERR_INVALID_ARG, "phi_b is NULL");
  op_interp(m, dtype, ncomp, bc, phi, phi_b, phi_f);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_op_grad(const difvm_mesh* m, int dtype, int ncomp, int bc, const void* phi, const void* phi_b,
                           void* grad) {
  DIFVM_API_BEGIN
  check_mesh(m); check_dtype(dtype); check_ncomp(ncomp); check_bc(bc);
  check_ptr(phi, "phi"); check_ptr(grad, "grad");
  DIFVM_CHECK(phi_b || bc == DIFVM_BC_ALL_ZEROGRAD || m->d.nfb == 0, DIFVM_ERR_INVALID_ARG, "phi_b is NULL");
  op_grad(m, dtype, ncomp, bc, phi, phi_b, grad);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_op_div(const difvm_mesh* m, int dtype, int scheme, int ncomp, int bc, const void* flux,
                          const void* psi, const void* psi_b, void* out) {
  DIFVM_API_BEGIN
  check_mesh(m); check_dtype(dtype); check_ncomp(ncomp); check_bc(bc);
  DIFVM_CHECK(scheme >= DIFVM_SCHEME_ONE && scheme <= DIFVM_SCHEME_LINEAR, DIFVM_ERR_INVALID_ARG, "unknown scheme");
  check_ptr(flux, "flux"); check_ptr(out, "out");
  if (scheme != DIFVM_SCHEME_ONE) {
    check_ptr(psi, "psi");
    DIFVM_CHECK(psi_b || bc == DIFVM_BC_ALL_ZEROGRAD || m->d.nfb == 0, DIFVM_ERR_INVALID_ARG, "psi_b is NULL");
  }
  op_div(m, dtype, scheme, ncomp, bc, flux, psi, psi_b, out);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_op_deferred_correction(const difvm_mesh* m, int dtype, int conv, int ncomp, const void* flux,
                                          const void* phi, const void* grad, void* out) {
  DIFVM_API_BEGIN
  check_mesh(m); check_dtype(dtype); check_ncomp(ncomp);
  DIFVM_CHECK(dtype == DIFVM_F64, DIFVM_ERR_UNSUPPORTED, "deferred correction is F64 only");
  DIFVM_CHECK(conv >= DIFVM_CONV_UPWIND && conv <= DIFVM_CONV_QUICK, DIFVM_ERR_INVALID_ARG, "unknown convection scheme");
  check_ptr(out, "out");
  if (conv != DIFVM_CONV_UPWIND) { check_ptr(flux, "flux"); check_ptr(phi, "phi"); check_ptr(grad, "grad"); }
  op_deferred_correction(m, conv, ncomp, (const double*)flux, (const double*)phi, (const double*)grad, (double*)out);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_op_laplacian(const difvm_mesh* m, int dtype, int bc, const void* gamma_f, const void* phi,
                                const void* grad_phi, const void* phi_b, void* out) {
  DIFVM_API_BEGIN
  check_mesh(m); check_dtype(dtype); check_bc(bc);
  check_ptr(phi, "phi"); check_ptr(grad_phi, "grad_phi"); check_ptr(out, "out");
  DIFVM_CHECK(phi_b || bc == DIFVM_BC_ALL_ZEROGRAD || m->d.nfb == 0, DIFVM_ERR_INVALID_ARG, "phi_b is NULL");
  op_laplacian(m, dtype, bc, gamma_f, phi, grad_phi, phi_b, out);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_ldu_spmv(const difvm_mesh* m, int ncomp, int transpose, const difvm_ldu* A, const void* x, void* y) {
  DIFVM_API_BEGIN
  check_mesh(m); check_ncomp(ncomp); check_ptr(A, "A");
  check_dtype(A->dtype);
  check_ptr(A->diag, "A->diag"); check_ptr(x, "x"); check_ptr(y, "y");
  DIFVM_CHECK(A->upper || m->d.nfi == 0, DIFVM_ERR_INVALID_ARG, "A->upper is NULL");
  DIFVM_CHECK(x != y, DIFVM_ERR_INVALID_ARG, "x and y must differ");
  op_ldu_spmv(m, A->dtype, ncomp, transpose, A->diag, A->upper, A->lower, x, y);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_ldu_assemble_laplace(const difvm_mesh* m, int bc, const void* gamma_f, const void* phi_b, difvm_ldu* A,
                                        void* rhs_bc) {
  DIFVM_API_BEGIN
  check_mesh(m); check_bc(bc); check_ptr(A, "A");
  DIFVM_CHECK(A->dtype == DIFVM_F64, DIFVM_ERR_UNSUPPORTED, "assembly is F64 only");
  check_ptr(A->diag, "A->diag");
  DIFVM_CHECK(A->upper || m->d.nfi == 0, DIFVM_ERR_INVALID_ARG, "A->upper is NULL");
  DIFVM_CHECK(phi_b || !rhs_bc, DIFVM_ERR_INVALID_ARG, "rhs_bc needs phi_b");
  op_assemble_laplace(m, bc, (const double*)gamma_f, (const double*)phi_b, (double*)A->diag, (double*)A->upper,
                      (double*)rhs_bc);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_ldu_assemble_momentum(const difvm_mesh* m, double nu, double dt, const void* flux, const void* U,
                                         const void* U_b, difvm_ldu* A, void* b) {
  DIFVM_API_BEGIN
  check_mesh(m); check_ptr(A, "A"); check_ptr(flux, "flux"); check_ptr(U, "U"); check_ptr(b, "b");
  DIFVM_CHECK(A->dtype == DIFVM_F64, DIFVM_ERR_UNSUPPORTED, "assembly is F64 only");
  check_ptr(A->diag, "A->diag");
  DIFVM_CHECK((A->upper && A->lower) || m->d.nfi == 0, DIFVM_ERR_INVALID_ARG, "A->upper or A->lower is NULL");
  DIFVM_CHECK(dt > 0, DIFVM_ERR_INVALID_ARG, "dt must be > 0");
  DIFVM_CHECK(U_b || m->d.nfb == 0, DIFVM_ERR_INVALID_ARG, "U_b is NULL");
  // the gradient of U lives in mesh scratch: no allocation after the first call
  double* gU = mesh_scratch(const_cast<difvm_mesh*>(m), 1, (size_t)9 * m->d.nc);
  op_grad(m, DIFVM_F64, 3, DIFVM_BC_U, U, U_b, gU);
  op_assemble_momentum(m, DIFVM_CONV_UPWIND, DIFVM_TIME_BACKWARD_EULER, nu, nullptr, dt, (const double*)flux,
                       (const double*)U, gU, (const double*)U_b, (double*)A->diag, (double*)A->upper,
                       (double*)A->lower, nullptr, (double*)b);
  DIFVM_HIP(hipStreamSynchronize(stream_of(m)));
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_ldu_assemble_momentum_noalloc(const difvm_mesh* m, double nu, double dt, const void* flux,
                                                 const void* U, const void* U_b, difvm_ldu* A, void* b) {
  DIFVM_API_BEGIN
  check_mesh(m); check_ptr(A, "A"); check_ptr(flux, "flux"); check_ptr(U, "U"); check_ptr(b, "b");
  DIFVM_CHECK(A->dtype == DIFVM_F64, DIFVM_ERR_UNSUPPORTED, "assembly is F64 only");
  check_ptr(A->diag, "A->diag");
  DIFVM_CHECK((A->upper && A->lower) || m->d.nfi == 0, DIFVM_ERR_INVALID_ARG, "A->upper or A->lower is NULL");
  DIFVM_CHECK(dt > 0, DIFVM_ERR_INVALID_ARG, "dt must be > 0");
  DIFVM_CHECK(U_b || m->d.nfb == 0, DIFVM_ERR_INVALID_ARG, "U_b is NULL");
  DIFVM_CHECK(m->d.nc <= DIFVM_NOALLOC_MAX_CELLS, DIFVM_ERR_INVALID_ARG,
              "difvm_ldu_assemble_momentum_noalloc: the mesh has " + std::to_string(m->d.nc) +
                  " cells, more than the fixed scratch holds (DIFVM_NOALLOC_MAX_CELLS = " +
                  std::to_string(DIFVM_NOALLOC_MAX_CELLS) + ")");
  double* gU = noalloc_scratch(ctx_of(m).device);
  DIFVM_CHECK(gU != nullptr, DIFVM_ERR_INVALID_ARG, "no fixed scratch on the mesh's device (ordinal >= 64)");
  // the gradient is written in full before the assembly reads it: nothing to clear
  op_grad(m, DIFVM_F64, 3, DIFVM_BC_U, U, U_b, gU);
  op_assemble_momentum(m, DIFVM_CONV_UPWIND, DIFVM_TIME_BACKWARD_EULER, nu, nullptr, dt, (const double*)flux,
                       (const double*)U, gU, (const double*)U_b, (double*)A->diag, (double*)A->upper,
                       (double*)A->lower, nullptr, (double*)b);
  DIFVM_HIP(hipStreamSynchronize(stream_of(m)));
  DIFVM_API_END
  return DIFVM_OK;
}

static difvm_status solve_common(const difvm_mesh* cm, const difvm_ldu* A, int ncomp, const void* b, void* x, double tol,
                                 int32_t maxit, difvm_solve_stats* stats, bool sym, const AmgDev* amg = nullptr) {
  difvm_mesh* m = const_cast<difvm_mesh*>(cm);
  check_mesh(m); check_ptr(A, "A"); check_ptr(b, "b"); check_ptr(x, "x"); check_ncomp(ncomp);
  check_whole(m);
  DIFVM_CHECK(A->dtype == DIFVM_F64, DIFVM_ERR_UNSUPPORTED, "solvers are F64 only");
  check_ptr(A->diag, "A->diag");
  DIFVM_CHECK(A->upper || m->d.nfi == 0, DIFVM_ERR_INVALID_ARG, "A->upper is NULL");
  DIFVM_CHECK(tol >= 0 && maxit >= 0, DIFVM_ERR_INVALID_ARG, "tol and maxit must be >= 0");
  // the cell-slot copy of the matrix lives in mesh scratch: no allocation after the first call
  double* val = mesh_scratch(m, 0, m->d.nslot);
  SolveResult R;
  sell_from_ldu(m, (const double*)A->upper, sym ? nullptr : (const double*)A->lower, val);
  SellMatrix S{(const double*)A->diag, val};
  int* hint = &m->abi_hint[sym ? (amg ? 1 : 0) : 2];
  if (sym) R = pcg(m, S, (const double*)b, (double*)x, tol, maxit, nullptr, amg, hint);
  else R = bicgstab(m, ncomp, S, (const double*)b, (double*)x, tol, maxit, nullptr, hint);
  if (stats) {
    for (int c = 0; c < 3; ++c) { stats->iters[c] = R.iters[c]; stats->residual[c] = R.res[c]; }
    stats->status = R.status;
  }
  return R.status;
}

difvm_status difvm_solve_pcg(const difvm_mesh* m, const difvm_ldu* A, const void* b, void* x, double tol, int32_t maxit,
                             difvm_solve_stats* stats) {
  DIFVM_API_BEGIN
  return solve_common(m, A, 1, b, x, tol, maxit, stats, true);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_solve_bicgstab(const difvm_mesh* m, const difvm_ldu* A, int ncomp, const void* b, void* x, double tol,
                                  int32_t maxit, difvm_solve_stats* stats) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(A && (A->lower || (m && m->d.nfi == 0)), DIFVM_ERR_INVALID_ARG, "BiCGStab needs A->lower");
  return solve_common(m, A, ncomp, b, x, tol, maxit, stats, false);
  DIFVM_API_END
  return DIFVM_OK;
}

}  // extern "C"

struct difvm_amg {
  difvm_mesh* mesh = nullptr;
  AmgDev* dev = nullptr;
  double *diag = nullptr, *val = nullptr;  // the matrix the hierarchy was built from (cell-slot form)
};

static void amg_release(difvm_amg* a) {
  if (!a) return;
  amg_free(a->dev);
  dfree(ctx_of(a->mesh), a->diag);
  dfree(ctx_of(a->mesh), a->val);
  difvm_mesh* m = a->mesh;
  delete a;
  mesh_release(m);
}

static void check_sym_ldu(const difvm_mesh* m, const difvm_ldu* A) {
  check_ptr(A, "A");
  DIFVM_CHECK(A->dtype == DIFVM_F64, DIFVM_ERR_UNSUPPORTED, "solvers are F64 only");
  check_ptr(A->diag, "A->diag");
  DIFVM_CHECK(A->upper || m->d.nfi == 0, DIFVM_ERR_INVALID_ARG, "A->upper is NULL");
}

extern "C" {

difvm_status difvm_amg_create(const difvm_mesh* cm, const difvm_ldu* A, difvm_amg** out) {
  DIFVM_API_BEGIN
  check_mesh(cm); check_ptr(out, "out");
  check_whole(cm);
  difvm_mesh* m = const_cast<difvm_mesh*>(cm);
  check_sym_ldu(m, A);
  difvm_amg* a = new difvm_amg();
  try {
    a->diag = dalloc<double>(ctx_of(m), m->d.nc);
    a->val = dalloc<double>(ctx_of(m), m->d.nslot);
    DIFVM_HIP(hipMemcpyAsync(a->diag, A->diag, sizeof(double) * m->d.nc, hipMemcpyDeviceToDevice, stream_of(m)));
    sell_from_ldu(m, (const double*)A->upper, nullptr, a->val);
    a->dev = amg_create(m, SellMatrix{a->diag, a->val}, AmgOptions{});
  } catch (...) {
    amg_free(a->dev);
    dfree(ctx_of(m), a->diag);
    dfree(ctx_of(m), a->val);
    delete a;
    throw;
  }
  a->mesh = m;
  m->refs++;
  *out = a;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_amg_setup_host(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, const double* diag,
                                  int32_t* agg, int32_t* rows, int32_t cap, int32_t* n_levels) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(n > 0 && ptr && diag && (ptr[n] == 0 || (col && val)), DIFVM_ERR_INVALID_ARG, "bad CSR matrix");
  DIFVM_CHECK(cap >= 0 && (rows || cap == 0), DIFVM_ERR_INVALID_ARG, "rows is NULL");
  AmgCsr A;
  A.n = n;
  A.ptr.assign(ptr, ptr + n + 1);
  DIFVM_CHECK(A.ptr[0] == 0, DIFVM_ERR_INVALID_ARG, "ptr[0] must be 0");
  for (int i = 0; i < n; ++i) DIFVM_CHECK(A.ptr[i + 1] >= A.ptr[i], DIFVM_ERR_INVALID_ARG, "ptr must not decrease");
  A.col.assign(col, col + A.ptr[n]);
  A.val.assign(val, val + A.ptr[n]);
  A.diag.assign(diag, diag + n);
  for (int i = 0; i < n; ++i) {
    DIFVM_CHECK(A.diag[i] > 0.0, DIFVM_ERR_INVALID_ARG, "AMG needs a matrix with a positive diagonal");
    for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
      DIFVM_CHECK(A.col[q] >= 0 && A.col[q] < n && A.col[q] != i, DIFVM_ERR_INVALID_ARG, "column out of range or on the diagonal");
  }
  AmgHierarchy H;
  try {
    amg_build(A, AmgOptions{}, H);
  } catch (const AmgError& e) {
    throw Error{DIFVM_ERR_UNSUPPORTED, "AMG setup: " + e.msg};
  }
  if (agg) std::copy(H.agg0.begin(), H.agg0.end(), agg);
  int nl = (int)H.levels.size() + 1;
  for (int l = 0; l < nl && l < cap; ++l) rows[l] = l == 0 ? n : H.coarse[l - 1].n;
  if (n_levels) *n_levels = nl;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_amg_destroy(difvm_amg* amg) {
  DIFVM_API_BEGIN
  amg_release(amg);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_amg_levels(const difvm_amg* amg, int32_t* rows, int32_t cap, int32_t* n_levels) {
  DIFVM_API_BEGIN
  check_ptr(amg, "amg");
  DIFVM_CHECK(cap >= 0 && (rows || cap == 0), DIFVM_ERR_INVALID_ARG, "rows is NULL");
  std::vector<int> r(64);
  int n = amg_levels(amg->dev, r.data(), 64);
  for (int l = 0; l < n && l < cap; ++l) rows[l] = r[l];
  if (n_levels) *n_levels = n;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_amg_apply(difvm_amg* amg, const void* r, void* z) {
  DIFVM_API_BEGIN
  check_ptr(amg, "amg"); check_ptr(r, "r"); check_ptr(z, "z");
  DIFVM_CHECK(r != z, DIFVM_ERR_INVALID_ARG, "r and z must differ");
  amg_vcycle(amg->dev, SellMatrix{amg->diag, amg->val}, (const double*)r, (double*)z, nullptr, nullptr);
  DIFVM_HIP(hipStreamSynchronize(stream_of(amg->mesh)));
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_solve_pcg_amg(difvm_amg* amg, const difvm_ldu* A, const void* b, void* x, double tol, int32_t maxit,
                                 difvm_solve_stats* stats) {
  DIFVM_API_BEGIN
  check_ptr(amg, "amg");
  return solve_common(amg->mesh, A, 1, b, x, tol, maxit, stats, true, amg->dev);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_rebuild_preconditioner(difvm_piso* piso) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  piso_rebuild_preconditioner(piso);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_create(const difvm_mesh* m, const difvm_piso_params* params, difvm_piso** out) {
  DIFVM_API_BEGIN
  check_mesh(m); check_ptr(params, "params"); check_ptr(out, "out");
  check_whole(m);
  piso_create(const_cast<difvm_mesh*>(m), params, out);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_destroy(difvm_piso* piso) {
  DIFVM_API_BEGIN
  piso_release(piso);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_set_boundary(difvm_piso* piso, const void* U_b, const void* p_b) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  piso_set_boundary(piso, (const double*)U_b, (const double*)p_b);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_set_windkessel(difvm_piso* piso, int32_t id, double Rp, double C, double Rd, double pc) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  piso_set_windkessel(piso, id, Rp, C, Rd, pc);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_set_state(difvm_piso* piso, const void* U, const void* p, const void* phi) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  piso_set_state(piso, (const double*)U, (const double*)p, (const double*)phi);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_set_viscosity(difvm_piso* piso, int32_t n_seg, const double* nu_seg) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  check_ptr(nu_seg, "nu_seg");
  piso_set_viscosity(piso, n_seg, nu_seg);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_segment_stats(const difvm_piso* piso, int32_t n_seg, difvm_step_stats* out_host) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  check_ptr(out_host, "out_host");
  piso_segment_stats(piso, n_seg, out_host);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_transport_scalar(difvm_piso* piso, double D, int32_t bc, const void* c_b, void* c,
                                         difvm_solve_stats* stats) {
  int status = 0;
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  check_ptr(c, "c");
  SolveResult r = piso_transport_scalar(piso, D, bc, (const double*)c_b, (double*)c);
  if (stats) {
    *stats = difvm_solve_stats{};
    stats->iters[0] = r.iters[0];
    stats->residual[0] = r.res[0];
    stats->status = r.status;
  }
  status = r.status;
  DIFVM_API_END
  return (difvm_status)status;
}

difvm_status difvm_piso_set_graph(difvm_piso* piso, int32_t enable, int32_t extra_iters) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  piso_set_graph(piso, enable, extra_iters);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_graph_info(const difvm_piso* piso, int64_t* replays, int64_t* redos, int64_t* captures) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  long long r = 0, d = 0, c = 0;
  piso_graph_info(piso, &r, &d, &c);
  if (replays) *replays = r;
  if (redos) *redos = d;
  if (captures) *captures = c;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_get_state(difvm_piso* piso, void* U, void* p, void* phi, double* pc_host) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  piso_get_state(piso, (double*)U, (double*)p, (double*)phi, pc_host);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_step(difvm_piso* piso, int32_t nsteps, difvm_step_stats* stats_host) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  DIFVM_CHECK(nsteps >= 0, DIFVM_ERR_INVALID_ARG, "nsteps must be >= 0");
  return piso_step(piso, nsteps, stats_host);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_precond_info(const difvm_piso* piso, int32_t* n_levels, int32_t* rows, int32_t cap,
                                     double* vcycle_bytes) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  check_ptr(n_levels, "n_levels");
  DIFVM_CHECK(cap >= 0 && (rows || cap == 0), DIFVM_ERR_INVALID_ARG, "rows is NULL");
  piso_precond_info(piso, n_levels, rows, cap, vcycle_bytes);
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_piso_step_trace(difvm_piso* piso, void* U_star, void* p_corr, difvm_step_stats* stats_host) {
  DIFVM_API_BEGIN
  check_ptr(piso, "piso");
  check_ptr(U_star, "U_star");
  check_ptr(p_corr, "p_corr");
  return piso_step_trace(piso, (double*)U_star, (double*)p_corr, stats_host);
  DIFVM_API_END
  return DIFVM_OK;
}

}  // extern "C"
