// Internal definitions of libdifvm: mesh and context objects, error plumbing, launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/difvm.h"
#include "layout.h"

namespace difvm {

// ---------------------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------------------
void set_error(const std::string& msg);

struct Error {
  difvm_status code;
  std::string msg;
};

#define DIFVM_HIP(call)                                                                              \
  do {                                                                                               \
    hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess)                                                                            \
      throw ::difvm::Error{DIFVM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)};        \
  } while (0)

#define DIFVM_CHECK(cond, code, msg)                     \
  do {                                                   \
    if (!(cond)) throw ::difvm::Error{(code), (msg)};    \
  } while (0)

// ---------------------------------------------------------------------------------------------
// device-side allocations
// ---------------------------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// event-pair timing of selected kernel launches (difvm_ctx_profile)
struct Profiler {
  bool on = false;
  bool phases = false;        // time the phases of each eager PISO step (scope names "step: ...")
  int stride = 1;             // time every stride-th launch of each kernel name
  std::vector<long> seen;     // launches per name since profiling was enabled
  struct Rec {
    int id;
    hipEvent_t a, b;
    long iter;  // CG iteration of the launch (-1: none)
  };
  std::vector<std::string> names;
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::vector<double> total_ms;
  std::vector<long> launches;
};

// device memory of the library: the caller's allocator (difvm_ctx_set_allocator) or hipMalloc/hipFree
struct Allocator {
  void* (*alloc)(size_t bytes, void* stream, void* user) = nullptr;
  void (*free)(void* p, void* stream, void* user) = nullptr;
  void* user = nullptr;
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Profiler prof;
  bool capturing = false;  // a step is being captured: launches are not timed
  Allocator alloc;
};

// Brackets the next launch on `s` with events when profiling is on; returns a handle for prof_end.
int prof_begin(Ctx& c, const char* name, long iter = -1);
void prof_end(Ctx& c, int handle);
// Timed launches recorded since pending index `from` with an iteration past `last` (queued after the
// CG stopped, they returned at once) are moved to "<name> (idle)".
void prof_idle_after(Ctx& c, size_t from, long last);

// every device allocation of the library goes through its context's allocator
void* dmalloc(const Ctx& c, size_t bytes);
void dfree(const Ctx& c, void* p);
template <class T>
T* dalloc(const Ctx& c, size_t n) {
  return static_cast<T*>(dmalloc(c, sizeof(T) * (n ? n : 1)));
}
template <class T>
void upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (!src.empty()) DIFVM_HIP(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s));
}

// device mesh
struct DMesh {
  int nc, nfi, nfb, nslice, nslot, n_wk;
  bool has_fixed_p;
  // internal faces, owner-sorted
  int32_t *own, *nbr;
  double4* geomS;   // (Sx, Sy, Sz, w)
  double4* geomK;   // (kx, ky, kz, delta)
  double* w;
  float4 *geomS32, *geomK32;
  float* w32;
  // boundary faces
  int32_t* bown;
  double4* bgeom;   // (Sx, Sy, Sz, delta_b)
  float4* bgeom32;
  int8_t* bcode;    // [N_TABLES][nfb]
  int32_t *wk_start, *wk_faces;
  // cells
  double* V;
  float* V32;
  // cell-slot layout (SELL, slices of 64 cells, slot-major inside a slice)
  int32_t *slice_start, *slot_face, *slot_col;
  int16_t* slot_off16;  // slot_col - row as 16 bits, or NULL when some offset does not fit
  uint8_t* cell_nslot;
  int uw;               // > 0: every cell has exactly uw slots (uniform rows), else 0
  int32_t *face_slot_own, *face_slot_nbr;
  // segments and reduction tiles
  int nseg, ntile;
  int32_t *cell_seg, *tile_lo, *tile_hi, *tile_seg, *seg_tile_first, *seg_tile_n;
  // permutations for user <-> internal conversions
  int32_t *cell_perm, *face_perm, *bface_perm;
  uint8_t* face_flip;
  // internal faces: x_f - x_O and x_f - x_N (w unused), for the higher-order convection schemes
  double4 *face_rO, *face_rN;
};

}  // namespace difvm

// Handles are reference counted: a mesh holds its context, a PISO object its mesh, a tape its PISO
// object.  *_destroy drops the caller's reference; the object is freed when none is left.
struct difvm_ctx {
  difvm::Ctx c;
  int refs = 1;
};

namespace difvm {
struct KrylovWork;
}
struct difvm_mesh {
  difvm_ctx* ctx;
  difvm::HostLayout host;
  difvm::DMesh d;
  std::vector<void*> allocs;                 // device allocations owned by the mesh
  difvm::KrylovWork* krylov = nullptr;       // solver workspace, created on first solve
  double* scratch[2] = {nullptr, nullptr};   // entry-point scratch (slot matrix; 3-component gradient)
  int abi_hint[3] = {0, 0, 0};               // iterations of the last difvm_solve_pcg / _pcg_amg / _bicgstab
  int refs = 1;
  int tune[DIFVM_TUNE_COUNT] = {256, 256, 256, 256, 256, 256, 256, 256, 256, 256, 0};  // launch knobs
  // part of a slab partition (difvm_mesh_create_part): owned cells first, then ghosts; n_owned < 0
  // for a whole mesh
  int part_n_owned = -1, part_n_ghost = 0, part_n_send = 0;
  int32_t* part_send = nullptr;              // device: local indices of the owned cells sent
};

namespace difvm {
inline hipStream_t stream_of(const difvm_mesh* m) { return m->ctx->c.stream; }
void mesh_release(difvm_mesh* m);  // drops one reference (frees at zero)
inline Ctx& ctx_of(const difvm_mesh* m) { return m->ctx->c; }
// scratch buffer `slot` of the mesh (n doubles), allocated at its first use and kept with the mesh
double* mesh_scratch(difvm_mesh* m, int slot, size_t n);
// RAII event bracket around one launch
// consecutive timed phases: next() ends the current one and starts another; the destructor ends the
// last (also when an exception leaves the scope, so no record is left without its end event)
struct PhaseScope {
  Ctx& c;
  int h;
  PhaseScope(const difvm_mesh* m, const char* name) : c(ctx_of(m)), h(prof_begin(ctx_of(m), name)) {}
  void next(const char* name) {
    prof_end(c, h);
    h = prof_begin(c, name);
  }
  void end() {
    prof_end(c, h);
    h = -1;
  }
  ~PhaseScope() { prof_end(c, h); }
};

struct ProfScope {
  Ctx& c;
  int h;
  ProfScope(const difvm_mesh* m, const char* name, long iter = -1)
      : c(ctx_of(m)), h(prof_begin(ctx_of(m), name, iter)) {}
  ~ProfScope() { prof_end(c, h); }
};
inline int grid_for(int n, int per_block = BLOCK) { return (n + per_block - 1) / per_block; }
}  // namespace difvm
