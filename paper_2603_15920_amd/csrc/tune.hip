// Launch tuning of libdifvm: per-mesh knobs (threads per block of the operator kernels, grid of the
// PCG product kernel) that change how work is spread over the GPU but never what is computed, and
// an autotuner that times the candidates with HIP events and caches the choices in a JSON file
// keyed by GPU architecture, knob and mesh size bucket.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "abi_util.h"
#include "device.h"
#include "ops.h"

namespace difvm {

double time_pcg_spmv(difvm_mesh* m, int grid, int reps, hipEvent_t e0, hipEvent_t e1);  // krylov.hip

static const char* const KNOB_NAME[DIFVM_TUNE_COUNT] = {
    "interp_f64", "interp_f32", "grad_f64", "grad_f32", "div_f64", "div_f32",
    "laplacian_f64", "laplacian_f32", "ldu_spmv_f64", "ldu_spmv_f32", "pcg_grid"};

static bool op_knob(int k) { return k >= 0 && k < DIFVM_TUNE_PCG_GRID; }

void check_launch(int knob, int value) {
  DIFVM_CHECK(knob >= 0 && knob < DIFVM_TUNE_COUNT, DIFVM_ERR_INVALID_ARG, "unknown tuning knob");
  if (op_knob(knob))
    DIFVM_CHECK(value == 64 || value == 128 || value == 256 || value == 512, DIFVM_ERR_INVALID_ARG,
                "threads per block must be 64, 128, 256 or 512");
  else
    DIFVM_CHECK(value == 0 || (value > 0 && value % 8 == 0), DIFVM_ERR_INVALID_ARG,
                "PCG grid must be 0 or a positive multiple of 8");
}

template <class T>
__global__ void k_fill(T* __restrict__ a, size_t n, T v) {
  size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) a[q] = v;
}

// scratch inputs of one precision for timing the operator kernels (values 1, never read back)
struct Scratch {
  void *phi = nullptr, *phib = nullptr, *flux = nullptr, *g = nullptr, *out = nullptr, *diag = nullptr, *up = nullptr;
  std::vector<void*> all;
  const Ctx* ctx;
  explicit Scratch(const Ctx& c) : ctx(&c) {}
  ~Scratch() {
    for (void* a : all) dfree(*ctx, a);
  }
  template <class T>
  void* make(size_t n, hipStream_t s) {
    T* a = dalloc<T>(*ctx, n);
    all.push_back(a);
    size_t m = n ? n : 1;
    k_fill<T><<<(unsigned)((m + 255) / 256), 256, 0, s>>>(a, m, T(1));
    DIFVM_HIP(hipGetLastError());
    return a;
  }
  template <class T>
  void init(const DMesh& d, hipStream_t s) {
    size_t nc = d.nc, nf = (size_t)d.nfi + d.nfb;
    phi = make<T>(3 * nc, s);
    phib = make<T>(3 * (size_t)d.nfb, s);
    flux = make<T>(nf, s);
    g = make<T>(3 * nc, s);
    out = make<T>(std::max(9 * nc, 3 * nf), s);
    diag = make<T>(nc, s);
    up = make<T>(std::max<size_t>(1, d.nfi), s);
  }
};

static void run_op(difvm_mesh* m, int knob, const Scratch& S) {
  int dt = (knob & 1) ? DIFVM_F32 : DIFVM_F64;
  switch (knob >> 1) {
    case 0: op_interp(m, dt, 1, DIFVM_BC_ALL_FIXED, S.phi, S.phib, S.out); break;
    case 1: op_grad(m, dt, 1, DIFVM_BC_ALL_FIXED, S.phi, S.phib, S.out); break;
    case 2: op_div(m, dt, DIFVM_SCHEME_UPWIND, 3, DIFVM_BC_ALL_FIXED, S.flux, S.phi, S.phib, S.out); break;
    case 3: op_laplacian(m, dt, DIFVM_BC_ALL_FIXED, nullptr, S.phi, S.g, S.phib, S.out); break;
    default: op_ldu_spmv(m, dt, 1, 0, S.diag, S.up, S.up, S.phi, S.out); break;
  }
}

static double time_op(difvm_mesh* m, int knob, const Scratch& S, int reps, hipEvent_t e0, hipEvent_t e1) {
  hipStream_t s = stream_of(m);
  run_op(m, knob, S);
  DIFVM_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) run_op(m, knob, S);
  DIFVM_HIP(hipEventRecord(e1, s));
  DIFVM_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  DIFVM_HIP(hipEventElapsedTime(&ms, e0, e1));
  return ms * 1e-3 / reps;
}

// ---- the cache: a flat JSON object {"key": integer, ...}
static std::map<std::string, int> read_cache(const char* path) {
  std::map<std::string, int> c;
  std::ifstream in(path);
  if (!in) return c;  // no file yet
  std::stringstream ss;
  ss << in.rdbuf();
  std::string t = ss.str();
  size_t p = 0;
  while ((p = t.find('"', p)) != std::string::npos) {
    size_t q = t.find('"', p + 1);
    DIFVM_CHECK(q != std::string::npos, DIFVM_ERR_INVALID_ARG, "tuning cache: unterminated key");
    std::string key = t.substr(p + 1, q - p - 1);
    size_t colon = t.find(':', q);
    DIFVM_CHECK(colon != std::string::npos, DIFVM_ERR_INVALID_ARG, "tuning cache: missing ':'");
    char* end = nullptr;
    long v = std::strtol(t.c_str() + colon + 1, &end, 10);
    DIFVM_CHECK(end && end != t.c_str() + colon + 1, DIFVM_ERR_INVALID_ARG, "tuning cache: value is not an integer");
    c[key] = (int)v;
    p = (size_t)(end - t.c_str());
  }
  return c;
}

static void write_cache(const char* path, const std::map<std::string, int>& c) {
  std::ofstream out(path, std::ios::trunc);
  DIFVM_CHECK((bool)out, DIFVM_ERR_INVALID_ARG, std::string("tuning cache: cannot write ") + path);
  out << "{\n";
  size_t k = 0;
  for (const auto& kv : c) out << "  \"" << kv.first << "\": " << kv.second << (++k < c.size() ? ",\n" : "\n");
  out << "}\n";
  DIFVM_CHECK((bool)out, DIFVM_ERR_INVALID_ARG, std::string("tuning cache: write failed for ") + path);
}

static std::string arch_name(int device) {
  hipDeviceProp_t prop;
  DIFVM_HIP(hipGetDeviceProperties(&prop, device));
  std::string a = prop.gcnArchName;
  size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

int tune(difvm_mesh* m, const char* cache_path) {
  const DMesh& d = m->d;
  std::string prefix = arch_name(ctx_of(m).device) + "|";
  int bucket = (int)std::floor(std::log2((double)std::max(1, d.nc)));
  std::string suffix = "|n" + std::to_string(bucket) + (d.nseg > 1 ? "|multi" : "|single");
  std::map<std::string, int> cache;
  if (cache_path) cache = read_cache(cache_path);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DIFVM_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  DIFVM_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  int timed = 0;
  try {
    Scratch S64(ctx_of(m)), S32(ctx_of(m));
    bool made64 = false, made32 = false;
    for (int k = 0; k < DIFVM_TUNE_COUNT; ++k) {
      std::string key = prefix + KNOB_NAME[k] + suffix;
      auto it = cache.find(key);
      if (it != cache.end()) {
        check_launch(k, it->second);
        m->tune[k] = it->second;
        continue;
      }
      double best = 1e300;
      int best_v = m->tune[k];
      if (op_knob(k)) {
        Scratch& S = (k & 1) ? S32 : S64;
        if ((k & 1) && !made32) { S32.init<float>(d, stream_of(m)); made32 = true; }
        if (!(k & 1) && !made64) { S64.init<double>(d, stream_of(m)); made64 = true; }
        for (int v : {64, 128, 256, 512}) {
          m->tune[k] = v;
          double t = time_op(m, k, S, 10, e0, e1);
          if (t < best) { best = t; best_v = v; }
        }
      } else {
        // one block per tile (0), fixed persistent grids, and the grids that give every block of an
        // XCD's eighth of the tiles at most 2 or 4 of them (a fixed grid can leave one block a tile
        // more than the others, which then finishes alone)
        const int per_xcd = (d.ntile + 7) / 8;
        std::vector<int> grids = {0, 1024, 512, 256};
        for (int most : {2, 4}) {
          int g = 8 * ((per_xcd + most - 1) / most);
          if (std::find(grids.begin(), grids.end(), g) == grids.end()) grids.push_back(g);
        }
        for (int v : grids) {
          if (v && v >= d.ntile) continue;
          double t = time_pcg_spmv(m, v, 10, e0, e1);
          if (t < best) { best = t; best_v = v; }
        }
      }
      m->tune[k] = best_v;
      cache[key] = best_v;
      ++timed;
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (cache_path && timed) write_cache(cache_path, cache);
  return timed;
}

}  // namespace difvm

using namespace difvm;

extern "C" {

difvm_status difvm_mesh_set_launch(difvm_mesh* mesh, int32_t knob, int32_t value) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(mesh, DIFVM_ERR_INVALID_ARG, "mesh is NULL");
  check_launch(knob, value);
  mesh->tune[knob] = value;
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_mesh_get_launch(const difvm_mesh* mesh, int32_t knob, int32_t* value) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(mesh && value, DIFVM_ERR_INVALID_ARG, "mesh and value must not be NULL");
  DIFVM_CHECK(knob >= 0 && knob < DIFVM_TUNE_COUNT, DIFVM_ERR_INVALID_ARG, "unknown tuning knob");
  *value = mesh->tune[knob];
  DIFVM_API_END
  return DIFVM_OK;
}

difvm_status difvm_tune(difvm_mesh* mesh, const char* cache_path, int32_t* n_timed) {
  DIFVM_API_BEGIN
  DIFVM_CHECK(mesh, DIFVM_ERR_INVALID_ARG, "mesh is NULL");
  DIFVM_HIP(hipSetDevice(ctx_of(mesh).device));
  int t = tune(mesh, cache_path);
  if (n_timed) *n_timed = t;
  DIFVM_API_END
  return DIFVM_OK;
}

}  // extern "C"
