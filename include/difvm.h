/* difvm.h -- C ABI of the MI355X face-graph finite-volume / PISO library.
 *
 * The library computes the hot path of DiFVM (arXiv 2603.15920): the finite-volume operators of an
 * incompressible PISO step on an unstructured polyhedral mesh, written as gather/flux/aggregate
 * passes over the mesh graph (paper Sec. "Graph-Based Reformulation of the FVM Solver"), and the
 * Krylov solves inside the step.
 *
 * Conventions for every entry point
 *  - Plain C: integers are int32, floating point is double (DIFVM_F64) or float (DIFVM_F32).
 *  - "device" pointers are HIP device memory on the context's device (for example the data pointer
 *    of a contiguous torch tensor); "host" pointers are ordinary CPU memory.
 *  - Host arrays passed in are borrowed for the duration of the call and copied.  Device arrays are
 *    owned by the caller and must stay alive until the work queued on the context's stream ends.
 *  - Work is queued on the context's HIP stream and the call returns without waiting, except where
 *    a function is documented to synchronise (mesh creation, exports, solves, PISO steps: these
 *    wait because their Krylov loops read a convergence flag).
 *  - Return value: 0 success; > 0 a warning with outputs written (e.g. not converged); < 0 an
 *    error with outputs untouched.  difvm_last_error() gives a message for the calling thread.
 *  - Field arrays passed to operators are in the library's INTERNAL order (cells renumbered by
 *    reverse Cuthill-McKee, faces re-oriented and sorted); difvm_permute converts.  Vector fields
 *    are cell-major [n][3]; gradients of an ncomp-component field are [n][ncomp][3].
 *  - Boundary-face arrays are [n_boundary_faces * ncomp] in internal boundary order; values are read
 *    only where the selected boundary table says "fixed value".
 */
#ifndef DIFVM_H
#define DIFVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DIFVM_ABI_VERSION 1

typedef int32_t difvm_status;
enum {
  DIFVM_OK = 0,
  DIFVM_WARN_NOT_CONVERGED = 1,
  DIFVM_WARN_BREAKDOWN = 2,
  DIFVM_ERR_INVALID_ARG = -1,
  DIFVM_ERR_INVALID_MESH = -2,
  DIFVM_ERR_HIP = -3,
  DIFVM_ERR_OOM = -4,
  DIFVM_ERR_UNSUPPORTED = -5,
  DIFVM_ERR_NONFINITE = -6
};

enum { DIFVM_F64 = 0, DIFVM_F32 = 1 };

/* boundary types per patch (paper Sec. "Supported Boundary Conditions"): fixedValue (Dirichlet),
 * zeroGradient (Neumann), empty (2D front/back, excluded from every sum), Windkessel RCR outlet */
enum { DIFVM_U_FIXED = 0, DIFVM_U_ZEROGRAD = 1, DIFVM_U_EMPTY = 2 };
enum { DIFVM_P_ZEROGRAD = 0, DIFVM_P_FIXED = 1, DIFVM_P_WINDKESSEL = 2, DIFVM_P_EMPTY = 3 };

/* which boundary table an operator uses: the patches' velocity types, their pressure types
 * (Windkessel counts as fixed), or every non-empty face fixed / zeroGradient */
enum { DIFVM_BC_U = 0, DIFVM_BC_P = 1, DIFVM_BC_ALL_FIXED = 2, DIFVM_BC_ALL_ZEROGRAD = 3 };

/* face value used by the divergence operator (eqs. conv_face_flux, upwind) */
enum { DIFVM_SCHEME_ONE = 0, DIFVM_SCHEME_UPWIND = 1, DIFVM_SCHEME_LINEAR = 2 };
/* convection schemes of the momentum predictor and scalar transport (Sec. "Spatial discretization",
 * scheme table): upwind is implicit; the others add the deferred correction of eq.
 * deferred_correction to an implicit upwind matrix (see difvm_op_deferred_correction) */
enum { DIFVM_CONV_UPWIND = 0, DIFVM_CONV_LINEAR = 1, DIFVM_CONV_SOU = 2, DIFVM_CONV_QUICK = 3 };
/* time schemes (scheme table): a theta-method on the matrix part of the predictor (upwind convection
 * of the lagged flux and orthogonal diffusion), (V/dt)(u' - u^n) + theta A u' + (1 - theta) A u^n =
 * explicit terms, with theta = 1 (backward Euler), 0 (forward Euler: the predictor is the explicit
 * update of eq. momentum_predictor), 1/2 (Crank-Nicolson).  Explicit terms (non-orthogonal and
 * deferred corrections, the pressure gradient of the predictor) come whole from the old level.  One set
 * of boundary values serves a step: give them at t^n + theta dt. */
enum { DIFVM_TIME_BACKWARD_EULER = 0, DIFVM_TIME_FORWARD_EULER = 1, DIFVM_TIME_CRANK_NICOLSON = 2 };

/* array kinds for difvm_permute */
enum {
  DIFVM_KIND_CELL = 0,      /* [n_cells * ncomp]                                                 */
  DIFVM_KIND_FACE = 1,      /* [(n_internal + n_boundary) * ncomp], values (no sign change)      */
  DIFVM_KIND_FACE_FLUX = 2, /* as FACE, but a re-oriented internal face changes sign (fluxes)    */
  DIFVM_KIND_BFACE = 3      /* [n_boundary * ncomp]                                              */
};
enum { DIFVM_TO_INTERNAL = 0, DIFVM_FROM_INTERNAL = 1 };

/* Mesh flags.  DIFVM_RENUMBER_RCM: reverse Cuthill-McKee cell order.  DIFVM_NONORTH_*: the split of a
 * face vector S = Delta + k used by every diffusion-type flux (Laplacian, momentum viscous term,
 * pressure equation, face-flux correction, adjoint), Sec. "Diffusive flux discretization", eq.
 * nonortho_flux.  Delta = delta d lies along the cell-to-cell vector d (boundary: d = Cf - C_O, where
 * k is dropped) and the orthogonal part of S.grad(phi) is delta (phi_N - phi_O):
 *   OVERRELAXED (default)  delta = |S|^2 / (S.d)      k = S - delta d   (k perpendicular to S)
 *   MINIMUM                delta = (S.d) / |d|^2      k = S - delta d   (k perpendicular to d)
 *   ORTHOGONAL             delta = |S| / |d|          k = S - delta d   (|Delta| = |S|)
 *   NONE                   delta = |S| / |d|          k = 0             (two-point stencil, eq. diff_ortho)
 * The four are values of a two-bit field (DIFVM_NONORTH_MASK); all coincide when S is parallel to d. */
#define DIFVM_RENUMBER_RCM 1u
#define DIFVM_NONORTH_OVERRELAXED 0u
#define DIFVM_NONORTH_MINIMUM 2u
#define DIFVM_NONORTH_ORTHOGONAL 4u
#define DIFVM_NONORTH_NONE 6u
#define DIFVM_NONORTH_MASK 6u

typedef struct difvm_ctx difvm_ctx;
typedef struct difvm_mesh difvm_mesh;
typedef struct difvm_piso difvm_piso;

int difvm_abi_version(void);
const char* difvm_last_error(void);

/* ---- context ------------------------------------------------------------------------------
 * device: HIP device ordinal.  hip_stream: a hipStream_t (NULL = the default stream).  The context
 * owns nothing of the caller's; destroy waits for its stream.
 *
 * Lifetimes: handles are reference counted.  A mesh holds its context, a PISO object its mesh and a
 * tape its PISO object; every *_destroy drops the caller's reference, and an object is freed (after
 * waiting for its stream) once nothing refers to it, so handles may be destroyed in any order.  A
 * handle must not be used after its own *_destroy.  Objects are not thread-safe: one host thread at a
 * time per context. */
difvm_status difvm_ctx_create(int device, void* hip_stream, difvm_ctx** out);
difvm_status difvm_ctx_set_stream(difvm_ctx* ctx, void* hip_stream);
difvm_status difvm_ctx_destroy(difvm_ctx* ctx); /* NULL is a no-op */

/* Device-memory allocator of the context.  The paper keeps the whole simulation on the device and
 * leaves memory to its framework (Sec. "Computational Efficiency": the run's GPU footprint); here the
 * caller supplies it, so that under Python every block the library holds is memory of torch's
 * caching allocator.  Every device allocation the library makes for objects of this context (mesh
 * arrays, solver workspaces and scratch, PISO state, AMG hierarchies, tapes, autotuner scratch)
 * calls alloc(bytes, stream, user), with stream the context's hipStream_t, and returns the block
 * with free(ptr, stream, user); alloc returns NULL on failure (the call that needed the memory then
 * fails with DIFVM_ERR_OOM).  Blocks must be device memory of the context's device, aligned to at
 * least 256 bytes; the library frees a block only after the work that used it has finished on the
 * context's stream (or that stream has been synchronised).  Both NULL restores the default
 * (hipMalloc / hipFree).  Pinned host mirrors of solver flags are not device memory and are not
 * routed here.  Allocations happen when objects are created and at the first use of a workspace
 * (first solve on a mesh, first AMG solve of a PISO object, first step with a tape or in graph mode);
 * repeated solves, steps and operator calls allocate nothing.  Errors: DIFVM_ERR_INVALID_ARG when
 * exactly one of alloc and free is NULL, or when an object (mesh, PISO, ...) still holds the
 * context, since every block must be returned to the allocator that made it. */
difvm_status difvm_ctx_set_allocator(difvm_ctx* ctx, void* (*alloc)(size_t bytes, void* stream, void* user),
                                     void (*free)(void* ptr, void* stream, void* user), void* user);

/* Kernel timing for benchmarks.  difvm_ctx_profile(ctx, n) with n >= 1 enables it: every n-th launch
 * of each of the library's PCG kernels inside difvm_solve_pcg and difvm_piso_step (counted per
 * kernel name from the call that enabled it) is bracketed by a pair of HIP events on the context's
 * stream, the stream the kernels run on (n > 1 keeps the events' own cost out of most launches);
 * n = 0 disables it, n < 0 is DIFVM_ERR_INVALID_ARG.  Launches inside a captured step (graph mode,
 * difvm_piso_set_graph) are not timed.  difvm_ctx_profile_read
 * synchronises, returns per-kernel counts of timed launches and their summed event durations
 * (kernel names in out[k].name), and clears the record.  Launches of CG iterations queued after the
 * solve had stopped (they return at once) are reported under "<name> (idle)". */
typedef struct {
  char name[32];
  int32_t launches;
  double total_ms;
} difvm_kernel_time;
difvm_status difvm_ctx_profile(difvm_ctx* ctx, int every_nth);
/* Phase timing of eager PISO steps (the per-phase breakdown of a step): with enable != 0 every eager
 * step made by difvm_piso_step brackets its phases with HIP events on the context's stream, named
 * "step: momentum assembly" (Windkessel update, velocity gradient, momentum matrix and source),
 * "step: momentum solve" (pressure gradient, predictor right-hand side, BiCGStab), and per corrector
 * "step: pressure assembly" (HbyA, face fluxes, pressure matrix), "step: pressure solve" (CG with its
 * preconditioner, including the GPU's idle time while the host polls the solver) and
 * "step: correction" (flux and velocity correction).  Independent of difvm_ctx_profile's kernel
 * timing and of its stride; the AMG setup and captured steps are not timed.  Read with
 * difvm_ctx_profile_read; enable = 0 stops it. */
difvm_status difvm_ctx_profile_phases(difvm_ctx* ctx, int enable);
difvm_status difvm_ctx_profile_read(difvm_ctx* ctx, difvm_kernel_time* out, int32_t max_out, int32_t* n_out);

/* ---- mesh ----------------------------------------------------------------------------------
 * The paper's static graph (Sec. "Structural isomorphism ... static graph construction"): owner and
 * neighbour per face, face area vectors Sf pointing out of the owner, face centroids Cf, cell
 * centroids C, cell volumes V, and boundary patches.  Faces [0, Fi) are internal; boundary faces
 * [Fi, Fi+Fb) are grouped in patches that tile that range in order.  w is the owner interpolation
 * weight per internal face; NULL means w = S.(C_N - C_f) / S.(C_N - C_O) (the point where the line
 * between the two centroids meets the face plane).  All arrays are HOST memory in user order. */
typedef struct {
  int32_t start, size;   /* boundary-face range [start, start+size), absolute face indices  */
  int32_t u_type;        /* DIFVM_U_*                                                        */
  int32_t p_type;        /* DIFVM_P_*                                                        */
  int32_t windkessel_id; /* >= 0 for DIFVM_P_WINDKESSEL patches, else -1                     */
} difvm_patch;

typedef struct {
  size_t struct_size; /* sizeof(difvm_mesh_desc) */
  int32_t n_cells, n_internal_faces, n_boundary_faces, n_patches;
  const int32_t* owner;     /* [Fi+Fb]       */
  const int32_t* neighbour; /* [Fi]          */
  const double* Sf;         /* [(Fi+Fb)*3]   */
  const double* Cf;         /* [(Fi+Fb)*3]   */
  const double* C;          /* [Nc*3]        */
  const double* V;          /* [Nc]          */
  const double* w;          /* [Fi] or NULL  */
  const difvm_patch* patches;
} difvm_mesh_desc;

typedef struct {
  int32_t n_cells, n_internal_faces, n_boundary_faces, n_patches;
  int32_t n_slices, n_slots;        /* cell-slot layout: 64-cell slices, one slot per non-empty face side */
  int32_t bandwidth_in, bandwidth_out; /* max |O-N| before and after renumbering */
  int32_t n_windkessel;
  int32_t has_fixed_p;              /* 1 if some face carries a fixed or Windkessel pressure */
  int32_t n_segments;               /* independent cell ranges (1 unless made by _create_segments) */
} difvm_mesh_info;

/* Host-only renumbering (no device needed): reverse Cuthill-McKee cell order (flag
 * DIFVM_RENUMBER_RCM; 0 keeps the order), internal faces re-oriented so owner < neighbour (a flip
 * negates S and maps w to 1-w) and sorted by (owner, neighbour), boundary faces stably sorted by new
 * owner inside each patch, and the neighbour-sorted face list ("losort").  Outputs are host arrays
 * (new -> old where a permutation): cell_perm[Nc], face_perm[Fi], face_flip[Fi], owner[Fi],
 * neighbour[Fi], own_start[Nc+1], losort[Fi], losort_start[Nc+1], bface_perm[Fb] (indices within the
 * boundary block), bowner[Fb].  Optional (NULL to skip) permuted geometry: S[(Fi+Fb)*3], w[Fi],
 * delta[Fi+Fb] and k[Fi*3] of the DIFVM_NONORTH_* scheme in flags (boundary d = Cf - C_O).  Unknown
 * flag bits: DIFVM_ERR_INVALID_ARG. */
difvm_status difvm_mesh_renumber_host(const difvm_mesh_desc* desc, uint32_t flags, int32_t* cell_perm,
                                      int32_t* face_perm, uint8_t* face_flip, int32_t* owner, int32_t* neighbour,
                                      int32_t* own_start, int32_t* losort, int32_t* losort_start,
                                      int32_t* bface_perm, int32_t* bowner, double* S, double* w, double* delta,
                                      double* k);

/* Validates, renumbers and uploads a mesh (synchronises).  flags: DIFVM_RENUMBER_RCM or 0, or-ed with
 * one DIFVM_NONORTH_* scheme.  Errors: DIFVM_ERR_INVALID_ARG for unknown flag bits;
 * DIFVM_ERR_INVALID_MESH for counts that do not match, patches that do not tile the boundary block,
 * indices out of range, neighbour == owner, V <= 0 or S.d <= 0 on a non-empty face. */
difvm_status difvm_mesh_create(difvm_ctx* ctx, const difvm_mesh_desc* desc, uint32_t flags, difvm_mesh** out);

/* Batched form: one mesh made of n_seg independent meshes packed block-diagonally (the paper's
 * outlook on batching many small simulations on one device).  seg_cell_start[n_seg+1] (host) gives
 * the user cell range of each segment: 0 = start[0] < start[1] < ... < start[n_seg] = Nc.  No internal
 * face may join two segments.  Every reduction (dot products, stopping tests) is taken per segment,
 * so each member solves its own system with its own iteration count and results equal to those of
 * the member run alone (same operations in the same order).  Errors as difvm_mesh_create, plus
 * DIFVM_ERR_INVALID_ARG for bad offsets and DIFVM_ERR_INVALID_MESH for a face joining segments.
 * difvm_mesh_create is this call with one segment. */
difvm_status difvm_mesh_create_segments(difvm_ctx* ctx, const difvm_mesh_desc* desc, uint32_t flags, int32_t n_seg,
                                        const int32_t* seg_cell_start, difvm_mesh** out);
difvm_status difvm_mesh_get_info(const difvm_mesh* mesh, difvm_mesh_info* info);
difvm_status difvm_mesh_destroy(difvm_mesh* mesh); /* NULL is a no-op; waits for the stream */

/* ---- slab partition and halo exchange ------------------------------------------------------
 * The paper runs one mesh per GPU and leaves multi-GPU partitioning to future work (Sec.
 * "Limitations and Future Work").  These calls hold the part of that design that one GPU can run: a
 * partition of one mesh into n_parts slabs, each slab's mesh with ghost copies of the cells across
 * its cut faces, and the pack / unpack of one exchange.  The transfer between GPUs (RCCL send/recv
 * or a peer copy of each send segment into the matching receive segment) is the caller's.
 *
 * Part p owns the internal (renumbered) cells [cell_lo, cell_hi) of the whole mesh, with cell_lo =
 * floor(p Nc / n_parts): RCM ranges are slabs across the mesh.  Its local cell order is the owned
 * cells in whole-mesh order, then the ghosts in ascending whole-mesh index.  Its internal faces are
 * those of the whole mesh with an owned side (whole-mesh orientation and order), its boundary faces
 * those of its owned cells (patch order kept).  Every owned cell keeps its whole-mesh row (the same
 * faces in the same order), so once the ghost rows hold the current values, the owned rows of
 * every operator (difvm_op_*, difvm_ldu_spmv, difvm_ldu_assemble_laplace) equal the whole mesh's
 * rows bit for bit; ghost rows of the outputs are not meaningful.  Part meshes take fields in their
 * local order (difvm_permute is the identity on them).  Solvers, AMG and PISO objects need
 * reductions over the whole mesh and refuse part meshes (DIFVM_ERR_UNSUPPORTED). */
typedef struct difvm_partition difvm_partition;
typedef struct {
  int32_t n_parts;
  int32_t cell_lo, cell_hi;                    /* owned cells, whole-mesh internal numbering          */
  int32_t n_owned, n_ghost;                    /* local cells: n_owned + n_ghost                      */
  int32_t n_internal_faces, n_boundary_faces;  /* local faces                                         */
  int32_t n_send;                              /* rows this part sends per exchange, all destinations */
  int32_t n_neighbours;                        /* parts it sends to or receives from                  */
} difvm_part_info;

/* Renumbers the mesh as difvm_mesh_create does (same flags) and splits it into n_parts slabs (host
 * only, no device needed).  Errors as difvm_mesh_create; DIFVM_ERR_INVALID_ARG unless 1 <= n_parts
 * <= Nc. */
difvm_status difvm_partition_create(const difvm_mesh_desc* desc, uint32_t flags, int32_t n_parts,
                                    difvm_partition** out);
difvm_status difvm_partition_destroy(difvm_partition* part); /* NULL is a no-op */
difvm_status difvm_partition_info(const difvm_partition* part, int32_t p, difvm_part_info* info);
/* Host maps of part p (each output may be NULL): cell_global[n_owned+n_ghost] (local cell -> whole-
 * mesh internal cell), face_global[n_internal_faces] and bface_global[n_boundary_faces] (local ->
 * whole-mesh internal face, boundary index within the boundary block), recv_start[n_parts+1] (the
 * ghosts owned by part q are local ghost rows [recv_start[q], recv_start[q+1]) after the owned
 * rows), send_start[n_parts+1] and send_cells[n_send] (local owned rows sent to part q:
 * send_cells[send_start[q] .. send_start[q+1]), in the receiving part's ghost order).  So the
 * receive buffer of one exchange, in ghost order, takes from part q's send buffer the rows
 * [send_start_q[p], send_start_q[p+1]) at rows [recv_start_p[q], recv_start_p[q+1]).  Errors:
 * DIFVM_ERR_INVALID_ARG for p out of range. */
difvm_status difvm_partition_maps(const difvm_partition* part, int32_t p, int32_t* cell_global,
                                  int32_t* face_global, int32_t* bface_global, int32_t* recv_start,
                                  int32_t* send_start, int32_t* send_cells);
/* Uploads part p as a mesh of ctx (synchronises).  The partition may be destroyed afterwards. */
difvm_status difvm_mesh_create_part(difvm_ctx* ctx, const difvm_partition* part, int32_t p, difvm_mesh** out);
/* One exchange on the mesh's stream (device arrays, rows of ncomp values, dtype DIFVM_F64/F32):
 * pack writes send_buf[n_send*ncomp] = the sent rows of x[(n_owned+n_ghost)*ncomp]; unpack copies
 * recv_buf[n_ghost*ncomp] (ghost order) into the ghost rows of x.  Errors: DIFVM_ERR_INVALID_ARG on a
 * mesh that is not a part, ncomp outside 1..9 or NULL buffers where rows are moved. */
difvm_status difvm_halo_pack(const difvm_mesh* mesh, int dtype, int ncomp, const void* x, void* send_buf);
difvm_status difvm_halo_unpack(const difvm_mesh* mesh, int dtype, int ncomp, const void* recv_buf, void* x);

/* ---- launch tuning (autotuner) ------------------------------------------------------------
 * Knobs that change how work is spread over the GPU but not what any output computes: threads per
 * block of the operator kernels (one cell or face per thread, no reductions), and the grid of the
 * PCG product kernel (one block per 1024-cell tile, or a persistent grid whose blocks walk several
 * tiles; every tile's partial sum is formed the same way).  Outputs are bitwise identical for every
 * value.  Each mesh starts with 256 threads and one block per tile. */
enum {
  DIFVM_TUNE_INTERP_F64 = 0, DIFVM_TUNE_INTERP_F32 = 1,
  DIFVM_TUNE_GRAD_F64 = 2, DIFVM_TUNE_GRAD_F32 = 3,
  DIFVM_TUNE_DIV_F64 = 4, DIFVM_TUNE_DIV_F32 = 5,
  DIFVM_TUNE_LAPLACIAN_F64 = 6, DIFVM_TUNE_LAPLACIAN_F32 = 7,
  DIFVM_TUNE_LDU_SPMV_F64 = 8, DIFVM_TUNE_LDU_SPMV_F32 = 9,
  DIFVM_TUNE_PCG_GRID = 10,
  DIFVM_TUNE_COUNT = 11
};

/* Sets one knob: operator knobs take 64, 128, 256 or 512 (threads per block); DIFVM_TUNE_PCG_GRID
 * takes 0 (one block per tile) or a multiple of 8 (persistent grid; values >= the tile count mean
 * one block per tile).  Other values or knobs: DIFVM_ERR_INVALID_ARG. */
difvm_status difvm_mesh_set_launch(difvm_mesh* mesh, int32_t knob, int32_t value);
difvm_status difvm_mesh_get_launch(const difvm_mesh* mesh, int32_t knob, int32_t* value);

/* Autotuner: for every knob, times each candidate value on this mesh (HIP events on the context's
 * stream, scratch inputs allocated and freed here, one warm-up and repeated launches) and keeps the
 * fastest.  The PCG grid's candidates are one block per tile, 1024, 512 and 256 blocks, and the
 * grids that give every block at most 2 or 4 of the tiles its XCD owns.  cache_path (may be NULL) names a JSON file of choices keyed by GPU architecture, knob and
 * mesh size bucket (floor(log2(cells)), and whether the mesh has one or several segments): knobs
 * found there are applied without timing, the others are timed and the file is rewritten with them
 * added.  n_timed (may be NULL) receives the number of knobs timed.  Synchronises.  Errors:
 * DIFVM_ERR_INVALID_ARG for an unreadable or unwritable cache file. */
difvm_status difvm_tune(difvm_mesh* mesh, const char* cache_path, int32_t* n_timed);

/* Reorders a field between user and internal order (device arrays, src != dst). */
difvm_status difvm_permute(const difvm_mesh* mesh, int dtype, int ncomp, int kind, int dir, const void* src,
                           void* dst);

/* ---- operators (device arrays, internal order; dtype F64 or F32) -------------------------- */

/* Linear face interpolation (Sec. "Spatial discretization", the face value of eq. gauss_green):
 * phi_f = w phi_O + (1-w) phi_N; boundary: fixed -> phi_b, zeroGradient -> phi_O, empty -> 0.
 * phi[Nc*ncomp] -> phi_f[(Fi+Fb)*ncomp]. */
difvm_status difvm_op_interp(const difvm_mesh* mesh, int dtype, int ncomp, int bc, const void* phi,
                             const void* phi_b, void* phi_f);

/* Gauss-Green gradient (eq. gauss_green): G_i = (1/V_i) sum_f sigma phi_f S_f with phi_f from the
 * linear interpolation above.  phi[Nc*ncomp] -> grad[Nc*ncomp*3]. */
difvm_status difvm_op_grad(const difvm_mesh* mesh, int dtype, int ncomp, int bc, const void* phi, const void* phi_b,
                           void* grad);

/* Face-sum divergence (eqs. conv_face_flux, upwind, aggregate): D_i = sum_f sigma F_f psi_f, not
 * divided by V.  flux[Fi+Fb] (internal orientation), psi[Nc*ncomp], psi_b[Fb*ncomp] ->
 * out[Nc*ncomp].  Upwind picks the owner value when F >= 0. */
difvm_status difvm_op_div(const difvm_mesh* mesh, int dtype, int scheme, int ncomp, int bc, const void* flux,
                          const void* psi, const void* psi_b, void* out);

/* Deferred-correction source of a convection scheme (eq. deferred_correction): the explicit part
 * F_f (phi_f^HO - phi_f^U) of every internal face moved to the right-hand side,
 *   out_i = - sum_f sigma F_f (phi_f^HO - phi_f^U),   sigma = +1 for the owner, -1 for the neighbour,
 * with C the upwind cell (the owner when F >= 0), D the other cell, phi^U = phi_C and
 *   DIFVM_CONV_LINEAR  phi^HO = w phi_O + (1-w) phi_N
 *   DIFVM_CONV_SOU     phi^HO = phi_C + g_C . (x_f - x_C)                  (eq. sou)
 *   DIFVM_CONV_QUICK   phi^HO = phi_C + (phi_D - phi_C)/4 + g_C . (x_D - x_C)/4
 *   DIFVM_CONV_UPWIND  no correction (out = 0).
 * (QUICK: the uniform-grid 3/8 phi_D + 6/8 phi_C - 1/8 phi_U with the far-upwind value taken as
 * phi_D - 2 g_C . (x_D - x_C).)  Boundary faces carry no correction.  dtype F64 only (F32:
 * DIFVM_ERR_UNSUPPORTED).  flux[Fi+Fb] (internal orientation), phi[Nc*ncomp], grad[Nc*ncomp*3] (the
 * cell gradients, e.g. difvm_op_grad) -> out[Nc*ncomp]. */
difvm_status difvm_op_deferred_correction(const difvm_mesh* mesh, int dtype, int conv, int ncomp, const void* flux,
                                          const void* phi, const void* grad, void* out);

/* Laplacian with non-orthogonal correction (the mesh's DIFVM_NONORTH_* scheme; eqs. diff_ortho, nonortho_flux):
 * L_i = sum_f sigma G_f [delta_f (phi_N - phi_O) + k_f . (w g_O + (1-w) g_N)]
 *       + sum_{b fixed} G_b delta_b (phi_b - phi_O).
 * gamma_f[Fi+Fb] or NULL (= 1), phi[Nc], grad_phi[Nc*3] (given), phi_b[Fb] -> out[Nc]. */
difvm_status difvm_op_laplacian(const difvm_mesh* mesh, int dtype, int bc, const void* gamma_f, const void* phi,
                                const void* grad_phi, const void* phi_b, void* out);

/* LDU matrix (OpenFOAM-style, the form behind eq. Ap_H): diag[Nc], upper[Fi] (row owner, column
 * neighbour), lower[Fi] (row neighbour, column owner); lower == NULL means symmetric. */
typedef struct {
  int32_t dtype;
  void* diag;
  void* upper;
  void* lower;
} difvm_ldu;

/* y = A x (transpose = 0) or A^T x; x, y [Nc*ncomp], ncomp in {1, 3}. */
difvm_status difvm_ldu_spmv(const difvm_mesh* mesh, int ncomp, int transpose, const difvm_ldu* A, const void* x,
                            void* y);

/* SPD orthogonal part of -div(G grad phi) (F64): upper_f = -G_f delta_f, diag = sum G_f delta_f +
 * sum_{b fixed} G_b delta_b, rhs_bc = sum_{b fixed} G_b delta_b phi_b.  A->lower is not written. */
difvm_status difvm_ldu_assemble_laplace(const difvm_mesh* mesh, int bc, const void* gamma_f, const void* phi_b,
                                        difvm_ldu* A, void* rhs_bc);

/* Momentum matrix of the implicit predictor (F64): implicit Euler, implicit upwind convection of the
 * lagged flux, implicit orthogonal diffusion; b carries V/dt U^n, fixed-value boundary terms and the
 * explicit non-orthogonal diffusion from grad(U^n).  flux[Fi+Fb], U[Nc*3], U_b[Fb*3] (velocity
 * table) -> A (diag, upper, lower), b[Nc*3]. */
difvm_status difvm_ldu_assemble_momentum(const difvm_mesh* mesh, double nu, double dt, const void* flux,
                                         const void* U, const void* U_b, difvm_ldu* A, void* b);

/* For callers that cannot allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): difvm_ldu_assemble_momentum with its scratch (the velocity
 * gradient, 9 doubles per cell) in a fixed device array of 9 * DIFVM_NOALLOC_MAX_CELLS doubles (9 MiB)
 * that every GPU the library runs on holds until the process ends; the call allocates nothing
 * (no hipMalloc, no allocator callback) and computes bitwise what difvm_ldu_assemble_momentum
 * computes.  The array's address on a device is taken by difvm_ctx_create on that device, so the
 * mesh's context must exist (it does, the mesh holds it).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race and must be serialised by
 * the caller.  Synchronises the mesh's stream.  Errors as difvm_ldu_assemble_momentum, plus
 * DIFVM_ERR_INVALID_ARG for a mesh of more than DIFVM_NOALLOC_MAX_CELLS cells or on a device ordinal
 * of 64 or more. */
#define DIFVM_NOALLOC_MAX_CELLS 131072
difvm_status difvm_ldu_assemble_momentum_noalloc(const difvm_mesh* mesh, double nu, double dt, const void* flux,
                                                 const void* U, const void* U_b, difvm_ldu* A, void* b);

typedef struct {
  int32_t iters[3];
  double residual[3]; /* final ||r||_2 / ||b||_2 per component */
  int32_t status;
} difvm_solve_stats;

/* Jacobi-preconditioned CG on a symmetric F64 LDU matrix (A->lower ignored).  Stops when
 * ||r||_2 <= tol ||b||_2 (checked before the first iteration and after each update); b = 0 gives
 * x = 0.  x holds the initial guess on entry.  Synchronises; stats is a host struct (may be NULL). */
difvm_status difvm_solve_pcg(const difvm_mesh* mesh, const difvm_ldu* A, const void* b, void* x, double tol,
                             int32_t maxit, difvm_solve_stats* stats);

/* Right-Jacobi BiCGStab (van der Vorst) on an F64 LDU matrix, ncomp in {1, 3} independent systems
 * sharing the matrix (b, x interleaved [Nc*ncomp]).  Same stopping rule and synchronisation. */
difvm_status difvm_solve_bicgstab(const difvm_mesh* mesh, const difvm_ldu* A, int ncomp, const void* b, void* x,
                                  double tol, int32_t maxit, difvm_solve_stats* stats);

/* ---- smoothed-aggregation AMG preconditioner for symmetric pressure systems ---------------------
 * The paper preconditions its pressure CG with ILU.  Besides Jacobi the library offers one V-cycle of
 * smoothed-aggregation algebraic multigrid per CG iteration: aggregates of distance-2 strong
 * neighbourhoods on the finest level and distance-1 below (strength threshold 0.08 on the finest,
 * 0 below), the constant vector as near-null space, prolongators smoothed by one damped-Jacobi step
 * with weight 4/(3 rho(D^-1 A)), Galerkin coarse operators, and the dense inverse of the coarsest level
 * (coarsening stops at or below 2,048 rows; the inverse is taken on the device at setup).  Every
 * level smooths with one degree-2 Chebyshev sweep in D^-1 A over [hi/10, hi], the same before and
 * after each coarse correction: on the finest level hi is the largest of 2 and the Gershgorin bound
 * of D^-1 A at setup (2 bounds every weakly diagonally dominant matrix, such as the pressure
 * operators); on coarser levels 1.1 times a power-iteration estimate of rho(D^-1 A), capped by the
 * Gershgorin bound.  The hierarchy is built on the host from one matrix and kept; the finest level
 * of each V-cycle uses the matrix being solved, so M^-1 stays symmetric positive definite while the
 * matrix drifts within that spectral bound.  On a batched mesh no aggregate crosses a segment, so
 * the V-cycle is block-diagonal and each segment's CG still stops on its own test.  CG with it
 * converges to the same solution as with Jacobi (the preconditioner changes
 * the iterates, not the stopping rule). */
enum { DIFVM_PRECOND_JACOBI = 0, DIFVM_PRECOND_AMG = 1 };
typedef struct difvm_amg difvm_amg;
/* Builds the hierarchy of the symmetric F64 LDU matrix A (device arrays, lower ignored; synchronises).
 * The object holds a reference to the mesh and a copy of A for difvm_amg_apply.  Errors: INVALID_ARG
 * for a non-positive diagonal, UNSUPPORTED for a matrix of at most 96 rows, one that does not coarsen
 * below 2,048 rows, or one whose coarsest operator is not positive definite. */
difvm_status difvm_amg_create(const difvm_mesh* mesh, const difvm_ldu* A, difvm_amg** out);
difvm_status difvm_amg_destroy(difvm_amg* amg); /* NULL is a no-op */
/* Host-only setup of the same hierarchy (no device), for inspection: a symmetric matrix with n rows
 * given as CSR of its off-diagonal entries (ptr[n+1], col, val; host arrays) and its diagonal diag[n].
 * Outputs (host, may be NULL): agg[n], the finest level's aggregate of each row; rows[0..cap), the rows
 * of each level, finest first; *n_levels.  Errors: INVALID_ARG for a malformed matrix or a
 * non-positive diagonal, UNSUPPORTED when it does not coarsen below 2,048 rows (the coarsest operator's
 * definiteness is checked by difvm_amg_create only). */
difvm_status difvm_amg_setup_host(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, const double* diag,
                                  int32_t* agg, int32_t* rows, int32_t cap, int32_t* n_levels);
/* rows of each level, finest first, into rows[0..cap) (host); *n_levels receives the level count */
difvm_status difvm_amg_levels(const difvm_amg* amg, int32_t* rows, int32_t cap, int32_t* n_levels);
/* z = M^-1 r, one V-cycle with the stored copy of A as finest level (device arrays, internal order,
 * r != z; synchronises) */
difvm_status difvm_amg_apply(difvm_amg* amg, const void* r, void* z);
/* CG on the symmetric F64 LDU matrix A preconditioned by the V-cycle (A as finest level, the stored
 * hierarchy below); arguments, stopping rule and stats as difvm_solve_pcg. */
difvm_status difvm_solve_pcg_amg(difvm_amg* amg, const difvm_ldu* A, const void* b, void* x, double tol, int32_t maxit,
                                 difvm_solve_stats* stats);

/* ---- PISO (paper Sec. "PISO as divergence-free constrained message passing") --------------- */
typedef struct {
  size_t struct_size;     /* sizeof(difvm_piso_params) */
  double nu, dt;          /* kinematic viscosity, time step (p is kinematic, rho = 1)        */
  int32_t n_corr;         /* pressure correctors per step (paper: typically 2), 1..8        */
  double tol_p, tol_u;    /* relative residual tolerances of the pressure / momentum solves  */
  int32_t maxit_p, maxit_u;
  int32_t p_ref_cell;     /* cell fixing the pressure level where no pressure is fixed: the
                             p_ref_cell-th user cell of each such segment (the user cell itself
                             for a one-segment mesh)                                          */
  double p_ref_value;
  int32_t conv;           /* convection scheme (DIFVM_CONV_*) of the predictor and of scalar
                             transport; the deferred correction is evaluated once per step from
                             U^n and its Gauss gradient and is part of the momentum source b, so
                             it also enters H in every corrector                               */
  int32_t time;           /* time scheme (DIFVM_TIME_*) of the predictor and of scalar transport   */
  int32_t precond;        /* pressure preconditioner (DIFVM_PRECOND_*); AMG builds its hierarchy from
                             the pressure matrix of the first solve and keeps it (see
                             difvm_piso_rebuild_preconditioner).  On a batched mesh the
                             hierarchy is block-diagonal over the segments, but a member's
                             iterates then differ from its standalone run's (its aggregates
                             follow the packed numbering)                                       */
} difvm_piso_params;

typedef struct {
  int32_t it_u[3];
  double res_u[3];
  int32_t it_p[8];
  double res_p[8];
  int32_t status;
} difvm_step_stats;

difvm_status difvm_piso_create(const difvm_mesh* mesh, const difvm_piso_params* params, difvm_piso** out);
difvm_status difvm_piso_destroy(difvm_piso* piso);

/* Fixed boundary values in USER boundary order, device arrays: U_b[Fb*3] (read on fixed-U faces),
 * p_b[Fb] (read on fixed-p faces); either may be NULL to keep the current values (initially 0).
 * May be called between steps (time-varying inflow). */
difvm_status difvm_piso_set_boundary(difvm_piso* piso, const void* U_b, const void* p_b);

/* Three-element Windkessel of outlet id (eqs. windkessel_ode, windkessel_discrete): proximal
 * resistance Rp, compliance C, distal resistance Rd, capacitor pressure pc. */
difvm_status difvm_piso_set_windkessel(difvm_piso* piso, int32_t id, double Rp, double C, double Rd, double pc);

/* Batched form: kinematic viscosity of each segment, nu_seg[n_seg] host (n_seg must equal the
 * mesh's segment count; initially params.nu everywhere).  Synchronises. */
difvm_status difvm_piso_set_viscosity(difvm_piso* piso, int32_t n_seg, const double* nu_seg);

/* Solver statistics of the most recent step per segment, out_host[n_seg] (n_seg must equal the
 * mesh's segment count).  The stats of difvm_piso_step are the maxima over segments. */
difvm_status difvm_piso_segment_stats(const difvm_piso* piso, int32_t n_seg, difvm_step_stats* out_host);

/* State in USER order (device arrays): U[Nc*3], p[Nc], phi[Fi+Fb] (user orientation).  phi == NULL
 * in set_state computes phi = interp(U).S with boundary values from the velocity table.
 * get_state also returns the Windkessel capacitor pressures to pc_host[n_windkessel] (may be NULL);
 * it synchronises. */
difvm_status difvm_piso_set_state(difvm_piso* piso, const void* U, const void* p, const void* phi);
difvm_status difvm_piso_get_state(difvm_piso* piso, void* U, void* p, void* phi, double* pc_host);

/* Passive scalar transport over one time step with the PISO object's current face flux (the
 * paper's convection-diffusion discretisation, Sec. "Spatial discretization", applied to one scalar
 * c): (V/dt)(c' - c) + sum_f F_f c'_upwind - D sum_f (delta_f (c'_N - c'_O) + k_f . grad(c)_f) = 0,
 * i.e. the momentum predictor's matrix with one component and diffusivity D >= 0 (written here for
 * the default backward Euler; params.time selects the theta-method of DIFVM_TIME_*): implicit Euler,
 * implicit upwind of the flux (tie F = 0 to the owner) plus the deferred correction of the PISO
 * object's convection scheme (params.conv) from c, implicit orthogonal diffusion, explicit
 * non-orthogonal correction from the Gauss gradient of c.  bc selects the boundary table (DIFVM_BC_*);
 * c_b[Fb] (device, user boundary order) gives the values on its fixed faces; c[Nc] (device, user order)
 * holds c on entry and c' on return.  Right-Jacobi BiCGStab from c with the PISO object's tol_u and
 * maxit_u; stats (host, may be NULL) receives iterations and residual in component 0.  Synchronises.
 * Returns a warning (c' still written) when the solve did not converge or broke down. */
difvm_status difvm_piso_transport_scalar(difvm_piso* piso, double D, int32_t bc, const void* c_b, void* c,
                                         difvm_solve_stats* stats);

/* Graph mode (the paper runs its time loop as one compiled scan, Sec. 2.4; here the step is a
 * replayed hipGraph).  With enable != 0, the first difvm_piso_step step after this call runs eagerly
 * and records its Krylov iteration counts; the whole step (Windkessel, assembly, BiCGStab, every
 * corrector) is then captured once on a private stream with a budget per solve: the largest count of
 * its kind (BiCGStab components, or pressure correctors) over the last 8 steps, plus a margin, plus
 * 1/64 of that count.  Each later step is one hipGraphLaunch on the context's stream followed by one
 * read of the solvers' states.  Iterations past a solve's stop are predicated no-ops, so results are
 * bitwise those of eager stepping.  A step in which some solve had not stopped within its budget is
 * discarded (its starting state, saved by the graph, is restored on the device) and run eagerly; the
 * margin grows by one and the graph is recaptured with the larger counts.  The margin starts at
 * min(1, extra_iters) and never exceeds extra_iters (>= 0); when the recent counts fall two or more
 * below the budgets the step is recaptured with tighter ones.  enable = 0 returns to eager stepping.
 * Changing boundary values, Windkessel parameters, viscosity or the state between steps is allowed
 * (the graph reads the device buffers).  Errors: DIFVM_ERR_INVALID_ARG for extra_iters < 0. */
difvm_status difvm_piso_set_graph(difvm_piso* piso, int32_t enable, int32_t extra_iters);

/* Graph-mode counters since creation: kept replays, discarded-and-redone steps, captures. */
difvm_status difvm_piso_graph_info(const difvm_piso* piso, int64_t* replays, int64_t* redos, int64_t* captures);

/* Drops the AMG hierarchy of the pressure preconditioner (and a captured step using it); the next
 * pressure solve builds a new one from its own matrix (e.g. after a change of dt or viscosity).
 * DIFVM_ERR_INVALID_ARG when the PISO object uses Jacobi. */
difvm_status difvm_piso_rebuild_preconditioner(difvm_piso* piso);

/* The pressure preconditioner's hierarchy (AMG only; DIFVM_ERR_INVALID_ARG for Jacobi): *n_levels
 * (0 before the first pressure solve built it), the rows of each level, finest first, into
 * rows[0..cap) (host), and *vcycle_bytes (may be NULL) the algorithmic bytes of one V-cycle: every
 * kernel's distinct inputs read once and outputs written once, the finest matrix counted in its LDU
 * form (diagonal; owner, neighbour and coefficient per internal face), coarse matrices in CSR (row
 * pointers, 4-byte columns, 8-byte values, diagonal) and the coarsest level's dense inverse.  For
 * rooflines of the preconditioner phase. */
difvm_status difvm_piso_precond_info(const difvm_piso* piso, int32_t* n_levels, int32_t* rows, int32_t cap,
                                     double* vcycle_bytes);

/* Advances nsteps time steps.  stats_host[nsteps] (may be NULL) receives solver iterations and
 * residuals per step.  Synchronises.  Returns the worst solver status over the steps. */
difvm_status difvm_piso_step(difvm_piso* piso, int32_t nsteps, difvm_step_stats* stats_host);

/* One step as difvm_piso_step(piso, 1, stats_host) (run eagerly, also in graph mode) that also writes
 * the solution of each linear system of the step, in USER order, to device arrays: U_star[Nc*3], the
 * momentum predictor's solution (eq. momentum_predictor, before the correctors), and p_corr[n_corr*Nc],
 * the pressure solved by each corrector in turn (eq. pressure_poisson).  With the state before the
 * step, these let a caller assemble every system of the step independently and check each solution's
 * true residual against the solver tolerance.  The first call allocates the internal-order copies
 * (kept by the PISO object).  Synchronises; returns the step's worst solver status. */
difvm_status difvm_piso_step_trace(difvm_piso* piso, void* U_star, void* p_corr, difvm_step_stats* stats_host);

/* ---- differentiation (paper Sec. "End-to-End Automatic Differentiation") -------------------
 * Reverse mode through an N-step window of the PISO: a discrete adjoint of every step (transposed
 * gathers; each linear solve differentiated implicitly with the same Krylov solver on the
 * transposed matrix, eq. implicit_diff; upwind branches frozen at the forward's choice), with the
 * state checkpointed every ckpt_every steps and each segment recomputed once (eq. checkpointing).
 * The window starts from the PISO's state when difvm_piso_forward_record is called and uses the
 * boundary values and Windkessel parameters set at that time; they must not change in between. */
typedef struct difvm_tape difvm_tape;
difvm_status difvm_tape_create(difvm_piso* piso, int32_t nsteps, int32_t ckpt_every, difvm_tape** out);
difvm_status difvm_tape_destroy(difvm_tape* tape); /* NULL is a no-op */

/* Runs the window's nsteps forward steps, storing checkpoints and the step records of the last
 * checkpoint segment, which the following difvm_piso_adjoint then reverses without recomputing it
 * (later sweeps on the same tape recompute every segment; the results are the same bits).
 * Synchronises.  stats_host[nsteps] may be NULL.  The PISO ends at the window's final state. */
difvm_status difvm_piso_forward_record(difvm_piso* piso, difvm_tape* tape, difvm_step_stats* stats_host);

/* Vector-Jacobian product of the window (eq. vjp).  Cotangents of the final state in USER order
 * (device arrays, NULL = zero): gU_N[Nc*3], gp_N[Nc], gphi_N[Fi+Fb] (user orientation), and
 * gpc_N_host[n_windkessel] (host, NULL = zero).  Outputs: cotangents of the initial state (device,
 * user order, NULL to skip) gU_0, gp_0, gphi_0 (the initial flux is an independent input), gpc_0_host,
 * and of the Windkessel parameters gwk_host[n_windkessel*3] as (Rp, C, Rd) per outlet (host).
 * adj_tol is the relative tolerance of the transposed solves.  Each transposed pressure solve starts
 * from the same corrector's solution of the step reversed just before (the later time step), the
 * sweep's first from zero, so results depend on the window and adj_tol alone, not on earlier calls.
 * Synchronises; the PISO is left at the window's final state. */
difvm_status difvm_piso_adjoint(difvm_piso* piso, difvm_tape* tape, const void* gU_N, const void* gp_N,
                                const void* gphi_N, const double* gpc_N_host, double adj_tol, void* gU_0, void* gp_0,
                                void* gphi_0, double* gpc_0_host, double* gwk_host);

/* Graph mode of the reverse sweep (the paper differentiates its time loop as one compiled scan, Sec.
 * "Computational Efficiency"; here the checkpoint segments are replayed hipGraphs).  With enable != 0,
 * difvm_piso_adjoint runs each segment of ckpt_every steps as two graphs: the recomputation of the
 * segment from its checkpoint (forward steps with their records) and its reverse sweep (the adjoint
 * steps, last first).  The sweep's first segment (the window's last) is always reversed eagerly, its
 * first pressure solves starting from zero.  The first full segment runs eagerly and records the
 * Krylov counts; both
 * graphs are then captured with a budget per solve kind (momentum, pressure) of the segment's largest
 * count plus a margin plus 1/64 of that count, and each later full segment is two hipGraphLaunches
 * and one read of the solvers' states per graph.  Iterations past a solve's stop are predicated
 * no-ops, so results are bitwise those of the eager sweep.  A replay in which some solve had not
 * stopped within its budget is discarded (the recomputation restarts from the checkpoint; the reverse
 * sweep restores the cotangents and the pressure solves' starting values saved by the graph's first
 * nodes), run eagerly, and the graph is
 * recaptured with the margin widened by one; when the counts fall two or more below the budgets the
 * graph is recaptured with tighter ones.  The margin starts at min(2, extra_iters) and never exceeds
 * extra_iters (>= 0).  A shorter last segment (nsteps not a multiple of ckpt_every) runs eagerly, and a
 * new adj_tol recaptures the reverse graph.  Errors: DIFVM_ERR_INVALID_ARG for extra_iters < 0. */
difvm_status difvm_tape_set_graph(difvm_tape* tape, int32_t enable, int32_t extra_iters);
/* Graph-mode counters of the tape since creation: kept replays (of the recomputation and reverse
 * graphs; two per full segment after the first), discarded-and-redone replays, captures. */
difvm_status difvm_tape_graph_info(const difvm_tape* tape, int64_t* replays, int64_t* redos, int64_t* captures);

/* Cotangent of the fixed velocity boundary values U_b of the window from the last difvm_piso_adjoint
 * on this tape (the boundary values are inputs of every step; their cotangent is summed over the
 * window).  gU_b[Fb*3]: device array, USER boundary order; zero on faces whose velocity is not fixed.
 * The lid-velocity inverse problem of Sec. "Lid velocity recovery" differentiates through it.
 * Errors: DIFVM_ERR_INVALID_ARG before an adjoint has run.  Synchronises. */
difvm_status difvm_tape_boundary_cotangent(const difvm_tape* tape, void* gU_b);

#ifdef __cplusplus
}
#endif
#endif /* DIFVM_H */
