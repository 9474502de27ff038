// Internal launchers of libdifvm (enqueue on the mesh's stream, device arrays in internal order).
#pragma once

#include "internal.h"

namespace difvm {

void permute(const difvm_mesh* m, int dtype, int ncomp, int kind, int dir, const void* src, void* dst);
void op_interp(const difvm_mesh* m, int dtype, int ncomp, int bc, const void* phi, const void* phib, void* out);
void op_grad(const difvm_mesh* m, int dtype, int ncomp, int bc, const void* phi, const void* phib, void* out);
void op_div(const difvm_mesh* m, int dtype, int scheme, int ncomp, int bc, const void* flux, const void* psi,
            const void* psib, void* out);
void op_laplacian(const difvm_mesh* m, int dtype, int bc, const void* gamma, const void* phi, const void* g,
                  const void* phib, void* out);
void op_ldu_spmv(const difvm_mesh* m, int dtype, int ncomp, int transpose, const void* diag, const void* up,
                 const void* lo, const void* x, void* y);
// halo exchange of a partition part: buf[k] = x[send[k]] (n_send rows of ncomp), and
// x[n_owned + k] = buf[k] for the n_ghost ghost rows
void op_halo_pack(const difvm_mesh* m, int dtype, int ncomp, const void* x, void* buf);
void op_halo_unpack(const difvm_mesh* m, int dtype, int ncomp, const void* buf, void* x);
void op_assemble_laplace(const difvm_mesh* m, int bc, const double* gamma, const double* phib, double* diag,
                         double* upper, double* rhs);

// momentum matrix of the predictor; writes face LDU (upper/lower, may be NULL) and/or per-slot values
// (nu_cell: per-cell viscosity, NULL for nu everywhere); conv adds its deferred correction to b; time
// selects the theta-method (the rest of the matrix part applied to U on the right-hand side)
double time_theta(int scheme);  // DIFVM_TIME_* -> theta of the matrix part (1, 0, 1/2)
void op_assemble_momentum(const difvm_mesh* m, int conv, int time, double nu, const double* nu_cell, double dt,
                          const double* flux, const double* U, const double* gradU, const double* Ub, double* diag,
                          double* upper, double* lower, double* slot_val, double* b);
// deferred-correction source alone (F64): out = - sum_f sigma F (phi^HO - phi^U)
void op_deferred_correction(const difvm_mesh* m, int conv, int ncomp, const double* flux, const double* phi,
                            const double* grad, double* out);

// ---- Krylov solvers on the cell-slot matrix (diag[Nc], val[n_slots]) ----
struct SellMatrix {
  const double* diag;
  const double* val;
};
void sell_from_ldu(const difvm_mesh* m, const double* upper, const double* lower, double* val);
void sell_spmv(const difvm_mesh* m, int ncomp, SellMatrix A, const double* x, double* y);

struct SegResult {
  int iters[3] = {0, 0, 0};
  double res[3] = {0, 0, 0};
  int status = 0;
};
// aggregate (maximum over segments) plus per-segment results
struct SolveResult {
  int iters[3] = {0, 0, 0};
  double res[3] = {0, 0, 0};
  int status = 0;
  std::vector<SegResult> seg;
};

// Solver workspaces live with the mesh-level solver object; created lazily per mesh.
struct KrylovWork;
KrylovWork* krylov_work(difvm_mesh* m);
void krylov_work_free(KrylovWork* w);

// x holds the initial guess; extra_rhs (may be NULL) is subtracted from b as (b - scale_cell * extra)
// per component: used by the predictor for b - V grad(p).
// Queue-only solves (for a captured step): min(budget, maxit) iterations are queued with no host
// synchronisation (iterations after a segment's stop are predicated no-ops) and the per-segment
// solver state is copied to state_out (device, *_state_bytes(m) bytes) at the end; the caller reads
// it back later and turns it into results with *_result, whose `complete` is false when some segment
// had not stopped within the budget.
struct QueueOnly {
  int budget;
  void* state_out;
};
struct AmgDev;
// amg: smoothed-aggregation V-cycle preconditioner instead of Jacobi
// hint (may be NULL): the iteration count of the previous solve made from the same call site; it sizes
// the first block of iterations queued before the host polls, and receives this solve's count.  Each
// call site (a PISO object's predictor, each corrector, scalar transport, adjoint solves, each solve
// entry point of the C-ABI) keeps its own, so a solve never inherits another system's count.
SolveResult pcg(difvm_mesh* m, SellMatrix A, const double* b, double* x, double tol, int maxit,
                const QueueOnly* qo = nullptr, const AmgDev* amg = nullptr, int* hint = nullptr);
SolveResult bicgstab(difvm_mesh* m, int ncomp, SellMatrix A, const double* b, double* x, double tol, int maxit,
                     const QueueOnly* qo = nullptr, int* hint = nullptr);
size_t pcg_state_bytes(const difvm_mesh* m);
int pcg_spmv_grid(const difvm_mesh* m);
size_t bicgstab_state_bytes(const difvm_mesh* m);
SolveResult pcg_result(const difvm_mesh* m, const void* host_state, bool* complete);
SolveResult bicgstab_result(const difvm_mesh* m, int ncomp, const void* host_state, bool* complete);

}  // namespace difvm
