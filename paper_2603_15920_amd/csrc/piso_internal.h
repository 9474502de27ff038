// PISO object shared by the forward step (piso.hip) and its discrete adjoint (adjoint.hip).
#pragma once

#include "amg_dev.h"
#include "internal.h"
#include "ops.h"

// Captured step (graph mode): the whole step as one hipGraph with a fixed iteration budget per solve
struct PisoGraph {
  bool on = false;
  int extra = 16;                       // largest margin the budgets may carry
  int margin = 1;                       // iterations added to the recent counts (adapts in [0, extra])
  int budget_u = 0, budget_p[8] = {};
  static constexpr int HIST = 8;
  int hist_u[HIST] = {}, hist_p[HIST] = {};  // largest counts of the last steps (ring)
  int nhist = 0, hist_at = 0;
  hipStream_t cap = nullptr;            // private stream the step is captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* state_dev = nullptr;            // solver states after each solve (BiCGStab, then each PCG)
  void* state_host = nullptr;           // pinned copy
  size_t bytes_u = 0, bytes_p = 0;
  double* backup = nullptr;             // U, p, phi, pc before the step
  long long replays = 0, redos = 0, captures = 0;
};

struct difvm_piso {
  difvm_mesh* mesh = nullptr;
  difvm_piso_params prm{};
  int8_t* is_ref = nullptr;  // per internal cell: 1 at the reference cell of a segment with no fixed pressure
  double* nu_cell = nullptr;  // per internal cell kinematic viscosity (the segment's)
  std::vector<double> seg_nu;
  std::vector<difvm_step_stats> seg_stats;  // last step, per segment
  double *U = nullptr, *p = nullptr, *phi = nullptr;
  double *Ub = nullptr, *pb = nullptr, *pbv = nullptr;
  double *wk = nullptr, *pc = nullptr, *wk_out = nullptr;
  double *gU = nullptr, *gp = nullptr, *dM = nullptr, *valM = nullptr, *bM = nullptr, *rhs = nullptr;
  double *HbyA = nullptr, *rAU = nullptr, *phiH = nullptr, *aF = nullptr, *ncorr = nullptr;
  double *dK = nullptr, *valK = nullptr, *rhsK = nullptr;
  double *sc = nullptr, *scb = nullptr, *sg = nullptr, *sd = nullptr, *sval = nullptr, *sb = nullptr;  // scalar step
  std::vector<void*> allocs;
  std::vector<double> wk_host;  // Rp, C, Rd per id
  difvm::AmgDev* amg = nullptr;  // pressure preconditioner hierarchy (built at the first AMG solve)
  int refs = 1;                 // the caller's handle plus one per tape
  PisoGraph g;
  // when set, the step copies the solution of each linear solve here (internal order): the
  // predictor's U* [nc*3] and the pressure after each corrector [n_corr][nc]
  double* trace_U = nullptr;
  double* trace_p = nullptr;
  double* trace_buf = nullptr;  // backing buffer of difvm_piso_step_trace (made at its first call)
  // iterations of the last solve per call site (sizes the first unpolled block of the next one)
  int hint_u = 0, hint_p[8] = {}, hint_sc = 0, hint_adj_u = 0, hint_adj_p[8] = {};
};


namespace difvm {
void piso_release(difvm_piso* P);  // drops one reference (frees at zero, then releases the mesh)

// Intermediates of one forward step kept for its reverse (device buffers owned by the tape).
struct StepRecord {
  static constexpr int MAXC = 8;
  double* phi_in = nullptr;  // lagged flux entering the step [nfi+nfb]
  double* pbv = nullptr;     // boundary pressure values used by the step [nfb]
  double* dM = nullptr;      // momentum diagonal [nc]
  double* valM = nullptr;    // momentum off-diagonals per slot [nslot]
  double* Ustar = nullptr;   // predictor solution [nc*3]
  double* rAU = nullptr;     // V / a_P [nc]
  double* Uin[MAXC] = {};    // velocity entering corrector c [nc*3]
  double* pold[MAXC] = {};   // pressure entering corrector c [nc]
  double* pnew[MAXC] = {};   // pressure solution of corrector c [nc]
  double* HbyA[MAXC] = {};   // [nc*3]
  double* gpo[MAXC] = {};    // grad of the entering pressure [nc*3]
  double* gpn[MAXC] = {};    // grad of the solved pressure [nc*3]
  double* wk_out = nullptr;  // (Q, p_o) per Windkessel [2*n_wk]
  double* pc_in = nullptr;   // capacitor pressures entering the step [n_wk]
  double* Un = nullptr;      // velocity entering the step [nc*3] (kept for a deferred-correction scheme)
};

// one PISO step of P's state; when rec != nullptr the intermediates are copied into it
void piso_advance(difvm_piso* P, difvm_step_stats* st, StepRecord* rec);
// Queue-only variant for capture: every solve queues its fixed budget and leaves its state at its
// QueueOnly::state_out; nothing is read back (st is left untouched).
struct StepQueue {
  QueueOnly u;
  QueueOnly p[StepRecord::MAXC];
};
void piso_advance_q(difvm_piso* P, difvm_step_stats* st, StepRecord* rec, const StepQueue* qu);
// pressure matrix (P->dK, P->valK) from the corrector quantities (also refreshes P->phiH, aF, ncorr, rhsK)
void piso_pressure_matrix(difvm_piso* P, const double* HbyA, const double* rAU, const double* gp, const double* pbv);
void dcopy(double* dst, const double* src, size_t n, hipStream_t s);

}  // namespace difvm
