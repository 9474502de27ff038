// Smoothed-aggregation AMG: host-side hierarchy (amg_host.cpp) and its device form (amg.hip).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace difvm {

struct AmgError {
  std::string msg;
};

// Square CSR matrix with n rows.  For operators, diag holds the diagonal and ptr/col/val the
// off-diagonal entries only; for transfer operators (P, R) diag is unused and every entry is in CSR.
struct AmgCsr {
  int n = 0;
  std::vector<int32_t> ptr, col;
  std::vector<double> val, diag;
};

// Transfer between level l (fine) and l+1: P (rows of level l, columns of level l+1) and R = P^T.
// For levels l >= 1 also A P (rows of level l) with P's values on its pattern (P_on_AP; the columns
// of row i of A P include those of row i of P, A having a positive diagonal), so that one pass gives
// both P x and A P x; and hi, the upper end of level l's Chebyshev smoothing interval (a bound on the
// spectrum of D^-1 A).  The finest level smooths with the operator of the current solve, which may
// have changed since the setup, so it keeps P alone and its bound is taken on the device side.
struct AmgLevel {
  AmgCsr P, R, AP;
  std::vector<double> P_on_AP;
  double hi = 0.0;
};

struct AmgOptions {
  double theta = 0.0;        // strength-of-connection threshold on coarse levels (0: every coupling)
  double theta_fine = 0.08;  // ... and on the finest
  int radius_fine = 2;       // aggregation over distance-1 or distance-2 strong neighbourhoods
  int radius = 1;
  int max_levels = 12;
  int coarsest = 2048;       // stop coarsening at or below this many rows (below the finest level)
  int tiny = 96;             // the finest level is coarsened when it has more rows than this
  int max_dense = 2048;      // largest coarsest level solved by its dense inverse
};

// levels[l] maps level l to l+1; coarse[l] is the operator of level l+1; the coarsest operator as a
// dense row-major n_coarsest^2 matrix, whose inverse (taken on the device) closes the V-cycle.
struct AmgHierarchy {
  std::vector<int32_t> agg0;  // aggregate of each finest-level row
  std::vector<AmgLevel> levels;
  std::vector<AmgCsr> coarse;
  int n_coarsest = 0;
  std::vector<double> coarsest_dense;
};

// Builds the hierarchy of a symmetric positive definite matrix A0 (diagonal apart).  Throws AmgError.
void amg_build(const AmgCsr& A0, const AmgOptions& opt, AmgHierarchy& H);

}  // namespace difvm
