// Smoothed-aggregation algebraic multigrid hierarchy for the pressure matrix (plain C++, host side).
//
// The paper preconditions its pressure CG with ILU; on a GPU an incomplete factorisation runs as long
// chains of dependent triangular sweeps, so the library offers Jacobi (every iteration fully parallel)
// and, as a stronger option, a multigrid V-cycle whose every stage is a parallel sparse product.  The
// hierarchy is built once on the host from one pressure matrix (Vanek-Mandel-Brezina smoothed
// aggregation with the constant vector as near-null space) and then kept fixed: the finest level of
// each V-cycle uses the current matrix, the coarser levels the stored Galerkin operators, so the
// preconditioner stays symmetric positive definite for every solve.
#include "amg.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

namespace difvm {

namespace {

// strong couplings of row i: |a_ij| >= theta sqrt(d_i d_j)
inline bool strong(double aij, double di, double dj, double theta) {
  return std::fabs(aij) >= theta * std::sqrt(std::fabs(di * dj));
}

// Three-phase greedy aggregation in row order.  Returns the number of aggregates; agg[i] in [0, n_agg).
int aggregate1(const AmgCsr& A, double theta, std::vector<int32_t>& agg) {
  const int n = A.n;
  agg.assign(n, -1);
  std::vector<char> phase1(n, 0);
  int na = 0;
  // phase 1: a root whose strong neighbourhood is entirely free takes it whole
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free = true;
    for (int q = A.ptr[i]; q < A.ptr[i + 1] && free; ++q) {
      int j = A.col[q];
      if (strong(A.val[q], A.diag[i], A.diag[j], theta) && agg[j] >= 0) free = false;
    }
    if (!free) continue;
    agg[i] = na;
    for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
      int j = A.col[q];
      if (strong(A.val[q], A.diag[i], A.diag[j], theta)) agg[j] = na;
    }
    ++na;
  }
  for (int i = 0; i < n; ++i) phase1[i] = agg[i] >= 0;
  // phase 2: a free row joins the phase-1 aggregate it is most strongly coupled to
  std::vector<int32_t> join(n, -1);
  for (int i = 0; i < n; ++i) {
    if (phase1[i]) continue;
    double best = 0.0;
    for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
      int j = A.col[q];
      if (!phase1[j] || !strong(A.val[q], A.diag[i], A.diag[j], theta)) continue;
      double s = std::fabs(A.val[q]);
      if (s > best) {
        best = s;
        join[i] = agg[j];
      }
    }
  }
  for (int i = 0; i < n; ++i)
    if (join[i] >= 0) agg[i] = join[i];
  // phase 3: what is left forms aggregates with its free strong neighbours (or alone)
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
      int j = A.col[q];
      if (agg[j] < 0 && strong(A.val[q], A.diag[i], A.diag[j], theta)) agg[j] = na;
    }
    ++na;
  }
  return na;
}

// strong-connection graph squared (distance-2 neighbours), as a CSR pattern with unit values
AmgCsr strong_square(const AmgCsr& A, double theta) {
  const int n = A.n;
  std::vector<int32_t> sp(n + 1, 0), sc;
  for (int i = 0; i < n; ++i) {
    for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
      if (strong(A.val[q], A.diag[i], A.diag[A.col[q]], theta)) sc.push_back(A.col[q]);
    sp[i + 1] = (int32_t)sc.size();
  }
  AmgCsr G;
  G.n = n;
  G.ptr.assign(n + 1, 0);
  G.diag.assign(n, 1.0);
  std::vector<int32_t> mark(n, -1);
  for (int i = 0; i < n; ++i) {
    mark[i] = i;
    for (int q = sp[i]; q < sp[i + 1]; ++q) {
      int j = sc[q];
      if (mark[j] != i) { mark[j] = i; G.col.push_back(j); }
      for (int r = sp[j]; r < sp[j + 1]; ++r) {
        int k = sc[r];
        if (mark[k] != i) { mark[k] = i; G.col.push_back(k); }
      }
    }
    G.ptr[i + 1] = (int32_t)G.col.size();
  }
  G.val.assign(G.col.size(), 1.0);
  return G;
}

int aggregate(const AmgCsr& A, double theta, std::vector<int32_t>& agg, int radius) {
  if (radius <= 1) return aggregate1(A, theta, agg);
  AmgCsr G = strong_square(A, theta);
  return aggregate1(G, 0.0, agg);
}

// largest eigenvalue of D^-1 A by power iteration from a fixed start vector
double spectral_radius_dinv_a(const AmgCsr& A, int iters) {
  const int n = A.n;
  std::vector<double> v(n), w(n);
  for (int i = 0; i < n; ++i) v[i] = 1.0 + 0.5 * std::sin(0.7 * i + 0.3);  // deterministic, not constant
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    double nv = 0.0;
    for (int i = 0; i < n; ++i) nv += v[i] * v[i];
    nv = std::sqrt(nv);
    if (nv == 0.0) return 1.0;
    for (int i = 0; i < n; ++i) v[i] /= nv;
    for (int i = 0; i < n; ++i) {
      double s = A.diag[i] * v[i];
      for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) s += A.val[q] * v[A.col[q]];
      w[i] = s / A.diag[i];
    }
    double num = 0.0;
    for (int i = 0; i < n; ++i) num += v[i] * w[i];
    lam = num;
    v.swap(w);
  }
  return std::max(lam, 1e-12);
}

// transpose of a CSR matrix with m columns
AmgCsr transpose(const AmgCsr& P, int m) {
  AmgCsr R;
  R.n = m;
  R.ptr.assign(m + 1, 0);
  for (int32_t c : P.col) R.ptr[c + 1]++;
  for (int I = 0; I < m; ++I) R.ptr[I + 1] += R.ptr[I];
  R.col.resize(P.col.size());
  R.val.resize(P.val.size());
  std::vector<int32_t> at(R.ptr.begin(), R.ptr.end() - 1);
  for (int i = 0; i < P.n; ++i)
    for (int q = P.ptr[i]; q < P.ptr[i + 1]; ++q) {
      int I = P.col[q];
      R.col[at[I]] = i;
      R.val[at[I]] = P.val[q];
      ++at[I];
    }
  return R;
}

// Sparse accumulator for one row at a time: values summed per column, columns listed in ascending
// order when the row is flushed.
struct SparseAcc {
  std::vector<double> acc;
  std::vector<int32_t> mark, touched;
  int32_t stamp = 0;
  explicit SparseAcc(int n) : acc(n, 0.0), mark(n, -1) {}
  void add(int I, double v) {
    if (mark[I] != stamp) {
      mark[I] = stamp;
      acc[I] = 0.0;
      touched.push_back(I);
    }
    acc[I] += v;
  }
  template <class F>
  void flush(F&& out) {
    std::sort(touched.begin(), touched.end());
    for (int I : touched) out(I, acc[I]);
    touched.clear();
    ++stamp;
  }
};

}  // namespace

// One coarsening step: aggregates, smoothed prolongator P (fine rows), restriction R = P^T (coarse
// rows), Galerkin operator P^T A P (off-diagonals in CSR, diagonal apart, symmetrised exactly), the
// coarse near-null-space vector and, with_ap, A P with P's values on its pattern.
static bool coarsen(const AmgCsr& A, const std::vector<double>& B, double theta, int radius, bool with_ap,
                    AmgLevel& L, AmgCsr& Ac, std::vector<double>& Bc, std::vector<int32_t>& agg) {
  const int n = A.n;
  int na = aggregate(A, theta, agg, radius);
  if (na >= n || na == 0) return false;
  // tentative prolongator: the near-null-space vector restricted to each aggregate, normalised
  Bc.assign(na, 0.0);
  for (int i = 0; i < n; ++i) Bc[agg[i]] += B[i] * B[i];
  for (int I = 0; I < na; ++I) Bc[I] = std::sqrt(Bc[I]);
  std::vector<double> tent(n);
  for (int i = 0; i < n; ++i) tent[i] = Bc[agg[i]] > 0.0 ? B[i] / Bc[agg[i]] : 0.0;
  // smoothed prolongator P = (I - w D^-1 A) P_tent, w = 4 / (3 rho(D^-1 A))
  double w = 4.0 / (3.0 * spectral_radius_dinv_a(A, 20));
  if (with_ap) {
    // upper end of the level's Chebyshev smoothing interval: 1.1 times a longer power iteration's
    // estimate of rho(D^-1 A), at least 1.1 (the eigenvalues of D^-1 A average 1, so rho >= 1), capped
    // by the Gershgorin bound (discs around 1 of radius sum_j |a_ij| / a_ii), which always holds
    double g = 0.0;
    for (int i = 0; i < n; ++i) {
      double off = 0.0;
      for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) off += std::fabs(A.val[q]);
      g = std::max(g, 1.0 + off / A.diag[i]);
    }
    L.hi = std::min(g, 1.1 * std::max(1.0, spectral_radius_dinv_a(A, 50)));
  }
  AmgCsr& P = L.P;
  P.n = n;
  P.ptr.assign(n + 1, 0);
  P.col.clear();
  P.val.clear();
  SparseAcc sa(na);
  for (int i = 0; i < n; ++i) {
    double s = w / A.diag[i];
    sa.add(agg[i], tent[i] - s * A.diag[i] * tent[i]);
    for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
      int j = A.col[q];
      sa.add(agg[j], -s * A.val[q] * tent[j]);
    }
    sa.flush([&](int I, double v) {
      P.col.push_back(I);
      P.val.push_back(v);
    });
    P.ptr[i + 1] = (int32_t)P.col.size();
  }
  L.R = transpose(P, na);
  // A P by fine rows (A = diag + off-diagonals)
  std::vector<int32_t> ap_ptr(n + 1, 0), ap_col;
  std::vector<double> ap_val;
  for (int i = 0; i < n; ++i) {
    for (int q = P.ptr[i]; q < P.ptr[i + 1]; ++q) sa.add(P.col[q], A.diag[i] * P.val[q]);
    for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
      int j = A.col[q];
      for (int r = P.ptr[j]; r < P.ptr[j + 1]; ++r) sa.add(P.col[r], A.val[q] * P.val[r]);
    }
    sa.flush([&](int I, double v) {
      ap_col.push_back(I);
      ap_val.push_back(v);
    });
    ap_ptr[i + 1] = (int32_t)ap_col.size();
  }
  if (with_ap) {
    L.AP.n = n;
    L.AP.ptr = ap_ptr;
    L.AP.col = ap_col;
    L.AP.val = ap_val;
    L.P_on_AP.assign(ap_val.size(), 0.0);
    for (int i = 0; i < n; ++i) {
      int q = P.ptr[i];
      for (int k = ap_ptr[i]; k < ap_ptr[i + 1] && q < P.ptr[i + 1]; ++k)
        if (P.col[q] == ap_col[k]) L.P_on_AP[k] = P.val[q++];
      if (q != P.ptr[i + 1]) throw AmgError{"prolongator pattern not inside that of A P"};
    }
  }
  // A_c = R (A P) by coarse rows
  Ac.n = na;
  Ac.ptr.assign(na + 1, 0);
  Ac.col.clear();
  Ac.val.clear();
  Ac.diag.assign(na, 0.0);
  const AmgCsr& R = L.R;
  for (int I = 0; I < na; ++I) {
    for (int q = R.ptr[I]; q < R.ptr[I + 1]; ++q) {
      int i = R.col[q];
      double r = R.val[q];
      for (int s2 = ap_ptr[i]; s2 < ap_ptr[i + 1]; ++s2) sa.add(ap_col[s2], r * ap_val[s2]);
    }
    sa.flush([&](int J, double v) {
      if (J == I) {
        Ac.diag[I] = v;
      } else {
        Ac.col.push_back(J);
        Ac.val.push_back(v);
      }
    });
    Ac.ptr[I + 1] = (int32_t)Ac.col.size();
  }
  // exact symmetry: a_IJ and a_JI replaced by their mean (rounding made them differ in the last bits)
  AmgCsr T = transpose(Ac, na);
  std::vector<double> sym(Ac.val.size());
  for (int I = 0; I < na; ++I) {
    // rows of Ac and of its transpose hold the same column set (the pattern is symmetric)
    int a = Ac.ptr[I], b = T.ptr[I];
    for (; a < Ac.ptr[I + 1]; ++a) {
      while (b < T.ptr[I + 1] && T.col[b] < Ac.col[a]) ++b;
      double t = (b < T.ptr[I + 1] && T.col[b] == Ac.col[a]) ? T.val[b] : 0.0;
      sym[a] = 0.5 * (Ac.val[a] + t);
    }
  }
  Ac.val.swap(sym);
  return true;
}

void amg_build(const AmgCsr& A0, const AmgOptions& opt, AmgHierarchy& H) {
  H.levels.clear();
  H.coarse.clear();
  H.coarsest_dense.clear();
  std::vector<double> B(A0.n, 1.0);
  AmgCsr A = A0;
  for (int l = 0; l < opt.max_levels; ++l) {
    if (A.n <= (l == 0 ? opt.tiny : opt.coarsest)) break;
    AmgLevel L;
    AmgCsr Ac;
    std::vector<double> Bc;
    std::vector<int32_t> agg;
    if (!coarsen(A, B, l == 0 ? opt.theta_fine : opt.theta, l == 0 ? opt.radius_fine : opt.radius, l > 0, L, Ac, Bc,
                 agg))
      break;
    if (l == 0) H.agg0 = agg;
    if (Ac.n > (int)(0.85 * A.n)) break;  // no real coarsening: stop here
    H.levels.push_back(std::move(L));
    H.coarse.push_back(Ac);
    A = std::move(Ac);
    B = std::move(Bc);
  }
  if (H.levels.empty()) throw AmgError{"the matrix does not coarsen"};
  if (A.n > opt.max_dense) throw AmgError{"coarsest AMG level too large for the dense solve"};
  H.n_coarsest = A.n;
  const size_t n = A.n;
  H.coarsest_dense.assign(n * n, 0.0);
  for (size_t i = 0; i < n; ++i) {
    H.coarsest_dense[i * n + i] = A.diag[i];
    for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) H.coarsest_dense[i * n + A.col[q]] = A.val[q];
  }
}

}  // namespace difvm
