// Host mesh preprocessing for libdifvm: validation, reverse Cuthill-McKee renumbering, face
// re-orientation and sorting, permuted geometry with the over-relaxed split, and the cell-slot layout.
//
// The graph being renumbered is the paper's static mesh graph (Sec. "Structural isomorphism ...
// static graph construction"): cells are vertices, internal faces are edges.  RCM packs each cell's
// neighbours close to it in memory so the gathers of the cell kernels stay within a few cache lines
// and within the L2 of the XCD that owns the slice.
//
// Built with strict IEEE host arithmetic (no FMA contraction): geometry is permuted, never
// re-derived, so the permuted arrays are bitwise reproducible from the user's arrays.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "layout.h"

namespace difvm {
namespace {

[[noreturn]] void fail(difvm_status code, const std::string& msg) { throw LayoutError{code, msg}; }

// Counting sort of `idx` (stable) by key[idx[i]] in [0, nkeys).
void counting_sort(std::vector<int32_t>& idx, const std::vector<int32_t>& key, int nkeys) {
  std::vector<int32_t> cnt(nkeys + 1, 0), out(idx.size());
  for (int32_t i : idx) cnt[key[i] + 1]++;
  for (int k = 0; k < nkeys; ++k) cnt[k + 1] += cnt[k];
  for (int32_t i : idx) out[cnt[key[i]]++] = i;
  idx.swap(out);
}

struct Adjacency {
  std::vector<int32_t> ptr, nb, deg;
};

Adjacency adjacency(int nc, int nfi, const int32_t* own, const int32_t* nbr) {
  Adjacency A;
  A.deg.assign(nc, 0);
  for (int f = 0; f < nfi; ++f) { A.deg[own[f]]++; A.deg[nbr[f]]++; }
  A.ptr.assign(nc + 1, 0);
  std::partial_sum(A.deg.begin(), A.deg.end(), A.ptr.begin() + 1);
  A.nb.resize(A.ptr[nc]);
  std::vector<int32_t> pos(A.ptr.begin(), A.ptr.end() - 1);
  for (int f = 0; f < nfi; ++f) {
    A.nb[pos[own[f]]++] = nbr[f];
    A.nb[pos[nbr[f]]++] = own[f];
  }
  return A;
}

// Level structure rooted at r: returns the depth (eccentricity of r) and the deepest level.
// `seen` holds a generation stamp per vertex so repeated searches need no clearing.
int level_structure(const Adjacency& A, int r, std::vector<int32_t>& seen, int32_t gen, std::vector<int32_t>& deepest,
                    std::vector<int32_t>* all = nullptr) {
  std::vector<int32_t> cur{r}, nxt;
  seen[r] = gen;
  if (all) all->push_back(r);
  int depth = 0;
  for (;;) {
    nxt.clear();
    for (int32_t v : cur)
      for (int32_t e = A.ptr[v]; e < A.ptr[v + 1]; ++e) {
        int32_t u = A.nb[e];
        if (seen[u] != gen) {
          seen[u] = gen;
          nxt.push_back(u);
          if (all) all->push_back(u);
        }
      }
    if (nxt.empty()) break;
    cur.swap(nxt);
    ++depth;
  }
  deepest = cur;
  return depth;
}

// Visit order L of reverse Cuthill-McKee: components in order of their lowest cell index; in each,
// start from the (degree, index)-minimal vertex, move to a George-Liu pseudo-peripheral vertex while
// the eccentricity grows, then breadth-first with unvisited neighbours taken by (degree, index).
std::vector<int32_t> rcm_visit_order(int nc, const Adjacency& A) {
  auto before = [&](int32_t a, int32_t b) { return A.deg[a] < A.deg[b] || (A.deg[a] == A.deg[b] && a < b); };
  std::vector<int32_t> seen(nc, -1), placed(nc, 0), L;
  L.reserve(nc);
  int32_t gen = 0;
  std::vector<int32_t> comp, deepest, deepest2, nbrs;
  for (int32_t s = 0; s < nc; ++s) {
    if (placed[s]) continue;
    comp.clear();
    level_structure(A, s, seen, gen++, deepest, &comp);
    int32_t r = *std::min_element(comp.begin(), comp.end(), before);
    int ecc = level_structure(A, r, seen, gen++, deepest);
    for (;;) {
      int32_t x = *std::min_element(deepest.begin(), deepest.end(), before);
      int ecc2 = level_structure(A, x, seen, gen++, deepest2);
      if (ecc2 <= ecc) break;
      r = x;
      ecc = ecc2;
      deepest.swap(deepest2);
    }
    size_t head = L.size();
    L.push_back(r);
    placed[r] = 1;
    while (head < L.size()) {
      int32_t v = L[head++];
      nbrs.clear();
      for (int32_t e = A.ptr[v]; e < A.ptr[v + 1]; ++e)
        if (!placed[A.nb[e]]) nbrs.push_back(A.nb[e]);
      std::sort(nbrs.begin(), nbrs.end(), before);
      nbrs.erase(std::unique(nbrs.begin(), nbrs.end()), nbrs.end());
      for (int32_t u : nbrs) {
        placed[u] = 1;
        L.push_back(u);
      }
    }
  }
  return L;
}

inline double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

}  // namespace

// S = Delta + k with Delta = delta d along the cell-to-cell vector d (eq. nonortho_flux); the scheme
// fixes |Delta|: over-relaxed |S|/|S^.d^|, minimum S.d^, orthogonal |S|; "none" keeps the two-point
// stencil of eq. diff_ortho (|Delta| = |S|) and drops k.  Returns delta, writes k.
static double split_face(uint32_t scheme, const double* S, const double* dv, double* k) {
  double delta;
  if (scheme == DIFVM_NONORTH_MINIMUM)
    delta = dot(S, dv) / dot(dv, dv);
  else if (scheme == DIFVM_NONORTH_ORTHOGONAL || scheme == DIFVM_NONORTH_NONE)
    delta = std::sqrt(dot(S, S)) / std::sqrt(dot(dv, dv));
  else
    delta = dot(S, S) / dot(S, dv);
  for (int c = 0; c < 3; ++c) k[c] = scheme == DIFVM_NONORTH_NONE ? 0.0 : S[c] - delta * dv[c];
  return delta;
}

void build_layout(const difvm_mesh_desc* d, uint32_t flags, HostLayout& L, bool with_slots, int nseg,
                  const int32_t* seg_start) {
  if (!d) fail(DIFVM_ERR_INVALID_ARG, "mesh descriptor is NULL");
  if (d->struct_size != sizeof(difvm_mesh_desc)) fail(DIFVM_ERR_INVALID_ARG, "difvm_mesh_desc.struct_size mismatch");
  const int nc = d->n_cells, nfi = d->n_internal_faces, nfb = d->n_boundary_faces, np = d->n_patches;
  if (nc <= 0 || nfi < 0 || nfb < 0 || np < 0) fail(DIFVM_ERR_INVALID_MESH, "negative or zero counts");
  if (!d->owner || (nfi && !d->neighbour) || !d->Sf || !d->Cf || !d->C || !d->V || (np && !d->patches))
    fail(DIFVM_ERR_INVALID_ARG, "NULL mesh array");
  if (flags & ~(DIFVM_RENUMBER_RCM | DIFVM_NONORTH_MASK)) fail(DIFVM_ERR_INVALID_ARG, "unknown mesh flag bits");
  const uint32_t scheme = flags & DIFVM_NONORTH_MASK;
  const int nf = nfi + nfb;
  for (int f = 0; f < nf; ++f)
    if (d->owner[f] < 0 || d->owner[f] >= nc) fail(DIFVM_ERR_INVALID_MESH, "owner index out of range");
  for (int f = 0; f < nfi; ++f) {
    if (d->neighbour[f] < 0 || d->neighbour[f] >= nc) fail(DIFVM_ERR_INVALID_MESH, "neighbour index out of range");
    if (d->neighbour[f] == d->owner[f]) fail(DIFVM_ERR_INVALID_MESH, "neighbour == owner");
  }
  for (int i = 0; i < nc; ++i)
    if (!(d->V[i] > 0.0)) fail(DIFVM_ERR_INVALID_MESH, "cell volume <= 0");
  // patches must tile [nfi, nfi+nfb) in order
  std::vector<int8_t> empty_face(nfb, 0);
  {
    int at = nfi;
    for (int p = 0; p < np; ++p) {
      const difvm_patch& P = d->patches[p];
      if (P.start != at || P.size < 0) fail(DIFVM_ERR_INVALID_MESH, "patches do not tile the boundary faces");
      if (P.u_type < 0 || P.u_type > 2 || P.p_type < 0 || P.p_type > 3)
        fail(DIFVM_ERR_INVALID_MESH, "unknown patch type");
      if (P.p_type == DIFVM_P_WINDKESSEL && P.windkessel_id < 0) fail(DIFVM_ERR_INVALID_MESH, "Windkessel patch without id");
      bool empty = P.u_type == DIFVM_U_EMPTY || P.p_type == DIFVM_P_EMPTY;
      if (empty) for (int b = 0; b < P.size; ++b) empty_face[P.start - nfi + b] = 1;
      at += P.size;
    }
    if (at != nf) fail(DIFVM_ERR_INVALID_MESH, "patches do not cover the boundary faces");
  }
  // user-orientation checks S.d > 0
  for (int f = 0; f < nfi; ++f) {
    const double* CO = d->C + 3 * d->owner[f];
    const double* CN = d->C + 3 * d->neighbour[f];
    double dd[3] = {CN[0] - CO[0], CN[1] - CO[1], CN[2] - CO[2]};
    if (!(dot(d->Sf + 3 * f, dd) > 0.0)) fail(DIFVM_ERR_INVALID_MESH, "internal face with S.d <= 0");
  }
  for (int b = 0; b < nfb; ++b) {
    if (empty_face[b]) continue;
    int f = nfi + b;
    const double* CO = d->C + 3 * d->owner[f];
    double dd[3] = {d->Cf[3 * f] - CO[0], d->Cf[3 * f + 1] - CO[1], d->Cf[3 * f + 2] - CO[2]};
    if (!(dot(d->Sf + 3 * f, dd) > 0.0)) fail(DIFVM_ERR_INVALID_MESH, "boundary face with S.d <= 0");
  }

  // segments (user cell ranges)
  std::vector<int32_t> useg(nseg + 1);
  if (nseg < 1) fail(DIFVM_ERR_INVALID_ARG, "need at least one segment");
  if (seg_start) {
    for (int s = 0; s <= nseg; ++s) useg[s] = seg_start[s];
    if (useg[0] != 0 || useg[nseg] != nc) fail(DIFVM_ERR_INVALID_ARG, "segments must cover the cells");
    for (int s = 0; s < nseg; ++s)
      if (useg[s + 1] <= useg[s]) fail(DIFVM_ERR_INVALID_ARG, "empty or unordered segment");
  } else {
    if (nseg != 1) fail(DIFVM_ERR_INVALID_ARG, "segment offsets missing");
    useg[0] = 0;
    useg[1] = nc;
  }
  std::vector<int32_t> useg_of(nc);
  for (int s = 0; s < nseg; ++s)
    for (int i = useg[s]; i < useg[s + 1]; ++i) useg_of[i] = s;
  for (int f = 0; f < nfi; ++f)
    if (useg_of[d->owner[f]] != useg_of[d->neighbour[f]]) fail(DIFVM_ERR_INVALID_MESH, "internal face joins two segments");

  L = HostLayout();
  L.nc = nc; L.nfi = nfi; L.nfb = nfb; L.npatch = np;
  L.nseg = nseg;
  L.seg_user_start = useg;
  L.patches.assign(d->patches, d->patches + np);
  for (int f = 0; f < nfi; ++f) L.bandwidth_in = std::max(L.bandwidth_in, std::abs(d->owner[f] - d->neighbour[f]));

  // ---- cell order ----
  std::vector<int32_t> newof(nc);
  L.cell_perm.resize(nc);
  if (flags & DIFVM_RENUMBER_RCM) {
    Adjacency A = adjacency(nc, nfi, d->owner, d->neighbour);
    std::vector<int32_t> visit = rcm_visit_order(nc, A);
    for (int k = 0; k < nc; ++k) {
      int32_t nw = nc - 1 - k;
      L.cell_perm[nw] = visit[k];
      newof[visit[k]] = nw;
    }
  } else {
    std::iota(L.cell_perm.begin(), L.cell_perm.end(), 0);
    std::iota(newof.begin(), newof.end(), 0);
  }

  // ---- segments in internal numbering (each must stay contiguous: true for RCM, since components are
  //      taken in order of their lowest index, and for the identity order) ----
  L.seg_lo.assign(nseg, nc);
  L.seg_hi.assign(nseg, 0);
  for (int i = 0; i < nc; ++i) {
    int s = useg_of[i];
    L.seg_lo[s] = std::min(L.seg_lo[s], newof[i]);
    L.seg_hi[s] = std::max(L.seg_hi[s], newof[i] + 1);
  }
  for (int s = 0; s < nseg; ++s)
    if (L.seg_hi[s] - L.seg_lo[s] != useg[s + 1] - useg[s]) fail(DIFVM_ERR_INVALID_MESH, "segment not contiguous after renumbering");
  L.cell_seg.resize(nc);
  for (int i = 0; i < nc; ++i) L.cell_seg[newof[i]] = useg_of[i];
  {
    std::vector<int32_t> order(nseg);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return L.seg_lo[a] < L.seg_lo[b]; });
    L.seg_by_tile_order = order;
    L.seg_tile_first.assign(nseg, 0);
    L.seg_tile_n.assign(nseg, 0);
    for (int s : order) {
      L.seg_tile_first[s] = (int32_t)L.tile_lo.size();
      for (int a = L.seg_lo[s]; a < L.seg_hi[s]; a += TILE) {
        L.tile_lo.push_back(a);
        L.tile_hi.push_back(std::min(a + TILE, L.seg_hi[s]));
        L.tile_seg.push_back(s);
      }
      L.seg_tile_n[s] = (int32_t)L.tile_lo.size() - L.seg_tile_first[s];
    }
  }

  // ---- internal faces: orient owner < neighbour, sort by (owner, neighbour) keeping input order ----
  std::vector<int32_t> o(nfi), n(nfi), order(nfi);
  std::vector<uint8_t> flip(nfi);
  for (int f = 0; f < nfi; ++f) {
    int32_t a = newof[d->owner[f]], b = newof[d->neighbour[f]];
    flip[f] = a > b;
    o[f] = std::min(a, b);
    n[f] = std::max(a, b);
  }
  std::iota(order.begin(), order.end(), 0);
  counting_sort(order, n, nc);  // least significant key first (stable)
  counting_sort(order, o, nc);
  L.face_perm = order;
  L.face_flip.resize(nfi);
  L.owner.resize(nfi);
  L.neighbour.resize(nfi);
  for (int f = 0; f < nfi; ++f) {
    int g = order[f];
    L.face_flip[f] = flip[g];
    L.owner[f] = o[g];
    L.neighbour[f] = n[g];
    L.bandwidth_out = std::max(L.bandwidth_out, n[g] - o[g]);
  }
  L.own_start.assign(nc + 1, 0);
  for (int f = 0; f < nfi; ++f) L.own_start[L.owner[f] + 1]++;
  std::partial_sum(L.own_start.begin(), L.own_start.end(), L.own_start.begin());
  L.losort.resize(nfi);
  std::iota(L.losort.begin(), L.losort.end(), 0);
  counting_sort(L.losort, L.neighbour, nc);
  L.losort_start.assign(nc + 1, 0);
  for (int f = 0; f < nfi; ++f) L.losort_start[L.neighbour[f] + 1]++;
  std::partial_sum(L.losort_start.begin(), L.losort_start.end(), L.losort_start.begin());

  // ---- boundary faces: stable by new owner inside each patch ----
  L.bface_perm.resize(nfb);
  L.bowner.resize(nfb);
  {
    std::vector<int32_t> bkey(nfb);
    for (int b = 0; b < nfb; ++b) bkey[b] = newof[d->owner[nfi + b]];
    for (int p = 0; p < np; ++p) {
      const difvm_patch& P = d->patches[p];
      std::vector<int32_t> ids(P.size);
      std::iota(ids.begin(), ids.end(), P.start - nfi);
      std::stable_sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) { return bkey[a] < bkey[b]; });
      for (int k = 0; k < P.size; ++k) {
        L.bface_perm[P.start - nfi + k] = ids[k];
        L.bowner[P.start - nfi + k] = bkey[ids[k]];
      }
    }
  }

  // ---- permuted geometry ----
  L.C.resize(3 * (size_t)nc);
  L.V.resize(nc);
  for (int i = 0; i < nc; ++i) {
    int g = L.cell_perm[i];
    L.V[i] = d->V[g];
    for (int c = 0; c < 3; ++c) L.C[3 * i + c] = d->C[3 * g + c];
  }
  L.S.resize(3 * (size_t)nf);
  L.Cf.resize(3 * (size_t)nf);
  L.w.resize(nfi);
  L.delta.resize(nf);
  L.k.resize(3 * (size_t)nfi);
  for (int f = 0; f < nfi; ++f) {
    int g = L.face_perm[f];
    const double* Sg = d->Sf + 3 * g;
    double wg;
    if (d->w) {
      wg = d->w[g];
    } else {
      const double* CO = d->C + 3 * d->owner[g];
      const double* CN = d->C + 3 * d->neighbour[g];
      const double* Cfg = d->Cf + 3 * g;
      double a[3] = {CN[0] - Cfg[0], CN[1] - Cfg[1], CN[2] - Cfg[2]};
      double b[3] = {CN[0] - CO[0], CN[1] - CO[1], CN[2] - CO[2]};
      wg = dot(Sg, a) / dot(Sg, b);
    }
    double* S = &L.S[3 * f];
    for (int c = 0; c < 3; ++c) {
      S[c] = L.face_flip[f] ? -Sg[c] : Sg[c];
      L.Cf[3 * f + c] = d->Cf[3 * g + c];
    }
    L.w[f] = L.face_flip[f] ? 1.0 - wg : wg;
    const double* CO = &L.C[3 * L.owner[f]];
    const double* CN = &L.C[3 * L.neighbour[f]];
    double dv[3] = {CN[0] - CO[0], CN[1] - CO[1], CN[2] - CO[2]};
    L.delta[f] = split_face(scheme, S, dv, &L.k[3 * f]);
  }
  for (int b = 0; b < nfb; ++b) {
    int g = nfi + L.bface_perm[b];
    int f = nfi + b;
    for (int c = 0; c < 3; ++c) {
      L.S[3 * f + c] = d->Sf[3 * g + c];
      L.Cf[3 * f + c] = d->Cf[3 * g + c];
    }
    const double* CO = &L.C[3 * L.bowner[b]];
    double dv[3] = {L.Cf[3 * f] - CO[0], L.Cf[3 * f + 1] - CO[1], L.Cf[3 * f + 2] - CO[2]};
    const double* S = &L.S[3 * f];
    double kb[3];
    L.delta[f] = split_face(scheme, S, dv, kb);  // no correction on boundary faces: kb is unused
  }

  // ---- boundary tables and Windkessel lists (patch ranges are unchanged by the sort) ----
  for (int t = 0; t < N_TABLES; ++t) L.bcode[t].assign(nfb, BC_ZEROGRAD);
  L.bwk.assign(nfb, -1);
  L.seg_has_fixed_p.assign(nseg, 0);
  for (int p = 0; p < np; ++p) {
    const difvm_patch& P = d->patches[p];
    bool empty = P.u_type == DIFVM_U_EMPTY || P.p_type == DIFVM_P_EMPTY;
    if (!empty && (P.p_type == DIFVM_P_FIXED || P.p_type == DIFVM_P_WINDKESSEL))
      for (int b = P.start - nfi; b < P.start - nfi + P.size; ++b) L.seg_has_fixed_p[useg_of[d->owner[nfi + b]]] = 1;
    int8_t cu = empty ? BC_EMPTY : (P.u_type == DIFVM_U_FIXED ? BC_FIXED : BC_ZEROGRAD);
    int8_t cp = empty ? BC_EMPTY
                      : ((P.p_type == DIFVM_P_FIXED || P.p_type == DIFVM_P_WINDKESSEL) ? BC_FIXED : BC_ZEROGRAD);
    if (cp == BC_FIXED) L.has_fixed_p = true;
    if (P.p_type == DIFVM_P_WINDKESSEL) L.n_wk = std::max(L.n_wk, P.windkessel_id + 1);
    for (int b = P.start - nfi; b < P.start - nfi + P.size; ++b) {
      L.bcode[DIFVM_BC_U][b] = cu;
      L.bcode[DIFVM_BC_P][b] = cp;
      L.bcode[DIFVM_BC_ALL_FIXED][b] = empty ? BC_EMPTY : BC_FIXED;
      L.bcode[DIFVM_BC_ALL_ZEROGRAD][b] = empty ? BC_EMPTY : BC_ZEROGRAD;
      if (P.p_type == DIFVM_P_WINDKESSEL) L.bwk[b] = P.windkessel_id;
    }
  }
  L.wk_start.assign(L.n_wk + 1, 0);
  for (int b = 0; b < nfb; ++b) if (L.bwk[b] >= 0) L.wk_start[L.bwk[b] + 1]++;
  std::partial_sum(L.wk_start.begin(), L.wk_start.end(), L.wk_start.begin());
  L.wk_faces.resize(L.wk_start[L.n_wk]);
  {
    std::vector<int32_t> pos(L.wk_start.begin(), L.wk_start.end() - (L.n_wk ? 1 : 0));
    for (int b = 0; b < nfb; ++b) if (L.bwk[b] >= 0) L.wk_faces[pos[L.bwk[b]]++] = b;
  }

  if (!with_slots) return;
  // ---- cell-slot layout: per cell its owner-side faces, neighbour-side faces (losort order), then
  //      its non-empty boundary faces; 64-cell slices padded to the widest cell of the slice ----
  std::vector<int32_t> bstart(nc + 1, 0), blist;
  for (int b = 0; b < nfb; ++b) if (!empty_face[L.bface_perm[b]]) bstart[L.bowner[b] + 1]++;
  std::partial_sum(bstart.begin(), bstart.end(), bstart.begin());
  blist.resize(bstart[nc]);
  {
    std::vector<int32_t> pos(bstart.begin(), bstart.end() - 1);
    for (int b = 0; b < nfb; ++b) if (!empty_face[L.bface_perm[b]]) blist[pos[L.bowner[b]]++] = b;
  }
  L.nslice = (nc + SLICE - 1) / SLICE;
  L.slice_start.assign(L.nslice + 1, 0);
  auto count = [&](int i) {
    return (L.own_start[i + 1] - L.own_start[i]) + (L.losort_start[i + 1] - L.losort_start[i]) + (bstart[i + 1] - bstart[i]);
  };
  L.cell_nslot.resize(nc);
  for (int i = 0; i < nc; ++i) L.cell_nslot[i] = (uint8_t)std::min(count(i), 255);
  for (int s = 0; s < L.nslice; ++s) {
    int wmax = 0;
    for (int i = s * SLICE; i < std::min(nc, (s + 1) * SLICE); ++i) wmax = std::max(wmax, count(i));
    L.slice_start[s + 1] = L.slice_start[s] + wmax * SLICE;
  }
  L.nslot = L.slice_start[L.nslice];
  L.slot_face.assign(L.nslot, SLOT_PAD);
  L.slot_col.assign(L.nslot, 0);
  L.face_slot_own.assign(nfi, -1);
  L.face_slot_nbr.assign(nfi, -1);
  for (int i = 0; i < nc; ++i) {
    int s = i / SLICE, lane = i % SLICE;
    int kslot = 0;
    auto put = [&](int32_t code, int32_t col) {
      size_t at = (size_t)L.slice_start[s] + (size_t)kslot * SLICE + lane;
      L.slot_face[at] = code;
      L.slot_col[at] = col;
      if (code != SLOT_PAD && code < nfi) {
        if (code >= 0) L.face_slot_own[code] = (int32_t)at;
        else L.face_slot_nbr[-code - 1] = (int32_t)at;
      }
      ++kslot;
    };
    for (int f = L.own_start[i]; f < L.own_start[i + 1]; ++f) put(f, L.neighbour[f]);
    for (int q = L.losort_start[i]; q < L.losort_start[i + 1]; ++q) put(-L.losort[q] - 1, L.owner[L.losort[q]]);
    for (int q = bstart[i]; q < bstart[i + 1]; ++q) put(nfi + blist[q], i);
    int width = (L.slice_start[s + 1] - L.slice_start[s]) / SLICE;
    while (kslot < width) put(SLOT_PAD, i);
  }
}

}  // namespace difvm
