// Slab partition of a renumbered mesh for a halo exchange (host, plain C++).
//
// The paper runs one mesh on one GPU and names multi-GPU partitioning as future work (Sec.
// "Limitations and Future Work").  With the face-graph form each operator reads, for a cell, only
// its own row of slots and the values of the cells across its faces, so a part that owns a range of
// cells can compute those rows exactly as the whole mesh does once it holds copies ("ghosts") of
// the cells across its cut faces: one exchange of the operator's cell inputs per face kernel.  The
// reverse Cuthill-McKee order makes contiguous ranges good slabs: level sets of the breadth-first
// order sweep across the mesh, so a slab has at most two neighbouring slabs when the slabs are
// wider than the bandwidth.
#include <algorithm>
#include <numeric>

#include "layout.h"

namespace difvm {
namespace {

[[noreturn]] void fail(difvm_status code, const std::string& msg) { throw LayoutError{code, msg}; }

int part_of(const std::vector<int>& lo, int cell) {
  // lo is ascending with lo[0] = 0: the last part whose first cell is <= cell
  return (int)(std::upper_bound(lo.begin(), lo.end() - 1, cell) - lo.begin()) - 1;
}

// true non-padding slots of whole-mesh cell g, in layout order
template <class F>
void for_slots(const HostLayout& G, int g, F&& f) {
  int s = g / SLICE, lane = g % SLICE;
  int width = (G.slice_start[s + 1] - G.slice_start[s]) / SLICE;
  for (int k = 0; k < width; ++k) {
    size_t at = (size_t)G.slice_start[s] + (size_t)k * SLICE + lane;
    if (G.slot_face[at] == SLOT_PAD) break;  // padding only follows a cell's own slots
    f(G.slot_face[at], G.slot_col[at]);
  }
}

}  // namespace

void build_partition(const HostLayout& G, int n_parts, std::vector<PartMaps>& parts) {
  if (G.nseg != 1) fail(DIFVM_ERR_UNSUPPORTED, "a packed (segmented) mesh cannot be partitioned");
  if (n_parts < 1 || n_parts > G.nc) fail(DIFVM_ERR_INVALID_ARG, "n_parts must be in [1, n_cells]");
  if (G.slot_face.empty() && G.nc) fail(DIFVM_ERR_INVALID_ARG, "partition needs the cell-slot layout");
  std::vector<int> lo(n_parts + 1);
  for (int p = 0; p <= n_parts; ++p) lo[p] = (int)((int64_t)p * G.nc / n_parts);
  parts.assign(n_parts, PartMaps());
  for (int p = 0; p < n_parts; ++p) {
    PartMaps& P = parts[p];
    P.lo = lo[p];
    P.hi = lo[p + 1];
    P.n_owned = P.hi - P.lo;
    // faces with an owned owner are one owner-sorted run; faces with an owned neighbour and a ghost
    // owner (owner < lo) come before it in face order
    std::vector<int32_t> ghosts, before;
    for (int f = G.own_start[P.lo]; f < G.own_start[P.hi]; ++f)
      if (G.neighbour[f] >= P.hi) ghosts.push_back(G.neighbour[f]);
    for (int q = G.losort_start[P.lo]; q < G.losort_start[P.hi]; ++q) {
      int f = G.losort[q];
      if (G.owner[f] < P.lo) {
        ghosts.push_back(G.owner[f]);
        before.push_back(f);
      }
    }
    std::sort(ghosts.begin(), ghosts.end());
    ghosts.erase(std::unique(ghosts.begin(), ghosts.end()), ghosts.end());
    std::sort(before.begin(), before.end());
    P.n_ghost = (int)ghosts.size();
    P.cell_global.resize(P.n_owned + P.n_ghost);
    std::iota(P.cell_global.begin(), P.cell_global.begin() + P.n_owned, P.lo);
    std::copy(ghosts.begin(), ghosts.end(), P.cell_global.begin() + P.n_owned);
    P.face_global = before;
    for (int f = G.own_start[P.lo]; f < G.own_start[P.hi]; ++f) P.face_global.push_back(f);
    for (int b = 0; b < G.nfb; ++b)
      if (G.bowner[b] >= P.lo && G.bowner[b] < P.hi) P.bface_global.push_back(b);
    P.recv_start.assign(n_parts + 1, 0);
    for (int g : ghosts) P.recv_start[part_of(lo, g) + 1]++;
    std::partial_sum(P.recv_start.begin(), P.recv_start.end(), P.recv_start.begin());
  }
  // part p sends to q the cells of p that q holds as ghosts, in q's ghost order
  std::vector<std::vector<std::vector<int32_t>>> out(n_parts, std::vector<std::vector<int32_t>>(n_parts));
  for (int q = 0; q < n_parts; ++q) {
    const PartMaps& Q = parts[q];
    for (int k = Q.n_owned; k < Q.n_owned + Q.n_ghost; ++k) {
      int g = Q.cell_global[k];
      int p = part_of(lo, g);
      out[p][q].push_back(g - parts[p].lo);
    }
  }
  for (int p = 0; p < n_parts; ++p) {
    PartMaps& P = parts[p];
    P.send_start.assign(n_parts + 1, 0);
    for (int q = 0; q < n_parts; ++q) {
      P.send_start[q + 1] = P.send_start[q] + (int32_t)out[p][q].size();
      P.send_cells.insert(P.send_cells.end(), out[p][q].begin(), out[p][q].end());
    }
  }
}

void build_part_layout(const HostLayout& G, const PartMaps& P, HostLayout& L) {
  const int nc = P.n_owned + P.n_ghost, nfi = (int)P.face_global.size(), nfb = (int)P.bface_global.size();
  std::vector<int32_t> cloc(G.nc, -1), floc(G.nfi, -1), bloc(G.nfb, -1);
  for (int i = 0; i < nc; ++i) cloc[P.cell_global[i]] = i;
  for (int f = 0; f < nfi; ++f) floc[P.face_global[f]] = f;
  for (int b = 0; b < nfb; ++b) bloc[P.bface_global[b]] = b;

  L = HostLayout();
  L.nc = nc; L.nfi = nfi; L.nfb = nfb; L.npatch = G.npatch;
  L.cell_perm.resize(nc);
  std::iota(L.cell_perm.begin(), L.cell_perm.end(), 0);
  L.face_perm.resize(nfi);
  std::iota(L.face_perm.begin(), L.face_perm.end(), 0);
  L.face_flip.assign(nfi, 0);
  L.bface_perm.resize(nfb);
  std::iota(L.bface_perm.begin(), L.bface_perm.end(), 0);

  // cells
  L.C.resize(3 * (size_t)nc);
  L.V.resize(nc);
  for (int i = 0; i < nc; ++i) {
    int g = P.cell_global[i];
    L.V[i] = G.V[g];
    for (int c = 0; c < 3; ++c) L.C[3 * i + c] = G.C[3 * g + c];
  }
  // internal faces (whole-mesh orientation and values)
  L.owner.resize(nfi);
  L.neighbour.resize(nfi);
  L.w.resize(nfi);
  L.k.resize(3 * (size_t)nfi);
  L.S.resize(3 * (size_t)(nfi + nfb));
  L.Cf.resize(3 * (size_t)(nfi + nfb));
  L.delta.resize(nfi + nfb);
  for (int f = 0; f < nfi; ++f) {
    int g = P.face_global[f];
    L.owner[f] = cloc[G.owner[g]];
    L.neighbour[f] = cloc[G.neighbour[g]];
    L.w[f] = G.w[g];
    L.delta[f] = G.delta[g];
    for (int c = 0; c < 3; ++c) {
      L.S[3 * f + c] = G.S[3 * g + c];
      L.Cf[3 * f + c] = G.Cf[3 * g + c];
      L.k[3 * f + c] = G.k[3 * g + c];
    }
    L.bandwidth_out = std::max(L.bandwidth_out, std::abs(L.neighbour[f] - L.owner[f]));
  }
  L.bandwidth_in = L.bandwidth_out;
  // owner / neighbour index lists of the local faces (kept for completeness: the kernels walk slots)
  L.own_start.assign(nc + 1, 0);
  L.losort_start.assign(nc + 1, 0);
  for (int f = 0; f < nfi; ++f) {
    L.own_start[L.owner[f] + 1]++;
    L.losort_start[L.neighbour[f] + 1]++;
  }
  std::partial_sum(L.own_start.begin(), L.own_start.end(), L.own_start.begin());
  std::partial_sum(L.losort_start.begin(), L.losort_start.end(), L.losort_start.begin());
  L.losort.resize(nfi);
  {
    std::vector<int32_t> pos(L.losort_start.begin(), L.losort_start.end() - 1);
    for (int f = 0; f < nfi; ++f) L.losort[pos[L.neighbour[f]]++] = f;
  }
  // boundary faces: the whole mesh's order restricted to the part, patch ranges recounted
  L.bowner.resize(nfb);
  for (int b = 0; b < nfb; ++b) {
    int g = P.bface_global[b];
    L.bowner[b] = cloc[G.bowner[g]];
    L.delta[nfi + b] = G.delta[G.nfi + g];
    for (int c = 0; c < 3; ++c) {
      L.S[3 * (nfi + b) + c] = G.S[3 * (G.nfi + g) + c];
      L.Cf[3 * (nfi + b) + c] = G.Cf[3 * (G.nfi + g) + c];
    }
  }
  L.patches = G.patches;
  {
    int at = nfi;
    for (auto& pt : L.patches) {
      int g0 = pt.start - G.nfi, g1 = g0 + pt.size;
      int n = (int)(std::lower_bound(P.bface_global.begin(), P.bface_global.end(), g1) -
                    std::lower_bound(P.bface_global.begin(), P.bface_global.end(), g0));
      pt.start = at;
      pt.size = n;
      at += n;
    }
  }
  for (int t = 0; t < N_TABLES; ++t) {
    L.bcode[t].resize(nfb);
    for (int b = 0; b < nfb; ++b) L.bcode[t][b] = G.bcode[t][P.bface_global[b]];
  }
  L.bwk.resize(nfb);
  for (int b = 0; b < nfb; ++b) L.bwk[b] = G.bwk[P.bface_global[b]];
  L.n_wk = G.n_wk;
  L.has_fixed_p = G.has_fixed_p;
  L.wk_start.assign(L.n_wk + 1, 0);
  for (int b = 0; b < nfb; ++b) if (L.bwk[b] >= 0) L.wk_start[L.bwk[b] + 1]++;
  std::partial_sum(L.wk_start.begin(), L.wk_start.end(), L.wk_start.begin());
  L.wk_faces.resize(L.wk_start[L.n_wk]);
  {
    std::vector<int32_t> pos(L.wk_start.begin(), L.wk_start.end() - (L.n_wk ? 1 : 0));
    for (int b = 0; b < nfb; ++b) if (L.bwk[b] >= 0) L.wk_faces[pos[L.bwk[b]]++] = b;
  }
  // one segment over every local cell
  L.nseg = 1;
  L.seg_user_start = {0, nc};
  L.seg_lo = {0};
  L.seg_hi = {nc};
  L.cell_seg.assign(nc, 0);
  L.seg_by_tile_order = {0};
  L.seg_tile_first = {0};
  for (int a = 0; a < nc; a += TILE) {
    L.tile_lo.push_back(a);
    L.tile_hi.push_back(std::min(a + TILE, nc));
    L.tile_seg.push_back(0);
  }
  L.seg_tile_n = {(int32_t)L.tile_lo.size()};
  L.seg_has_fixed_p = {(int8_t)(G.has_fixed_p ? 1 : 0)};

  // cell-slot layout: an owned cell's whole-mesh slots in their order, codes and columns mapped to
  // local indices; ghost cells have none
  std::vector<int> count(nc, 0);
  for (int i = 0; i < P.n_owned; ++i) for_slots(G, P.cell_global[i], [&](int32_t, int32_t) { count[i]++; });
  L.nslice = (nc + SLICE - 1) / SLICE;
  L.slice_start.assign(L.nslice + 1, 0);
  L.cell_nslot.resize(nc);
  for (int i = 0; i < nc; ++i) L.cell_nslot[i] = (uint8_t)std::min(count[i], 255);
  for (int s = 0; s < L.nslice; ++s) {
    int wmax = 0;
    for (int i = s * SLICE; i < std::min(nc, (s + 1) * SLICE); ++i) wmax = std::max(wmax, count[i]);
    L.slice_start[s + 1] = L.slice_start[s] + wmax * SLICE;
  }
  L.nslot = L.slice_start[L.nslice];
  L.slot_face.assign(L.nslot, SLOT_PAD);
  L.slot_col.assign(L.nslot, 0);
  L.face_slot_own.assign(nfi, -1);
  L.face_slot_nbr.assign(nfi, -1);
  for (int i = 0; i < nc; ++i) {
    int s = i / SLICE, lane = i % SLICE;
    int width = (L.slice_start[s + 1] - L.slice_start[s]) / SLICE;
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
    if (i < P.n_owned) {
      for_slots(G, P.cell_global[i], [&](int32_t code, int32_t col) {
        int32_t lc;
        if (code >= G.nfi) lc = nfi + bloc[code - G.nfi];
        else if (code >= 0) lc = floc[code];
        else lc = -floc[-code - 1] - 1;
        put(lc, cloc[col]);
      });
    }
    while (kslot < width) put(SLOT_PAD, i);
  }
}

}  // namespace difvm
