// Host-side mesh layout of libdifvm (plain C++, no HIP): renumbering, permuted geometry and the
// cell-slot (sliced-ELL) layout every cell kernel walks.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/difvm.h"

namespace difvm {

struct LayoutError {
  difvm_status code;
  std::string msg;
};

// ---------------------------------------------------------------------------------------------
// layout constants
// ---------------------------------------------------------------------------------------------
constexpr int SLICE = 64;            // cells per slice of the cell-slot layout (one wavefront)
constexpr int CHUNK = 256;           // cells per reduction partial (fixed: results do not depend on launch shape)
constexpr int BLOCK = 256;           // threads per block for cell and face kernels
constexpr int SLOT_PAD = INT32_MIN;  // slot code of a padding slot

// boundary codes per table
enum : int8_t { BC_FIXED = 0, BC_ZEROGRAD = 1, BC_EMPTY = 2 };
constexpr int N_TABLES = 4;

// slot code: f >= 0 and f < nfi -> owner side of internal face f; f >= nfi -> boundary face f - nfi;
// f < 0 (and != SLOT_PAD) -> neighbour side of internal face -f-1.

// host-side renumbering result (all in new numbering)
struct HostLayout {
  int nc = 0, nfi = 0, nfb = 0, npatch = 0;
  std::vector<int32_t> cell_perm, face_perm, bface_perm, owner, neighbour, own_start, losort, losort_start, bowner;
  std::vector<uint8_t> face_flip;
  std::vector<double> S, w, delta, k, Cf, C, V;   // permuted geometry: S[(nfi+nfb)*3], delta[nfi+nfb], k[nfi*3]
  std::vector<difvm_patch> patches;               // unchanged (boundary ranges are kept)
  std::vector<int8_t> bcode[N_TABLES];            // per boundary face
  std::vector<int32_t> bwk;                       // Windkessel id per boundary face or -1
  int n_wk = 0;
  bool has_fixed_p = false;
  int bandwidth_in = 0, bandwidth_out = 0;
  // cell-slot layout
  int nslice = 0, nslot = 0;
  std::vector<int32_t> slice_start, slot_face, slot_col;
  std::vector<uint8_t> cell_nslot;  // slots of each cell (its own, pads excluded), 255 = 255 or more
  std::vector<int32_t> face_slot_own, face_slot_nbr;   // slot index of each internal face's two sides
  // Windkessel face lists
  std::vector<int32_t> wk_start, wk_faces;
  // segments: independent meshes packed block-diagonally (one segment for a single mesh).  Segment m
  // (user numbering) occupies internal cells [seg_lo[m], seg_hi[m]); reduction tiles of TILE cells
  // start at each segment's first cell and are listed in internal cell order.
  int nseg = 1;
  std::vector<int32_t> seg_user_start, seg_lo, seg_hi, cell_seg;
  std::vector<int32_t> tile_lo, tile_hi, tile_seg, seg_tile_first, seg_tile_n, seg_by_tile_order;
  std::vector<int8_t> seg_has_fixed_p;
};

constexpr int TILE = 1024;  // cells per reduction tile of the Krylov kernels

// Throws LayoutError on invalid input.  seg_start (user cell offsets, nseg+1 entries) may be NULL for
// a single segment; no internal face may join two segments.
void build_layout(const difvm_mesh_desc* d, uint32_t flags, HostLayout& L, bool with_slots, int nseg = 1,
                  const int32_t* seg_start = nullptr);

// ---------------------------------------------------------------------------------------------
// slab partition for a halo exchange: part p owns the contiguous internal cell range [lo, hi) of
// the whole mesh (RCM order, so a slab touches few others) and keeps ghost copies of the cells
// across its cut faces.  Local cell order: owned cells (whole-mesh order), then ghosts (ascending
// whole-mesh index, so the ghosts each other part owns are one contiguous run).
// ---------------------------------------------------------------------------------------------
struct PartMaps {
  int lo = 0, hi = 0, n_owned = 0, n_ghost = 0;
  std::vector<int32_t> cell_global;   // local cell -> whole-mesh internal cell
  std::vector<int32_t> face_global;   // local internal face -> whole-mesh internal face (ascending)
  std::vector<int32_t> bface_global;  // local boundary face -> whole-mesh boundary face (ascending)
  std::vector<int32_t> recv_start;    // [n_parts+1]: ghosts owned by part q are [recv_start[q], recv_start[q+1])
  std::vector<int32_t> send_start;    // [n_parts+1]: cells sent to part q are send_cells[send_start[q] ..]
  std::vector<int32_t> send_cells;    // local indices of owned cells, by destination, ascending in each
};

// Maps of every part of the whole layout G (single segment, with slots); n_parts in [1, G.nc].
void build_partition(const HostLayout& G, int n_parts, std::vector<PartMaps>& parts);
// Layout of one part: its owned cells keep their whole-mesh slots in the same order (so every owned
// row is computed exactly as in the whole mesh), faces keep their whole-mesh orientation, ghost
// cells have no slots.  Permutations are the identity: a part's fields are in its local order.
void build_part_layout(const HostLayout& G, const PartMaps& P, HostLayout& L);


}  // namespace difvm
