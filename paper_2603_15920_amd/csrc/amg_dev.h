// Device form of the smoothed-aggregation AMG preconditioner (amg.hip).
#pragma once

#include "amg.h"
#include "internal.h"
#include "ops.h"

namespace difvm {

struct PcgCtl;
struct AmgDev;

// Builds the hierarchy from the symmetric cell-slot matrix K (copied to the host; synchronises) and
// uploads it.  No face joins two segments, so no aggregate does either and every level stays
// block-diagonal over the segments.  Throws Error.
AmgDev* amg_create(difvm_mesh* m, SellMatrix K, const AmgOptions& opt);
void amg_free(AmgDev* a);
// z = M^-1 r, one symmetric V-cycle (one degree-2 Chebyshev sweep on every level before and after
// each coarse correction, a dense solve on the coarsest; the finest level uses K, the coarser ones
// the stored Galerkin operators), queued on the mesh's stream.  part != nullptr: the last kernel stores per-tile partials of r.z at part[t].
// ctl != nullptr (the per-segment CG states): every kernel returns at once when all segments have
// stopped (iterations queued after the stop).
void amg_vcycle(const AmgDev* a, SellMatrix K, const double* r, double* z, double* part, const PcgCtl* ctl);
// rows per level (finest first) into rows[0..cap); returns the number of levels
int amg_levels(const AmgDev* a, int* rows, int cap);
// Algorithmic bytes of one V-cycle: every kernel's distinct inputs read once and outputs written
// once, the finest level's matrix in its LDU form (diagonal, one coefficient and the owner /
// neighbour indices per internal face), coarse matrices in CSR (row pointers, 4-byte columns, 8-byte
// values, diagonal), the coarsest inverse dense.
double amg_vcycle_bytes(const AmgDev* a);

}  // namespace difvm
