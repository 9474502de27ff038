// Deferred correction of a higher-order convection scheme (Sec. "Spatial discretization", eq.
// deferred_correction): the upwind face value stays in the matrix and F_f (phi_f^HO - phi_f^U) is
// applied explicitly.  Cell kernels see a face from one side: "self" is the cell the thread owns,
// "other" the cell across the face.  The schemes (C the upwind cell of the face, D the other one,
// g_C the Gauss gradient of C, x_f the face centroid):
//   linear  phi^HO = w phi_O + (1-w) phi_N                 (central differencing)
//   SOU     phi^HO = phi_C + g_C . (x_f - x_C)             (eq. sou)
//   QUICK   phi^HO = phi_C + (phi_D - phi_C)/4 + g_C . (x_D - x_C)/4
// QUICK is the classical 3/8 phi_D + 6/8 phi_C - 1/8 phi_U of a uniform line with the far-upwind value,
// which an unstructured mesh lacks, taken as phi_U = phi_D - 2 g_C . (x_D - x_C).  Only internal faces
// carry a correction.
#pragma once

#include "device.h"

namespace difvm {

// phi^HO - phi^U of one component.  self_up: self is the upwind cell; ws: interpolation weight of
// self; ps/po: values; gs/go: gradients (3 entries); rs/ro: x_f - x_self and x_f - x_other.
template <int CONV>
__device__ __forceinline__ double dc_delta(bool self_up, double ws, double ps, double po, const double* gs,
                                           const double* go, const double4& rs, const double4& ro) {
  double pC = self_up ? ps : po;
  if constexpr (CONV == DIFVM_CONV_LINEAR) {
    return (ws * ps + (1.0 - ws) * po) - pC;
  } else {
    const double* gC = self_up ? gs : go;
    const double4& rC = self_up ? rs : ro;
    if constexpr (CONV == DIFVM_CONV_SOU) {
      return gC[0] * rC.x + gC[1] * rC.y + gC[2] * rC.z;
    } else {
      static_assert(CONV == DIFVM_CONV_QUICK, "unknown convection scheme");
      const double4& rD = self_up ? ro : rs;
      double pD = self_up ? po : ps;
      double gd = gC[0] * (rC.x - rD.x) + gC[1] * (rC.y - rD.y) + gC[2] * (rC.z - rD.z);  // g_C . (x_D - x_C)
      return 0.25 * (pD - pC) + 0.25 * gd;
    }
  }
}

// upwind side test: F >= 0 sends the owner's value (eq. upwind, tie to the owner)
__device__ __forceinline__ bool dc_self_up(double F, bool nb) { return (F >= 0.0) != nb; }

}  // namespace difvm
