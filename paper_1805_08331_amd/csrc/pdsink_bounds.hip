// Launches of the pair-kernel variant that also computes the error-control
// bounds.  It lives in a translation unit of its own: instantiated next to the
// plain variant, it changes the plain kernel's register allocation.
#include <hip/hip_runtime.h>

#include "pdsink_device.h"
#include "sinkhorn_pair.h"

namespace pdsink {

namespace {
int launch_err() { return hipGetLastError() == hipSuccess ? 0 : -1; }

template <int D>
int launch_bounds_levels(PairParams pp, int n_slots, hipStream_t st) {
  pp.only_redo = 0;
  const unsigned g0 = D > 128 ? (unsigned)n_slots : (unsigned)pp.n_pairs;
  hipLaunchKernelGGL((sinkhorn_pair_kernel<D, 1, true>), dim3(g0), dim3(PWGS), 0, st, pp);
  if (launch_err()) return -1;
  pp.only_redo = 1;
  hipLaunchKernelGGL((sinkhorn_pair_kernel<D, 0, true>), dim3((unsigned)n_slots), dim3(PWGS), 0, st, pp);
  return launch_err();
}
}  // namespace

// Level 0 then level 1 of the bounds variant (same routing as the plain
// solve); returns 0, or -1 when a launch failed.
int launch_pair_bounds(int D, PairParams pp, int n_slots, hipStream_t st) {
  switch (D) {
    case 32: return launch_bounds_levels<32>(pp, n_slots, st);
    case 64: return launch_bounds_levels<64>(pp, n_slots, st);
    case 128: return launch_bounds_levels<128>(pp, n_slots, st);
    default: return launch_bounds_levels<256>(pp, n_slots, st);
  }
}

}  // namespace pdsink
