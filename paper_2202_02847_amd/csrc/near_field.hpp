// Host-side launchers of the near-field and segmented-sum kernels (k_aux.hip), used by the FMM
// driver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace shfmm {

// P2P: near field of `count` boxes of `npts` particles each; box c's neighbours (itself
// included) are nbr[27c .. 27c+26] (-1 for none); adds sum q/|x-y| and its gradient per
// target into out (4 doubles per particle; flags bit 0: accumulate, else overwrite).
hipError_t launch_p2p(int64_t count, int64_t npts, const double *pts, const double *q, const int32_t *nbr,
                      double *out, unsigned flags, hipStream_t s);

// L[b] = sum of the solids scratch[t - base], t in [seg[b], seg[b+1]), for b in [tb, te)
// (S reals per solid).
hipError_t launch_seg_sum(double *L, int64_t S, const int64_t *seg, int64_t tb, int64_t te, int64_t base,
                          const double *scratch, hipStream_t s);

}  // namespace shfmm
