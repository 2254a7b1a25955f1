// The stop rule on the device: applied after the inverse row pass (k_stop_rule in
// fft.hip) or, for one image, by the first workgroup of the next iteration's A u
// product (gemv.hip), which saves a launch per iteration.
#pragma once

#include <hip/hip_runtime.h>

#include "tvcs_internal.h"

namespace tvcs {

// The stop rule of eq. (stop), ||u^{k+1} - u^k|| <= tol ||u^k|| (inclusive, FP64),
// for one image from its row blocks' partial sums (added in block order by one
// 64-lane wave, so the result does not depend on how the pass was launched).
__device__ inline void stop_rule(ImgState *st, const double *parts, int nparts, int *counter) {
    const int lane = threadIdx.x & 63;
    double sd = 0.0, su = 0.0;
    for (int p = lane; p < nparts; p += 64) {
        sd += __hip_atomic_load(parts + 2 * p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        su += __hip_atomic_load(parts + 2 * p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sd += __shfl_xor(sd, off, 64);
        su += __shfl_xor(su, off, 64);
    }
    if (lane == 0) {
        ImgState s = *st;
        s.iters += 1;
        s.du2 = sd;
        s.u2 = su;
        const double du = sqrt(sd), nu = sqrt(su);
        s.rel = nu > 0.0 ? du / nu : (du > 0.0 ? INFINITY : 0.0);
        if (!isfinite(sd) || !isfinite(su)) {
            s.status = TVCS_ENONFINITE;
            s.active = 0;
        } else if (s.tol > 0.0 && du <= s.tol * nu) {
            s.status = TVCS_OK;
            s.active = 0;
        } else if (s.iters >= s.maxit) {
            s.status = s.tol > 0.0 ? TVCS_MAXIT : TVCS_OK;
            s.active = 0;
        }
        *st = s;
        if (counter) *counter = 0;   // ready for the next pass
    }
}

}  // namespace tvcs
