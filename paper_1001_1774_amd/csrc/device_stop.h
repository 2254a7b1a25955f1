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
// slot >= 0: also sets mode[slot] = 1 (fresh products two iterations later) when
// the relative change exceeds kFreshTheta or that iteration is a multiple of
// kFreshEvery.  Only the fields the rule changes are written: other passes of the
// next iteration may read mode[] of this image while the rule runs.
__device__ inline void stop_rule(ImgState *st, const double *parts, int nparts, int *counter,
                                 int slot = -1) {
    const int lane = threadIdx.x & 63;
    // the fields the rule reads are loaded with the partials (one round trip); an
    // image that is no longer active is left alone
    int iters = 0, status = 0, active = 0, maxit = 0;
    double tol = 0.0;
    if (lane == 0) {
        iters = st->iters + 1;
        status = st->status;
        active = st->active;
        tol = st->tol;
        maxit = st->maxit;
    }
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
    if (lane == 0 && active) {
        const double du = sqrt(sd), nu = sqrt(su);
        const double rel = nu > 0.0 ? du / nu : (du > 0.0 ? INFINITY : 0.0);
        if (!isfinite(sd) || !isfinite(su)) {
            status = TVCS_ENONFINITE;
            active = 0;
        } else if (tol > 0.0 && du <= tol * nu) {
            status = TVCS_OK;
            active = 0;
        } else if (iters >= maxit) {
            status = tol > 0.0 ? TVCS_MAXIT : TVCS_OK;
            active = 0;
        }
        st->iters = iters;
        st->du2 = sd;
        st->u2 = su;
        st->rel = rel;
        st->status = status;
        st->active = active;
        // iteration `iters - 1` just ended with the mode in mode[slot]; the slot now
        // takes the mode of iteration iters + 1
        if (slot >= 0) {
            st->fresh += st->mode[slot];
            st->mode[slot] = (rel > kFreshTheta || (iters + 1) % kFreshEvery == 0) ? 1 : 0;
        }
        if (counter) *counter = 0;   // ready for the next pass
    }
}

}  // namespace tvcs
