// Index arithmetic on an n-point periodic line, shared by the shrink, FFT and DCT
// passes: shifts and masks when n is a power of two (P2), divisions otherwise.
#pragma once

#include <hip/hip_runtime.h>

namespace tvcs {

// floor(e / d) for 0 <= e < 2^22 and 1 <= d < 2^22, with rd = 1.0f / d: the FP32
// product is within one of the quotient (relative error below 2^-22.9 on a value
// below 2^22), and one step on the remainder makes it exact.  Integer division by
// a run-time value is a long instruction sequence on the GPU.
__device__ inline int div_by(int e, int d, float rd) {
    int q = (int)((float)e * rd);
    const int r = e - q * d;
    return q + (r >= d) - (r < 0);
}

template <bool P2>
struct Ring {
    int n, ln;
    float rn;
    __device__ explicit Ring(int n_)
        : n(n_), ln(P2 ? __ffs(n_) - 1 : 0), rn(P2 ? 0.f : 1.0f / (float)n_) {}
    __device__ int div(int e) const { return P2 ? e >> ln : div_by(e, n, rn); }
    __device__ int mod(int e) const { return P2 ? e & (n - 1) : e - div(e) * n; }
    __device__ int mul(int i) const { return P2 ? i << ln : i * n; }
    // i in [-1, n] -> i mod n
    __device__ int wrap(int i) const {
        return P2 ? i & (n - 1) : (i < 0 ? i + n : (i >= n ? i - n : i));
    }
    // (n - k) mod n for k in [0, n)
    __device__ int neg(int k) const { return P2 ? (n - k) & (n - 1) : (k == 0 ? 0 : n - k); }
};

}  // namespace tvcs
