// Index arithmetic on an n-point periodic line, shared by the shrink, FFT and DCT
// passes: shifts and masks when n is a power of two (P2), divisions otherwise.
#pragma once

#include <hip/hip_runtime.h>

namespace tvcs {

template <bool P2>
struct Ring {
    int n, ln;
    __device__ explicit Ring(int n_) : n(n_), ln(P2 ? __ffs(n_) - 1 : 0) {}
    __device__ int div(int e) const { return P2 ? e >> ln : e / n; }
    __device__ int mod(int e) const { return P2 ? e & (n - 1) : e - (e / n) * n; }
    __device__ int mul(int i) const { return P2 ? i << ln : i * n; }
    // i in [-1, n] -> i mod n
    __device__ int wrap(int i) const {
        return P2 ? i & (n - 1) : (i < 0 ? i + n : (i >= n ? i - n : i));
    }
    // (n - k) mod n for k in [0, n)
    __device__ int neg(int k) const { return P2 ? (n - k) & (n - 1) : (k == 0 ? 0 : n - k); }
};

}  // namespace tvcs
