// Achievable peaks of the two resources the path is bound by, measured on the
// device at hand: HBM read bandwidth (a streaming read of a large buffer with
// 16-byte loads) and dense bf16 MFMA throughput (independent chains of
// v_mfma_f32_16x16x32_bf16 on register operands).  Rooflines are reported
// against these and against the datasheet figures.
#include "tvcs_internal.h"

#include <algorithm>

namespace tvcs {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kUnroll = 8;

// Sum of the buffer (float4 elements).  Workgroup g reads the contiguous chunk
// [g * per, (g + 1) * per), 8 x 4 KiB in flight per step, with ordinary (NT = false)
// or nontemporal loads.
template <bool NT>
__global__ __launch_bounds__(256) void k_stream_read(const f4 *__restrict__ x, size_t count,
                                                     size_t per, float *__restrict__ out) {
    const size_t begin = blockIdx.x * per, end = begin + per < count ? begin + per : count;
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    size_t i = begin + threadIdx.x;
    for (; i + (kUnroll - 1) * 256 < end; i += kUnroll * 256) {
        f4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            v[u] = NT ? __builtin_nontemporal_load(x + i + u * 256) : x[i + u * 256];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += v[u];
    }
    for (; i < end; i += 256) acc += x[i];
    const float s = acc.x + acc.y + acc.z + acc.w;
    if (s == 1234.5f) out[blockIdx.x] = s;   // keeps the loads; never true for the fill
}

// iters x 8 independent MFMAs per wave.
__global__ __launch_bounds__(256) void k_mfma_loop(int iters, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = (__bf16)(float)((lane + j) & 7);
        b[j] = (__bf16)(float)((lane * 3 + j) & 7);
    }
    f32x4 acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (s == -1.f) out[blockIdx.x] = s;      // keeps the MFMAs; the sums are >= 0
}

__global__ void k_fill_ones(f4 *x, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] = f4{1.f, 1.f, 1.f, 1.f};
}

}  // namespace

void measure_peaks(size_t bytes, int reps, double *read_gbs, double *mfma_tflops) {
    hipStream_t s;
    TVCS_HIP(hipStreamCreate(&s));
    hipEvent_t e0, e1;
    TVCS_HIP(hipEventCreate(&e0));
    TVCS_HIP(hipEventCreate(&e1));
    const size_t count = bytes / sizeof(f4);
    void *buf = nullptr, *out = nullptr;
    TVCS_HIP(hipMalloc(&buf, count * sizeof(f4)));
    TVCS_HIP(hipMalloc(&out, sizeof(float) * 65536));
    float ms = 0.f;
    // HBM read: contiguous chunks, enough workgroups for several per CU; the better
    // of ordinary and nontemporal loads
    const int grid = 8192;
    const size_t per = (count + grid - 1) / grid;
    hipLaunchKernelGGL(k_fill_ones, dim3(4096), dim3(256), 0, s, (f4 *)buf, count);
    double best = 0.0;
    for (int nt = 0; nt < 2; ++nt) {
        auto launch = [&] {
            if (nt)
                hipLaunchKernelGGL(k_stream_read<true>, dim3(grid), dim3(256), 0, s,
                                   (const f4 *)buf, count, per, (float *)out);
            else
                hipLaunchKernelGGL(k_stream_read<false>, dim3(grid), dim3(256), 0, s,
                                   (const f4 *)buf, count, per, (float *)out);
        };
        launch();
        TVCS_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch();
        TVCS_HIP(hipEventRecord(e1, s));
        TVCS_HIP(hipEventSynchronize(e1));
        TVCS_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::max(best, (double)count * sizeof(f4) * reps / (ms * 1e-3) / 1e9);
    }
    if (read_gbs) *read_gbs = best;
    // MFMA: 16 waves per CU (4 per SIMD) on every CU, long independent chains
    const int wgs = 1024, iters = 8192;
    hipLaunchKernelGGL(k_mfma_loop, dim3(wgs), dim3(256), 0, s, 64, (float *)out);
    TVCS_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_mfma_loop, dim3(wgs), dim3(256), 0, s, iters, (float *)out);
    TVCS_HIP(hipEventRecord(e1, s));
    TVCS_HIP(hipEventSynchronize(e1));
    TVCS_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double flops = (double)wgs * 4 * iters * 8 * (16.0 * 16 * 32 * 2) * reps;
    if (mfma_tflops) *mfma_tflops = flops / (ms * 1e-3) / 1e12;
    TVCS_HIP(hipGetLastError());
    (void)hipFree(buf);
    (void)hipFree(out);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
}

}  // namespace tvcs
