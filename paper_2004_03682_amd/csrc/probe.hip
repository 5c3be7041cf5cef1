// Matrix-core throughput probe: the rate the MFMA pipes of this GPU reach,
// at the clock they actually run, on the three matrix instructions the
// library's GEMMs issue (FP64 16x16x4, BF16 16x16x32 with fp32 accumulation,
// FP32 16x16x4).  Each wave runs kChains independent accumulator chains from
// register operands only (no memory traffic inside the loop), four waves per
// workgroup, as many workgroups per compute unit as can be resident at once
// (one round: no partly filled second wave of workgroups); the result is the
// denominator a roofline fraction can be taken against besides the
// spec-sheet peak.  This file is built with -mllvm -amdgpu-mfma-vgpr-form:
// without it the compiler keeps the loop-carried accumulators in VGPRs and
// copies all of them into AGPRs and back around every iteration (two
// register moves per accumulator register and MFMA chain step), which the
// probe would then measure instead of the matrix pipes.
#include <hip/hip_runtime.h>

#include "../../include/fscc.h"

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kChains = 8;
constexpr int kThreads = 256;

// flops of one wave-level instruction
constexpr double kFlops[3] = {2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 32, 2.0 * 16 * 16 * 4};

template <int KIND>
__global__ __launch_bounds__(kThreads) void k_mfma_probe(double* __restrict__ out, int iters) {
    const int t = threadIdx.x;
    double s = 0.0;
    if constexpr (KIND == 0) {
        const double a = 1.0 + 1e-9 * t, b = 1.0 - 1e-9 * t;
        dbl4 acc[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
        int i = 0;
        do {   // iters >= 1 (checked on the host)
#pragma unroll
            for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        } while (++i < iters);
#pragma unroll
        for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    } else if constexpr (KIND == 1) {
        bf8v a, b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            a[e] = (__bf16)(1.0f + 0.001f * (float)((t + e) & 7));
            b[e] = (__bf16)(1.0f - 0.001f * (float)((t + 3 * e) & 7));
        }
        f4v acc[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = f4v{0.f, 0.f, 0.f, 0.f};
        int i = 0;
        do {   // iters >= 1 (checked on the host)
#pragma unroll
            for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
        } while (++i < iters);
#pragma unroll
        for (int c = 0; c < kChains; ++c) s += (double)(acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3]);
    } else {
        const float a = 1.0f + 1e-6f * (float)t, b = 1.0f - 1e-6f * (float)t;
        f4v acc[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = f4v{0.f, 0.f, 0.f, 0.f};
        int i = 0;
        do {   // iters >= 1 (checked on the host)
#pragma unroll
            for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        } while (++i < iters);
#pragma unroll
        for (int c = 0; c < kChains; ++c) s += (double)(acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3]);
    }
    out[(size_t)blockIdx.x * kThreads + t] = s;   // keeps the chains live
}

int resident_per_cu(int kind) {
    int n = 0;
    hipError_t e = kind == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_probe<0>, kThreads, 0)
                 : kind == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_probe<1>, kThreads, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mfma_probe<2>, kThreads, 0);
    return e == hipSuccess ? n : 0;
}

hipError_t launch_probe(int kind, int grid, double* out, int iters, hipStream_t st) {
    if (kind == 0) k_mfma_probe<0><<<grid, kThreads, 0, st>>>(out, iters);
    else if (kind == 1) k_mfma_probe<1><<<grid, kThreads, 0, st>>>(out, iters);
    else k_mfma_probe<2><<<grid, kThreads, 0, st>>>(out, iters);
    return hipGetLastError();
}

}  // namespace

extern "C" fscc_status fscc_probe_mfma(int kind, int iters, void* hip_stream, double* tflops, double* ms) {
    if (kind < 0 || kind > 2 || iters < 1 || iters > (1 << 20) || !tflops) return FSCC_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cus < 1)
        return FSCC_EHIP;
    const int per_cu = resident_per_cu(kind);
    if (per_cu < 1) return FSCC_EHIP;
    const int grid = cus * per_cu;
    double* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    fscc_status rc = FSCC_OK;
    float t = 0.f;
    if (hipMalloc((void**)&out, sizeof(double) * (size_t)grid * kThreads) != hipSuccess) return FSCC_ENOMEM;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = FSCC_EHIP;
        goto done;
    }
    // one untimed launch brings the clock up
    if (launch_probe(kind, grid, out, iters, st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess ||
        launch_probe(kind, grid, out, iters, st) != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess || !(t > 0.f)) {
        rc = FSCC_EHIP;
        goto done;
    }
    *tflops = kFlops[kind] * kChains * (double)iters * 4.0 * grid / (t * 1e-3) / 1e12;
    if (ms) *ms = t;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
