// Measured matrix-core peak of the device: every wave of a full-chip launch
// issues long chains of independent MFMAs of one kind (FP64 16x16x4, or the
// BF16 / FP16 16x16x32 forms the split products use) and the rate is taken
// from HIP events.  A diagnostic beside the spec-sheet peaks that the
// factorisation's rates are compared with; no part of the factorisation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tileqr.h"
#include "tileqr_host.h"

namespace tq {

namespace {

typedef double d4p __attribute__((ext_vector_type(4)));
typedef float f4p __attribute__((ext_vector_type(4)));
typedef __bf16 bf8p __attribute__((ext_vector_type(8)));
typedef _Float16 h8p __attribute__((ext_vector_type(8)));

constexpr int CHAINS = 8;   // independent accumulators per wave

// KIND 0: v_mfma_f64_16x16x4_f64; 1: v_mfma_f32_16x16x32_bf16;
// 2: v_mfma_f32_16x16x32_f16.  `iters` rounds of CHAINS MFMAs per wave; the
// accumulators are summed into out[] so that nothing is dead code.
template <int KIND>
__global__ __launch_bounds__(256) void k_mfma_peak(int iters, double seed, double *out)
{
    const int lane = threadIdx.x & 63;
    double r = 0.0;
    if constexpr (KIND == 0) {
        d4p acc[CHAINS];
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = d4p{0.0, 0.0, 0.0, 0.0};
        const double a = seed * (lane + 1), b = seed * 0.5;
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) r += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    } else {
        f4p acc[CHAINS];
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = f4p{0.f, 0.f, 0.f, 0.f};
        if constexpr (KIND == 1) {
            bf8p a, b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = (__bf16)(float)(seed * (lane + e));
                b[e] = (__bf16)(float)(seed * 0.25);
            }
            for (int it = 0; it < iters; ++it)
#pragma unroll
                for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
        } else {
            h8p a, b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = (_Float16)(float)(seed * (lane + e));
                b[e] = (_Float16)(float)(seed * 0.25);
            }
            for (int it = 0; it < iters; ++it)
#pragma unroll
                for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[c], 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) r += (double)(acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3]);
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

}  // namespace

}  // namespace tq

using namespace tq;

extern "C" int tileqr_mfma_peak(int kind, double *tflops)
{
    if (kind < 0 || kind > 2) return -1;
    if (!tflops) return -2;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorNoDevice, "device");
    TQ_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // Four workgroups of four waves per CU: every SIMD holds four waves.
    const int blocks = ncu * 4, threads = 256;
    const int iters = kind == 0 ? 2000 : 8000;
    const double flops_per_mfma = kind == 0 ? 2.0 * 16 * 16 * 4 : 2.0 * 16 * 16 * 32;
    DevBuf out;
    int rc;
    if ((rc = out.ensure((size_t)blocks * threads * sizeof(double)))) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = 0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = hip_fail(hipErrorUnknown, "event");
    float best = -1.f;
    for (int rep = 0; rep < 4 && rc == 0; ++rep) {
        (void)hipEventRecord(e0, nullptr);
        if (kind == 0)
            hipLaunchKernelGGL(k_mfma_peak<0>, dim3(blocks), dim3(threads), 0, nullptr, iters, 1e-3, (double *)out.ptr);
        else if (kind == 1)
            hipLaunchKernelGGL(k_mfma_peak<1>, dim3(blocks), dim3(threads), 0, nullptr, iters, 1e-3, (double *)out.ptr);
        else
            hipLaunchKernelGGL(k_mfma_peak<2>, dim3(blocks), dim3(threads), 0, nullptr, iters, 1e-3, (double *)out.ptr);
        (void)hipEventRecord(e1, nullptr);
        hipError_t err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipGetLastError();
        if (err != hipSuccess) {
            rc = hip_fail(err, "k_mfma_peak");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && (best < 0.f || ms < best)) best = ms;   // the first run warms up
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    out.release();
    if (rc) return rc;
    const double flops = (double)blocks * (threads / 64) * (double)iters * CHAINS * flops_per_mfma;
    *tflops = flops / (best * 1e-3) / 1e12;
    return TILEQR_OK;
}
