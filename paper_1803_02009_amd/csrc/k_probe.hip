// Calibration kernel for measurement: the achievable dense bf16 matrix-core
// rate of the device, the ceiling a matrix-core kernel's roofline is read
// against (beside the datasheet figure).  Not part of the registration.
#include <hip/hip_runtime.h>

#include "misslam.h"

namespace msl {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;   // four waves
constexpr int kChains = 8;           // independent accumulators per wave

// Each wave runs kChains independent chains of v_mfma_f32_16x16x32_bf16 (16 x 16 x 32 multiply-adds, 16384
// flops each) for iters steps; the operands change every step so that nothing is loop-invariant, and the
// accumulators are stored so that nothing is dead.
__global__ void __launch_bounds__(kProbeThreads) mfma_bf16_probe_kernel(int iters, float *sink) {
    const int lane = threadIdx.x % 64;
    bf16x8_t a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(0.001f * (float)(lane + i));
        b[i] = (__bf16)(0.002f * (float)(lane - i));
    }
    f32x4_t acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f32x4_t{0.f, 0.f, 0.f, (float)c};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
        a[0] = (__bf16)((float)a[0] + 1.0f);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    sink[blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace
}  // namespace msl

extern "C" {

misslam_status misslam_probe_mfma_bf16(int32_t iters, int32_t blocks, float *sink, int64_t *flops, void *stream) {
    if (iters < 1 || blocks < 1 || !sink || !flops) return MISSLAM_EINVAL;
    hipLaunchKernelGGL(msl::mfma_bf16_probe_kernel, dim3(blocks), dim3(msl::kProbeThreads), 0,
                       reinterpret_cast<hipStream_t>(stream), iters, sink);
    *flops = (int64_t)blocks * (msl::kProbeThreads / 64) * iters * msl::kChains * 16384;
    return hipGetLastError() == hipSuccess ? MISSLAM_OK : MISSLAM_EHIP;
}

}  // extern "C"
