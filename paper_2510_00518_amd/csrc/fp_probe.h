// Peak probes: short kernels that keep one pipe busy, so that the rooflines the
// benchmark divides by can be measured on the device at hand next to the
// published figures.  Included once, by fp_lib.hip, after fp_mixed.h.
#pragma once

namespace fpk {

constexpr int kProbeChains = 8;  // independent FMA chains per lane
constexpr int kProbeAcc = 4;     // independent matrix-core accumulators per wave

// FP64 vector FMA: kProbeChains chains per lane, 2 FLOP per FMA.
__global__ __launch_bounds__(kBlock) void k_probe_fma64(double* __restrict__ out, int iters) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double a[kProbeChains];
#pragma unroll
    for (int i = 0; i < kProbeChains; ++i) a[i] = 1.0 + 1e-9 * (double)(threadIdx.x + i);
    const double b = 1.0000001, c = 1e-9;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kProbeChains; ++i) a[i] = fma(a[i], b, c);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kProbeChains; ++i) s += a[i];
    out[gid] = s;
}

// Matrix cores: kProbeAcc independent accumulators per wave.  KIND 0:
// v_mfma_f64_16x16x4f64, 1: v_mfma_f32_16x16x4f32 (2048 FLOP each), 2:
// v_mfma_f32_16x16x32_bf16 (16384 FLOP).
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_probe_mfma(double* __restrict__ out, int iters) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    double s = 0.0;
    if constexpr (KIND == 0) {
        d4 acc[kProbeAcc];
#pragma unroll
        for (int i = 0; i < kProbeAcc; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
        const double a = 1e-3 * (double)(lane + 1), b = 0.5;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kProbeAcc; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < kProbeAcc; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    } else if constexpr (KIND == 1) {
        f4v acc[kProbeAcc];
#pragma unroll
        for (int i = 0; i < kProbeAcc; ++i) acc[i] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
        const float a = 1e-3f * (float)(lane + 1), b = 0.5f;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kProbeAcc; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < kProbeAcc; ++i) s += (double)(acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3]);
    } else {
        f4v acc[kProbeAcc];
#pragma unroll
        for (int i = 0; i < kProbeAcc; ++i) acc[i] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
        // bf16 1/64 and 1/2 in every element (0x3C80, 0x3F00)
        const bf16x8 a = as_bf16x8(make_uint4(0x3C803C80u, 0x3C803C80u, 0x3C803C80u, 0x3C803C80u));
        const bf16x8 b = as_bf16x8(make_uint4(0x3F003F00u, 0x3F003F00u, 0x3F003F00u, 0x3F003F00u));
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int i = 0; i < kProbeAcc; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < kProbeAcc; ++i) s += (double)(acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3]);
    }
    out[gid] = s;
}

// HBM: dst[i] = src[i] over n 16-byte elements (grid-stride).
__global__ __launch_bounds__(kBlock) void k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                       int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace fpk
