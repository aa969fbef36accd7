// Measured issue rate of non-packed FP32 fused multiply-adds on the current
// GPU, and the shader clock it ran at: the denominator the benchmark puts
// beside the nominal VALU peak (256 CUs x 64 lanes x 2.4 GHz) when it reports
// the ray-test work as a fraction of what the vector unit can issue.
#include <hip/hip_runtime.h>

#include "srp.h"

namespace {

constexpr int PEAK_BLOCK = 256;
constexpr int PEAK_CHAINS = 8;   // independent dependency chains per lane

// Every lane runs PEAK_CHAINS independent chains of `iters` FMAs (v_fma_f32 /
// v_fmac_f32: packed FP32 is disabled for all code of this library); lane 0
// of block 0 records the shader clock and the constant-rate wall clock around
// its loop.  The sum is stored so that nothing is optimised away.
__global__ __launch_bounds__(PEAK_BLOCK) void k_fma_peak(float *out, int iters, float m, float c,
                                                       unsigned long long *clocks) {
    float a[PEAK_CHAINS];
    for (int k = 0; k < PEAK_CHAINS; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f;
    const unsigned long long s0 = clock64(), w0 = wall_clock64();
#pragma unroll 1
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int k = 0; k < PEAK_CHAINS; ++k) a[k] = fmaf(a[k], m, c);
    }
    const unsigned long long s1 = clock64(), w1 = wall_clock64();
    float s = 0.0f;
    for (int k = 0; k < PEAK_CHAINS; ++k) s += a[k];
    out[blockIdx.x * PEAK_BLOCK + threadIdx.x] = s;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clocks[0] = s1 - s0;
        clocks[1] = w1 - w0;
    }
}

}  // namespace

extern "C" int srp_valu_peak(double *lane_fma_per_s, double *shader_ghz, int32_t *n_cu) {
    if (!lane_fma_per_s || !shader_ghz || !n_cu) return SRP_ERR_ARG;
    int dev = 0, cus = 0, wall_khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return SRP_ERR_DEVICE;
    const int blocks = cus * 8;        // 8 blocks of 4 waves per CU: 8 waves per SIMD
    const int iters = 1 << 13;         // x 8 unrolled x 8 chains FMAs per lane
    float *out = nullptr;
    unsigned long long *clk = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SRP_OK;
    if (hipMalloc(&out, sizeof(float) * (size_t)blocks * PEAK_BLOCK) != hipSuccess ||
        hipMalloc(&clk, 2 * sizeof(unsigned long long)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = SRP_ERR_DEVICE;
    }
    float ms = 0.0f;
    unsigned long long hc[2] = {0, 0};
    if (!rc) {
        // one warm-up launch, then the timed one (the clock ramps up under load)
        hipLaunchKernelGGL(k_fma_peak, dim3(blocks), dim3(PEAK_BLOCK), 0, 0, out, iters, 0.9999f, 1e-4f, clk);
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(k_fma_peak, dim3(blocks), dim3(PEAK_BLOCK), 0, 0, out, iters, 0.9999f, 1e-4f, clk);
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
            hipMemcpy(hc, clk, sizeof hc, hipMemcpyDeviceToHost) != hipSuccess || hipGetLastError() != hipSuccess)
            rc = SRP_ERR_DEVICE;
    }
    if (!rc) {
        const double fma = (double)blocks * PEAK_BLOCK * (double)iters * 8.0 * PEAK_CHAINS;
        *lane_fma_per_s = fma / (ms * 1e-3);
        *shader_ghz = hc[1] ? (double)hc[0] / ((double)hc[1] / ((double)wall_khz * 1e3)) / 1e9 : 0.0;
        *n_cu = cus;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (clk) (void)hipFree(clk);
    return rc;
}
