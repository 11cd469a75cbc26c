// Issue rate of non-packed FP32 FMAs on one GPU, as a ceiling for the field
// pass's inner loop (which uses v_fmac_f32 only: packed FP32 is switched off in
// this library).  Each wave runs `iters` blocks of 128 FMAs over 16
// independent accumulators (8 multipliers, a ring of 8 two-component values,
// the same shape as a W = 8 block of the field pass), optionally with one LDS
// read per 16 FMAs as in that loop.  The grid holds k waves per SIMD (1024 k
// single-wave workgroups on 256 CUs x 4 SIMDs).  The shader clock during the
// run is taken from s_memtime against the 100 MHz s_memrealtime counter.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2403_07666_amd/calib/fp32_fma_rate.hip -o /tmp/fp32_fma_rate && /tmp/fp32_fma_rate
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                      \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));              \
            std::exit(1);                                                             \
        }                                                                             \
    } while (0)

template <int LDSRD>
__global__ __launch_bounds__(64) void k_fma(float *out, long long *clk, int iters, float a0) {
    __shared__ float2 t[512];
    const int lane = threadIdx.x;
    const long long c0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
    for (int i = lane; i < 512; i += 64) t[i] = make_float2(i * 1e-3f, i * 2e-3f);
    __syncthreads();
    float acc[16], m[8];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = lane * 1e-3f + i;
#pragma unroll
    for (int i = 0; i < 8; ++i) m[i] = a0 + i * 1e-4f;
    float2 g[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) g[i] = t[(lane + i * 64) & 511];
    int base = lane;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                acc[c] = fmaf(g[(c - u + 8) & 7].x, m[u], acc[c]);
                acc[8 + c] = fmaf(g[(c - u + 8) & 7].y, m[u], acc[8 + c]);
            }
            if (LDSRD) g[(7 - u) & 7] = t[(base + u * 64) & 511];
        }
        base += 1;
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += acc[i];
    out[blockIdx.x * 64 + lane] = s;
    const long long c1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    if (lane == 0) {
        clk[2 * blockIdx.x] = c1 - c0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
}

int main() {
    const int maxw = 8, nsimd = 1024, iters = 4000;
    float *out;
    long long *clk;
    CHECK(hipMalloc(&out, sizeof(float) * 64 * nsimd * maxw));
    CHECK(hipMalloc(&clk, sizeof(long long) * 2 * nsimd * maxw));
    std::vector<long long> hc(2 * nsimd * maxw);
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    std::printf("lds_reads waves_per_simd ms TFLOP/s clock_GHz fma_lanes_per_clk_per_simd(of_32_at_peak)\n");
    for (int lds = 0; lds < 2; ++lds)
        for (int wps = 1; wps <= maxw; ++wps) {
            const int nb = nsimd * wps;
            float ms = 0.f;
            for (int rep = 0; rep < 3; ++rep) {
                CHECK(hipEventRecord(e0));
                if (lds)
                    hipLaunchKernelGGL(k_fma<1>, dim3(nb), dim3(64), 0, 0, out, clk, iters, 1.0f);
                else
                    hipLaunchKernelGGL(k_fma<0>, dim3(nb), dim3(64), 0, 0, out, clk, iters, 1.0f);
                CHECK(hipGetLastError());
                CHECK(hipEventRecord(e1));
                CHECK(hipEventSynchronize(e1));
                CHECK(hipEventElapsedTime(&ms, e0, e1));
            }
            CHECK(hipMemcpy(hc.data(), clk, sizeof(long long) * 2 * nb, hipMemcpyDeviceToHost));
            double cyc = 0.0, rt = 0.0;
            for (int b = 0; b < nb; ++b) {
                cyc += (double)hc[2 * b];
                rt += (double)hc[2 * b + 1];
            }
            const double ghz = cyc / rt * 0.1;  // s_memrealtime runs at 100 MHz
            const double fl = 2.0 * 128.0 * iters * 64.0 * nb;
            const double lanes = fl / 2.0 / (ms * 1e-3) / nsimd / (ghz * 1e9);
            std::printf("%d %d %.3f %.1f %.2f %.2f\n", lds, wps, ms, fl / ms / 1e9, ghz, lanes);
        }
    CHECK(hipFree(out));
    CHECK(hipFree(clk));
    return 0;
}
