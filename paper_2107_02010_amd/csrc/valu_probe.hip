// Issue-rate probe of the vector ALU on the device the library runs on: the rate of
// plain FP32 adds and of v_exp_f32, alone and mixed, for the ALU-bound ceilings of
// the 3-D and p-cost softmin kernels.  Each thread runs 16 independent chains per
// iteration (e = 2^e, s = s + 1: no chain waits on another), every wave the same
// count; one float store per thread.  Prints one JSON line per occupancy.
#include <hip/hip_runtime.h>
#include <cstdio>

template <int NE, int NA>
__global__ __launch_bounds__(256) void k_valu_probe(float *out, int iters, float seed) {
    float e[16], s[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        e[r] = -1.0e30f * seed;  // 2^e: 0, 1, 2, 4, 16, 65536, inf, inf ... (no NaN)
        s[r] = seed * (float)(r + threadIdx.x);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (r < NE) e[r] = __builtin_amdgcn_exp2f(e[r]);
            if (r < NA) s[r] = s[r] + 1.0f;
        }
    }
    float t = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) t += e[r] + s[r];
    out[blockIdx.x * 256 + threadIdx.x] = t;
}

template <int NE, int NA>
static float time_ms(float *d, int grid, int iters) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0f;
    hipLaunchKernelGGL((k_valu_probe<NE, NA>), dim3(grid), dim3(256), 0, 0, d, iters, 1.0f);
    hipEventRecord(a);
    hipLaunchKernelGGL((k_valu_probe<NE, NA>), dim3(grid), dim3(256), 0, 0, d, iters, 1.0f);
    hipEventRecord(b);
    hipEventSynchronize(b);
    float ms = -1.0f;
    hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    return ms;
}

int main() {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 1;
    const int ncu = p.multiProcessorCount, iters = 4000;
    float *d = nullptr;
    if (hipMalloc(&d, (size_t)ncu * 8 * 256 * sizeof(float)) != hipSuccess) return 1;
    for (int wps = 2; wps <= 8; wps *= 2) {  // 256-thread workgroups per CU = waves per SIMD
        const int grid = ncu * wps;
        const float t_add = time_ms<0, 16>(d, grid, iters);
        const float t_exp = time_ms<16, 0>(d, grid, iters);
        const float t_both = time_ms<16, 16>(d, grid, iters);
        // lane operations per second over the chip: grid x 256 lanes x iters x 16 ops
        const double lanes = (double)grid * 256.0 * iters * 16.0;
        printf("{\"waves_per_simd\": %d, \"add_lane_ops_per_s\": %.4e, \"exp_lane_ops_per_s\": %.4e, "
               "\"exp_cost_in_adds\": %.3f, \"mixed_over_sum\": %.3f, \"ms\": [%.4f, %.4f, %.4f]}\n",
               wps, lanes / (t_add * 1e-3), lanes / (t_exp * 1e-3), t_exp / t_add,
               t_both / (t_exp + t_add), t_add, t_exp, t_both);
    }
    hipFree(d);
    return 0;
}
