// Log-sum-exp softmin for the cost C(x, y) = |x - y|^p / p with 1 <= p < 2
// (Section 2 states the method for a cost |x - y|^p / p; the contraction form
// of the p = 2 kernels does not exist for other p).
//
// Each thread owns one row.  Columns are staged in LDS (coordinates and the
// log2-domain offset u_j = log2(e) (log w_j + h_j / eps)) and read by every
// thread at the same address (broadcast).  Per pair:
//   D2 = sum_t (x_t - y_t)^2          (from coordinate differences: no
//                                       cancellation near D2 = 0)
//   C  = sqrt(D2) (p = 1), else 2^{(p/2) log2 D2} / p
//   s  = u_j - log2(e) C / eps
// and the row keeps (M, S) = (running maximum, sum of 2^{s - M}), refreshed
// once per group of 8 columns.  The record has the layout of the other
// softmin kernels, so the merge/averaging kernel is shared; the packed
// half-norms are zero for this cost, which removes the p = 2 expansion terms
// from the column offsets and the finish.
#include "skh_internal.h"

namespace skh {

static __device__ __forceinline__ float pc_ninf() { return -__builtin_huge_valf(); }
static __device__ __forceinline__ float pc_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
static __device__ __forceinline__ float pc_log2(float x) { return __builtin_amdgcn_logf(x); }

constexpr int kPcThreads = kRowsPerBlock;  // one row per thread

// P1: p = 1 (a square root per pair instead of a logarithm and an exponential)
template <int KP, bool P1>
__global__ __launch_bounds__(kPcThreads) void k_softmin_pcost(const SoftminBatch B) {
    constexpr int TC = KP <= 16 ? 256 : 16384 / (4 * KP);  // columns per LDS tile (16 KB max)
    constexpr int V4 = KP / 4;
    constexpr int G = 8;  // columns per running-maximum refresh
    __shared__ __attribute__((aligned(16))) float tile[TC * KP];
    __shared__ float tu[TC];

    const int wg = blockIdx.x;
    int q = 0;
#pragma unroll
    for (int t = 1; t < kMaxJobs; ++t)
        if (t < B.n_jobs && wg >= B.job[t].wg_begin) q = t;
    const SoftminJob &J = B.job[q];
    const float *__restrict__ rows = J.rows;
    const float *__restrict__ cols = J.cols;
    const float *__restrict__ u = J.u;
    float2 *__restrict__ part = J.part;
    const int n_rows = J.n_rows, n_cols = J.n_cols;
    const int local = wg - J.wg_begin;
    const int rt = local % J.row_tiles, chunk = local / J.row_tiles;
    const int c_begin = chunk * J.chunk_cols;
    const int c_end = min(n_cols, c_begin + J.chunk_cols);
    const float pexp = B.cost_p;
    const float kc = B.kscale / pexp;  // log2(e) / (p eps)
    const float half_p = 0.5f * pexp;

    const int tid = threadIdx.x;
    const int i = rt * kRowsPerBlock + tid;
    const int ic = i < n_rows ? i : n_rows - 1;
    float xr[KP];
    {
        const float4 *rp = reinterpret_cast<const float4 *>(rows + (size_t)ic * KP);
#pragma unroll
        for (int v = 0; v < V4; ++v) {
            const float4 t = rp[v];
            xr[4 * v] = t.x;
            xr[4 * v + 1] = t.y;
            xr[4 * v + 2] = t.z;
            xr[4 * v + 3] = t.w;
        }
    }

    float m = pc_ninf(), S = 0.0f;
    for (int j0 = c_begin; j0 < c_end; j0 += TC) {
        __syncthreads();
        const int nv = min(TC, c_end - j0);
        for (int e = tid; e < TC * V4; e += kPcThreads) {
            const int c = e / V4, v = e - c * V4;
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < nv) val = *reinterpret_cast<const float4 *>(cols + (size_t)(j0 + c) * KP + 4 * v);
            *reinterpret_cast<float4 *>(&tile[c * KP + 4 * v]) = val;
        }
        for (int c = tid; c < TC; c += kPcThreads) tu[c] = c < nv ? u[j0 + c] : pc_ninf();
        __syncthreads();
        const int ng = (nv + G - 1) / G;
        for (int gi = 0; gi < ng; ++gi) {
            float sv[G];
            float gmax = pc_ninf();
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int c = gi * G + k;  // < TC: TC is a multiple of G
                const float *yc = &tile[c * KP];
                float d2 = 0.0f;
#pragma unroll
                for (int t = 0; t < KP - 1; ++t) {  // slot KP - 1 is padding (KP >= d + 1)
                    const float df = xr[t] - yc[t];
                    d2 = fmaf(df, df, d2);
                }
                const float C = P1 ? __builtin_amdgcn_sqrtf(d2) : pc_exp2(half_p * pc_log2(d2));
                sv[k] = fmaf(-kc, C, tu[c]);
                gmax = fmaxf(gmax, sv[k]);
            }
            if (gmax > m) {
                S *= pc_exp2(m - gmax);  // 0 while m = -inf
                m = gmax;
            }
            const float base = m > pc_ninf() ? m : 0.0f;
            float sg = 0.0f;
#pragma unroll
            for (int k = 0; k < G; ++k) sg += pc_exp2(sv[k] - base);
            S += sg;
        }
    }
    if (i < n_rows) part[(size_t)chunk * n_rows + i] = make_float2(S > 0.0f ? m : pc_ninf(), S);
}

template <bool P1>
static hipError_t launch_pcost_kp(const SoftminBatch &b, int kp, dim3 grid, hipStream_t s) {
    const dim3 block(kPcThreads);
    switch (kp) {
    case 4: hipLaunchKernelGGL((k_softmin_pcost<4, P1>), grid, block, 0, s, b); break;
    case 8: hipLaunchKernelGGL((k_softmin_pcost<8, P1>), grid, block, 0, s, b); break;
    case 16: hipLaunchKernelGGL((k_softmin_pcost<16, P1>), grid, block, 0, s, b); break;
    case 32: hipLaunchKernelGGL((k_softmin_pcost<32, P1>), grid, block, 0, s, b); break;
    case 64: hipLaunchKernelGGL((k_softmin_pcost<64, P1>), grid, block, 0, s, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Weighted plan sums behind grad_x S for the cost |x - y|^p / p (dense FP32,
// one row per thread, columns in LDS as in k_softmin_pcost).  With
// pi_ij = a_i b_j exp((f_i + g_j - C_ij) / eps) and grad_x C = |x - y|^{p-2} (x - y),
// the record of row i over a column chunk is
//   [M_i, sum_j 2^{s_ij - M_i} w_ij, sum_j 2^{s_ij - M_i} w_ij y_j (d values)],
//   s_ij = u_j - log2(e) C_ij / eps,  w_ij = |x_i - y_j|^{p-2} (0 at distance 0),
// the layout of the plan records, so the plan merge gives sum_j pi_ij w_ij and
// sum_j pi_ij w_ij y_j and the gradient is (their first) x_i - (their second),
// as for p = 2 where w = 1.  A pair at distance 0 has a zero difference and
// contributes nothing (for p = 1 the zero subgradient).
template <int KP, bool P1>
__global__ __launch_bounds__(kPcThreads) void k_plan_pcost(const PlanBatch B, float pexp) {
    constexpr int TC = KP <= 16 ? 256 : 16384 / (4 * KP);
    constexpr int V4 = KP / 4;
    constexpr int G = 8;
    __shared__ __attribute__((aligned(16))) float tile[TC * KP];
    __shared__ float tu[TC];

    const int wg = blockIdx.x;
    int q = 0;
#pragma unroll
    for (int t = 1; t < kMaxJobs; ++t)
        if (t < B.n_jobs && wg >= B.job[t].wg_begin) q = t;
    const PlanJob &J = B.job[q];
    const float *__restrict__ rows = J.rows;
    const float *__restrict__ cols = J.cols;
    const float *__restrict__ u = J.u;
    float *__restrict__ part = J.part;
    const int n_rows = J.n_rows, n_cols = J.n_cols, L = J.L;
    const int local = wg - J.wg_begin;
    const int rt = local % J.row_tiles, chunk = local / J.row_tiles;
    const int c_begin = chunk * J.chunk_cols;
    const int c_end = min(n_cols, c_begin + J.chunk_cols);
    const float kc = B.kscale / pexp;  // log2(e) / (p eps)
    const float half_p = 0.5f * pexp;
    const float half_w = 0.5f * (pexp - 2.0f);  // w = (D2)^{(p-2)/2}

    const int tid = threadIdx.x;
    const int i = rt * kRowsPerBlock + tid;
    const int ic = i < n_rows ? i : n_rows - 1;
    float xr[KP];
    {
        const float4 *rp = reinterpret_cast<const float4 *>(rows + (size_t)ic * KP);
#pragma unroll
        for (int v = 0; v < V4; ++v) {
            const float4 t = rp[v];
            xr[4 * v] = t.x;
            xr[4 * v + 1] = t.y;
            xr[4 * v + 2] = t.z;
            xr[4 * v + 3] = t.w;
        }
    }

    float m = pc_ninf(), W = 0.0f;
    float acc[KP - 1];
#pragma unroll
    for (int t = 0; t < KP - 1; ++t) acc[t] = 0.0f;
    for (int j0 = c_begin; j0 < c_end; j0 += TC) {
        __syncthreads();
        const int nv = min(TC, c_end - j0);
        for (int e = tid; e < TC * V4; e += kPcThreads) {
            const int c = e / V4, v = e - c * V4;
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < nv) val = *reinterpret_cast<const float4 *>(cols + (size_t)(j0 + c) * KP + 4 * v);
            *reinterpret_cast<float4 *>(&tile[c * KP + 4 * v]) = val;
        }
        for (int c = tid; c < TC; c += kPcThreads) tu[c] = c < nv ? u[j0 + c] : pc_ninf();
        __syncthreads();
        const int ng = (nv + G - 1) / G;
        for (int gi = 0; gi < ng; ++gi) {
            float sv[G], wv[G];
            float gmax = pc_ninf();
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int c = gi * G + k;
                const float *yc = &tile[c * KP];
                float d2 = 0.0f;
#pragma unroll
                for (int t = 0; t < KP - 1; ++t) {
                    const float df = xr[t] - yc[t];
                    d2 = fmaf(df, df, d2);
                }
                const float C = P1 ? __builtin_amdgcn_sqrtf(d2) : pc_exp2(half_p * pc_log2(d2));
                sv[k] = fmaf(-kc, C, tu[c]);
                wv[k] = d2 > 0.0f ? (P1 ? __builtin_amdgcn_rsqf(d2) : pc_exp2(half_w * pc_log2(d2)))
                                  : 0.0f;
                gmax = fmaxf(gmax, sv[k]);
            }
            if (gmax > m) {
                const float r = pc_exp2(m - gmax);  // 0 while m = -inf
                W *= r;
#pragma unroll
                for (int t = 0; t < KP - 1; ++t) acc[t] *= r;
                m = gmax;
            }
            const float base = m > pc_ninf() ? m : 0.0f;
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int c = gi * G + k;
                const float e = pc_exp2(sv[k] - base) * wv[k];
                W += e;
#pragma unroll
                for (int t = 0; t < KP - 1; ++t) acc[t] = fmaf(e, tile[c * KP + t], acc[t]);
            }
        }
    }
    if (i < n_rows) {
        float *rec = part + ((size_t)chunk * n_rows + i) * (L + 2);
        rec[0] = W > 0.0f ? m : pc_ninf();
        rec[1] = W;
#pragma unroll
        for (int t = 0; t < KP - 1; ++t)
            if (t < L) rec[2 + t] = acc[t];
    }
}

template <bool P1>
static hipError_t launch_plan_pcost_kp(const PlanBatch &b, int kp, float pexp, dim3 grid,
                                       hipStream_t s) {
    const dim3 block(kPcThreads);
    switch (kp) {
    case 4: hipLaunchKernelGGL((k_plan_pcost<4, P1>), grid, block, 0, s, b, pexp); break;
    case 8: hipLaunchKernelGGL((k_plan_pcost<8, P1>), grid, block, 0, s, b, pexp); break;
    case 16: hipLaunchKernelGGL((k_plan_pcost<16, P1>), grid, block, 0, s, b, pexp); break;
    case 32: hipLaunchKernelGGL((k_plan_pcost<32, P1>), grid, block, 0, s, b, pexp); break;
    case 64: hipLaunchKernelGGL((k_plan_pcost<64, P1>), grid, block, 0, s, b, pexp); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_plan_pcost(const PlanBatch &b, int kp, float pexp, int total_wgs, hipStream_t s) {
    for (int q = 0; q < b.n_jobs; ++q)
        if (b.job[q].tiles || b.job[q].V || b.job[q].L >= kp) return hipErrorInvalidValue;
    const dim3 grid(total_wgs);
    return pexp == 1.0f ? launch_plan_pcost_kp<true>(b, kp, pexp, grid, s)
                        : launch_plan_pcost_kp<false>(b, kp, pexp, grid, s);
}

hipError_t launch_softmin_pcost(const SoftminBatch &b, int kp, int total_wgs, hipStream_t s) {
    const dim3 grid(total_wgs);
    return b.cost_p == 1.0f ? launch_pcost_kp<true>(b, kp, grid, s)
                            : launch_pcost_kp<false>(b, kp, grid, s);
}

}  // namespace skh
