// Log-sum-exp softmin with the contraction split into BF16 hi/lo products on
// the gfx950 matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation).
//
// Columns are stored in cluster order (K-means labels, clusters padded to 32),
// each as its offset dy_j = y_j - c_J from its cluster centre, split once into
// bf16 hi + lo.  Rows are the centred FP32 points x_i, scaled by k = log2(e)/eps
// and split in registers.  For the columns of cluster J:
//
//   k <x_i, y_j> = k <x_i, c_J>  +  k <x_i, dy_j>
//                  (FP32, once per    (three bf16 products: hi.hi + hi.lo + lo.hi,
//                   row and cluster)   FP32 accumulate, error ~ 3 * 2^-16 |x| |dy|)
//
// so the split error scales with the cluster radius |dy|, not with |y|; the
// cluster term is a per-row shift of the running maximum, applied once per
// cluster.  The column offset u_j (as in the FP32 kernel) is folded into the
// contraction as three bf16 terms (hi, mid, lo: 24 bits) in slots d, d+1,
// d+2, against 1.0 in the row's hi plane.  Padding and zero-weight columns use
// a finite sentinel (-1e30) rather than -inf so that the lo products stay
// finite (-inf * 0 would be NaN).
#include "skh_internal.h"

namespace skh {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kMasked = -1.0e30f;

static __device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

template <int KP>
__global__ __launch_bounds__(256) void k_softmin_bf16(const SoftminBatch B) {
    constexpr int H = KP / 2;       // dims per lane half
    constexpr int S = H / 8;        // k-steps of 16 (8 bf16 per lane)
    constexpr int RSB = KP * 2 + 16; // LDS row stride in bytes (padding against bank conflicts)
    constexpr int V16 = KP / 8;     // 16-byte chunks per packed column plane
    __shared__ __attribute__((aligned(16))) unsigned char lhi[kColsPerTile * RSB];
    __shared__ __attribute__((aligned(16))) unsigned char llo[kColsPerTile * RSB];
    __shared__ float lcent[kColsPerTile / 32][KP];
    __shared__ int lcl[kColsPerTile / 32];

    const int wg = blockIdx.x;
    int q = 0;
#pragma unroll
    for (int t = 1; t < kMaxJobs; ++t)
        if (t < B.n_jobs && wg >= B.job[t].wg_begin) q = t;
    const SoftminJob &J = B.job[q];
    const float *__restrict__ rows = J.rows;
    const unsigned char *__restrict__ chi = reinterpret_cast<const unsigned char *>(J.cols_hi);
    const unsigned char *__restrict__ clo = reinterpret_cast<const unsigned char *>(J.cols_lo);
    const int *__restrict__ blk_cluster = J.col_blk_cluster;
    const float *__restrict__ cent = J.col_centroids;
    const float *__restrict__ u = J.u;
    float2 *__restrict__ part = J.part;
    const int n_rows = J.n_rows, n_cols = J.n_cols;
    const int local = wg - J.wg_begin;
    const int d = B.d;
    const float kscale = B.kscale;

    // rows [rb, re) and the column ranges of this workgroup
    int rb, re, chunk, nranges;
    const int2 *rng = nullptr;
    int c_begin = 0, c_end = 0;
    if (J.tiles) {
        const int4 t = J.tiles[local];
        rb = t.x;
        re = t.y;
        chunk = 0;
        rng = J.ranges + (size_t)t.z * J.range_cap;
        nranges = J.range_count[t.z];
    } else {
        const int rt = local % J.row_tiles;
        chunk = local / J.row_tiles;
        rb = rt * kRowsPerBlock;
        re = min(n_rows, rb + kRowsPerBlock);
        c_begin = chunk * J.chunk_cols;
        c_end = min(n_cols, c_begin + J.chunk_cols);
        nranges = 1;
    }

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, li = lane & 31;
    const int i = rb + wave * 32 + li;
    const int ic = i < re ? i : re - 1;
    const bool wave_active = rb + wave * 32 < re;

    // Row: k * x_i in FP32 (for the cluster shift) and its bf16 hi/lo split.
    float xf[H];
    {
        const float *rp = rows + (size_t)ic * KP + h * H;
#pragma unroll
        for (int s = 0; s < H; s += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(rp + s);
            xf[s] = v.x * kscale;
            xf[s + 1] = v.y * kscale;
            xf[s + 2] = v.z * kscale;
            xf[s + 3] = v.w * kscale;
        }
    }
    bf16x8 xh[S], xl[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int dim = h * H + s * 8 + e;
            const float v = xf[s * 8 + e];
            const __bf16 hi = static_cast<__bf16>(v);
            const __bf16 lo = static_cast<__bf16>(v - static_cast<float>(hi));
            const bool aug = dim >= d && dim < d + 3;
            xh[s][e] = aug ? static_cast<__bf16>(1.0f) : hi;
            xl[s][e] = aug ? static_cast<__bf16>(0.0f) : lo;
        }
    }

    float m = -__builtin_huge_valf(), acc_sum = 0.0f, shift = 0.0f;
    int cur_cluster = -1;

    for (int ri = 0; ri < nranges; ++ri) {
    if (rng) {
        const int2 r = rng[ri];
        c_begin = r.x;
        c_end = r.y;
    }
    for (int j0 = c_begin; j0 < c_end; j0 += kColsPerTile) {
        __syncthreads();
        for (int e = tid; e < kColsPerTile * V16; e += 256) {
            const int c = e / V16, v = e - c * V16;
            const int j = j0 + c;
            uint4 vh = make_uint4(0u, 0u, 0u, 0u), vl = make_uint4(0u, 0u, 0u, 0u);
            if (j < c_end) {
                vh = *reinterpret_cast<const uint4 *>(chi + ((size_t)j * KP + v * 8) * 2);
                vl = *reinterpret_cast<const uint4 *>(clo + ((size_t)j * KP + v * 8) * 2);
            }
            *reinterpret_cast<uint4 *>(lhi + c * RSB + v * 16) = vh;
            *reinterpret_cast<uint4 *>(llo + c * RSB + v * 16) = vl;
        }
        if (tid < kColsPerTile / 32) {
            const int jb0 = j0 + 32 * tid;
            lcl[tid] = jb0 < c_end ? blk_cluster[jb0 >> 5] : -1;
        }
        __syncthreads();
        if (tid < kColsPerTile) {
            const int j = j0 + tid;
            float uu = j < c_end ? u[j] : kMasked;
            if (!(uu > kMasked)) uu = kMasked;
            const __bf16 t1 = static_cast<__bf16>(uu);
            const float r1 = uu - static_cast<float>(t1);
            const __bf16 t2 = static_cast<__bf16>(r1);
            const float r2 = r1 - static_cast<float>(t2);
            const __bf16 t3 = static_cast<__bf16>(r2);
            __bf16 *slot = reinterpret_cast<__bf16 *>(lhi + tid * RSB) + d;
            slot[0] = t1;
            slot[1] = t2;
            slot[2] = t3;
        }
        for (int e = tid; e < (kColsPerTile / 32) * KP; e += 256) {
            const int t = e / KP, dd = e - t * KP;
            const int cl = lcl[t];
            lcent[t][dd] = cl >= 0 ? cent[(size_t)cl * KP + dd] : 0.0f;
        }
        __syncthreads();
        const int nblk = wave_active ? min(kColsPerTile / 32, (c_end - j0 + 31) >> 5) : 0;
        for (int jb = 0; jb < nblk; ++jb) {
            const int cl = lcl[jb];
            if (cl != cur_cluster) {  // wave-uniform
                cur_cluster = cl;
                float r = 0.0f;
#pragma unroll
                for (int t = 0; t < H; ++t) r = fmaf(xf[t], lcent[jb][h * H + t], r);
                shift = r + __shfl_xor(r, 32, 64);
            }
            v16f acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                        0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const unsigned char *ph = lhi + (jb * 32 + li) * RSB + h * H * 2;
            const unsigned char *pl = llo + (jb * 32 + li) * RSB + h * H * 2;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(ph + s * 16);
                const bf16x8 al = *reinterpret_cast<const bf16x8 *>(pl + s * 16);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh[s], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh[s], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl[s], acc, 0, 0, 0);
            }
            float tmax = acc[0];
#pragma unroll
            for (int r = 1; r < 16; ++r) tmax = fmaxf(tmax, acc[r]);
            if (tmax > 0.5f * kMasked) {
                const float mn = fmaxf(m, tmax + shift);
                const float sub = mn - shift;
                float sblk = 0.0f;
#pragma unroll
                for (int r = 0; r < 16; ++r) sblk += fast_exp2(acc[r] - sub);
                acc_sum = acc_sum * fast_exp2(m - mn) + sblk;
                m = mn;
            }
        }
    }
    }

    const float m2 = __shfl_xor(m, 32, 64);
    const float s2 = __shfl_xor(acc_sum, 32, 64);
    const float M = fmaxf(m, m2);
    float Ssum = 0.0f;
    if (M > -__builtin_huge_valf()) Ssum = acc_sum * fast_exp2(m - M) + s2 * fast_exp2(m2 - M);
    if (h == 0 && i < re) part[(size_t)chunk * n_rows + i] = make_float2(M, Ssum);
}

hipError_t launch_softmin_bf16(const SoftminBatch &b, int kp, int total_wgs, hipStream_t s) {
    dim3 grid(total_wgs), block(256);
    switch (kp) {
    case 16: hipLaunchKernelGGL(k_softmin_bf16<16>, grid, block, 0, s, b); break;
    case 32: hipLaunchKernelGGL(k_softmin_bf16<32>, grid, block, 0, s, b); break;
    case 64: hipLaunchKernelGGL(k_softmin_bf16<64>, grid, block, 0, s, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace skh
