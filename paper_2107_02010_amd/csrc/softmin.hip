// Tiled log-sum-exp softmin on MFMA for gfx950.
//
// For a row point x_i and column points y_j (both already centred, FP32) the
// softmin of the Algorithm's four updates is
//
//   -eps log sum_j w_j exp((h_j - C(x_i, y_j)) / eps),   C = |x - y|^2 / 2,
//
// and with C(x, y) = |x|^2/2 + |y|^2/2 - <x, y> it becomes
//
//   = |x_i|^2/2 - eps ln2 * log2 sum_j 2^{s_ij},
//   s_ij = k <x_i, y_j> + u_j,  k = log2(e)/eps,  u_j = log2(e) (log w_j + (h_j - |y_j|^2/2)/eps).
//
// The kernel computes L2_i = log2 sum_j 2^{s_ij} for a block of rows and a
// chunk of columns, with an online maximum so that nothing but the running
// (max, sum) pair per row is kept: O(n + m) memory (Section 2, the
// linear-memory remark on eqs. (3)-(4)).
//
// Contraction on the matrix cores: v_mfma_f32_32x32x2f32 computes a 32 x 32
// block D[j][i] += Y[j][k] X[k][i] with the column tile Y as operand A (read
// from LDS) and the row block X as operand B (held in VGPRs for the whole
// column sweep).  The column offset u_j rides along as one more coordinate:
// row slot d holds 1.0, column slot d holds u_j, so the MFMA result is s_ij
// itself.  Output lanes index rows (i = lane % 32) and the 16 accumulator
// registers index columns, so each lane sums its 16 values with no cross-lane
// traffic.
//
// Wide points (KP >= 16): the products dominate, and each lane keeps a running
// (max, sum) per block; the two lane halves of a row merge once at the end.
// Narrow points (KP <= 8, e.g. 3-D clouds): the exponentials and sums dominate,
// so the per-block maximum is dropped.  The sum is kept relative to a reference
// level R_i shared by the two lane halves of row i, and -R_i enters the
// contraction as the accumulator input of the first product: the MFMA delivers
// s_ij - R_i, one exponential and one add per pair.  R_i moves, for the rows
// that need it, only when a row's sum would leave [2^-4, 2^59) (first mass,
// overflow): the new level is the larger of the block's maximum and the sum so
// far, and the block is re-summed from the accumulators.  Once every row of a
// wave holds mass, a block whose terms all lie below 2^T of the level is
// skipped after its products, T = min(-48, -28 - ceil(log2 m)) for m columns:
// with the row sum >= 2^-4 of the level, all m columns of such terms move it by
// less than FP32 rounding.
//
// Zero weights and the ragged column tail both enter as u_j = -inf, which the
// contraction turns into s_ij = -inf and the exponential into 0.
#include <algorithm>

#include "skh_internal.h"

namespace skh {

typedef float v16f __attribute__((ext_vector_type(16)));

static __device__ __forceinline__ float ninf() { return -__builtin_huge_valf(); }

static __device__ __forceinline__ float fast_exp2(float x) {
    return __builtin_amdgcn_exp2f(x);  // v_exp_f32; inputs below -126 flush toward 0
}
// sum / maximum of a value over the two lane halves that hold the same row
static __device__ __forceinline__ float row_sum(float v) {
    const unsigned w = __float_as_uint(v);
    const auto t = __builtin_amdgcn_permlane32_swap(w, w, false, false);
    return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}
static __device__ __forceinline__ float row_max(float v) {
    const unsigned w = __float_as_uint(v);
    const auto t = __builtin_amdgcn_permlane32_swap(w, w, false, false);
    return fmaxf(__uint_as_float(t[0]), __uint_as_float(t[1]));
}

template <int KP>
__global__ __launch_bounds__(256) void k_softmin_f32(const SoftminBatch B) {
    constexpr int H = KP / 2;      // k-steps per 32x32 block; lane half h holds dims [h*H, h*H+H)
    constexpr int STRIDE = KP + 4; // LDS row stride (floats)
    constexpr int V4 = KP / 4;     // float4 per packed point
    // columns per LDS tile: 64 for wide points (17 KB instead of 35 KB of LDS, so the
    // CU holds more than four workgroups), 128 otherwise
    constexpr int TC = KP >= 32 ? 64 : kColsPerTile;
    __shared__ __attribute__((aligned(16))) float tile[TC * STRIDE];

    const int wg = blockIdx.x;
    int q = 0;
#pragma unroll
    for (int t = 1; t < kMaxJobs; ++t)
        if (t < B.n_jobs && wg >= B.job[t].wg_begin) q = t;
    const SoftminJob &J = B.job[q];
    const float *__restrict__ rows = J.rows;  // FP32 packed
    const float *__restrict__ cols = J.cols;
    const float *__restrict__ u = J.u;
    float2 *__restrict__ part = J.part;
    const int n_rows = J.n_rows, n_cols = J.n_cols;
    const int local = wg - J.wg_begin;
    const int d = B.d;
    const float kscale = B.kscale;

    // rows [rb, re) and the column ranges of this workgroup
    int rb, re, chunk, nranges, cl_row = 0, r0 = 0, rstep = 1;
    const int2 *rng = nullptr;
    int c_begin = 0, c_end = 0;
    if (J.tiles) {  // chunk c of a row tile takes its ranges c, c + n_chunks, ...
        const int4 t = J.tiles[local % J.n_tiles];
        rb = t.x;
        re = t.y;
        cl_row = t.z;
        chunk = local / J.n_tiles;
        rng = J.ranges + (size_t)cl_row * J.range_cap;
        nranges = J.range_count[cl_row];
        r0 = chunk;
        rstep = J.n_chunks;
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

    // Row operand: x_i scaled by k, slot d = 1.
    float xr[H];
    {
        const float *rp = rows + (size_t)ic * KP + h * H;
        if constexpr (H % 4 == 0) {
#pragma unroll
            for (int s = 0; s < H; s += 4) {
                float4 v = *reinterpret_cast<const float4 *>(rp + s);
                xr[s] = v.x;
                xr[s + 1] = v.y;
                xr[s + 2] = v.z;
                xr[s + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int s = 0; s < H; ++s) xr[s] = rp[s];
        }
#pragma unroll
        for (int s = 0; s < H; ++s) xr[s] = (h * H + s == d) ? 1.0f : xr[s] * kscale;
    }

    constexpr bool kLevel = KP <= 8;  // reference-level form for narrow points
    // online maximum form: running (max, sum) per lane
    float m = ninf(), acc_sum = 0.0f;
    // reference-level form: level R (row-uniform) and this lane's sum relative to it
    float R = 0.0f, Sl = 0.0f;
    bool mass = false, all_mass = false;
    v16f base;  // -R in every register: the accumulator input of the first product
#pragma unroll
    for (int r = 0; r < 16; ++r) base[r] = kLevel ? -R : 0.0f;

    for (int ri = r0; ri < nranges; ri += rstep) {
    if (rng) {
        const int2 r = rng[ri];
        c_begin = r.x;
        c_end = r.y;
    }
    for (int j0 = c_begin; j0 < c_end; j0 += TC) {
        __syncthreads();
        for (int e = tid; e < TC * V4; e += 256) {
            const int c = e / V4, v = e - c * V4;
            const int j = j0 + c;
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < c_end) val = *reinterpret_cast<const float4 *>(cols + (size_t)j * KP + v * 4);
            if (v == (d >> 2)) {
                const float uu = j < c_end ? u[j] : ninf();
                const int r = d & 3;
                val.x = r == 0 ? uu : val.x;
                val.y = r == 1 ? uu : val.y;
                val.z = r == 2 ? uu : val.z;
                val.w = r == 3 ? uu : val.w;
            }
            *reinterpret_cast<float4 *>(&tile[c * STRIDE + v * 4]) = val;
        }
        __syncthreads();
        const int nvalid = c_end - j0;
        const int nblk = wave_active ? min(TC / 32, (nvalid + 31) >> 5) : 0;
        for (int jb = 0; jb < nblk; ++jb) {
            const float *tp = &tile[(jb * 32 + li) * STRIDE + h * H];
            v16f acc = __builtin_amdgcn_mfma_f32_32x32x2f32(tp[0], xr[0], base, 0, 0, 0);
#pragma unroll
            for (int s = 1; s < H; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(tp[s], xr[s], acc, 0, 0, 0);
            if constexpr (!kLevel) {  // acc[r] = s_ij
                float tmax = acc[0];
#pragma unroll
                for (int r = 1; r < 16; ++r) tmax = fmaxf(tmax, acc[r]);
                const float mn = fmaxf(m, tmax);
                if (mn > ninf()) {
                    float sblk = 0.0f;
#pragma unroll
                    for (int r = 0; r < 16; ++r) sblk += fast_exp2(acc[r] - mn);
                    acc_sum = acc_sum * fast_exp2(m - mn) + sblk;
                    m = mn;
                }
                continue;
            }
            // acc[r] = s_ij - R
            if (all_mass) {  // wave-uniform skip of a negligible block
                float mx = acc[0];
#pragma unroll
                for (int r = 1; r < 16; ++r) mx = fmaxf(mx, acc[r]);
                if (!__any(mx > B.skip_log2)) continue;
            }
            float ex[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) ex[r] = fast_exp2(acc[r]);
#pragma unroll
            for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
                for (int r = 0; r < w; ++r) ex[r] += ex[r + w];
            float Sn = Sl + ex[0];
            if (__any(!(Sn < 0x1p59f) || !mass)) {  // wave-uniform: look at whole rows
                const float Sc = row_sum(Sn);
                const bool need = !(Sc < 0x1p59f) || !(Sc >= 0x1p-4f);
                if (__any(need)) {  // wave-uniform: re-level the rows that need it
                    float tmax = acc[0];
#pragma unroll
                    for (int r = 1; r < 16; ++r) tmax = fmaxf(tmax, acc[r]);
                    tmax = row_max(tmax);
                    const float So = row_sum(Sl);
                    const float lg = So > 0.0f ? __log2f(So) : ninf();
                    const float top = fmaxf(tmax, lg);  // new level relative to R
                    if (need && top > ninf()) {
                        const float Rn = R + top;
                        const float dl = R - Rn;
                        float sb = 0.0f;
#pragma unroll
                        for (int r = 0; r < 16; ++r) sb += fast_exp2(acc[r] + dl);
                        Sn = (Sl > 0.0f ? Sl * fast_exp2(dl) : 0.0f) + sb;
                        R = Rn;
#pragma unroll
                        for (int r = 0; r < 16; ++r) base[r] = -R;
                    }
                }
                mass = row_sum(Sn) >= 0x1p-4f;
                all_mass = !__any(!mass);
            }
            Sl = Sn;
        }
    }
    }

    if constexpr (kLevel) {
        // both lane halves of a row share R: the row's partial is (R, sum of both halves)
        const float Sr = row_sum(Sl);
        const float M = Sr > 0.0f ? R : ninf();
        if (h == 0 && i < re) part[(size_t)chunk * n_rows + i] = make_float2(M, Sr);
    } else {
        // merge the two lane halves that hold the same row
        const float m2 = __shfl_xor(m, 32, 64);
        const float s2 = __shfl_xor(acc_sum, 32, 64);
        const float M = fmaxf(m, m2);
        float S = 0.0f;
        if (M > ninf()) S = acc_sum * fast_exp2(m - M) + s2 * fast_exp2(m2 - M);
        if (h == 0 && i < re) part[(size_t)chunk * n_rows + i] = make_float2(M, S);
    }
}

// log2 bound of a skippable term for column sets of at most m points (see skip_log2)
static float skip_threshold(int64_t m) {
    int lg = 0;
    while (lg < 62 && (int64_t(1) << lg) < m) ++lg;  // ceil(log2 m)
    return (float)std::min(-48, -28 - lg);
}

int plan_softmin_batch(SoftminBatch &b, int target_wgs) {
    int max_cols = 1;
    for (int q = 0; q < b.n_jobs; ++q) max_cols = std::max(max_cols, b.job[q].n_cols);
    b.skip_log2 = skip_threshold(max_cols);
    int row_tiles_total = 0;
    for (int q = 0; q < b.n_jobs; ++q) {
        SoftminJob &J = b.job[q];
        J.row_tiles = (J.n_rows + kRowsPerBlock - 1) / kRowsPerBlock;
        row_tiles_total += J.row_tiles;
    }
    int want_chunks = row_tiles_total > 0 ? (target_wgs + row_tiles_total - 1) / row_tiles_total : 1;
    if (want_chunks < 1) want_chunks = 1;
    // block-sparse jobs: split each row tile's column ranges over up to four workgroups
    // when the row tiles alone give few rounds of resident workgroups
    int tiles_total = 0;
    for (int q = 0; q < b.n_jobs; ++q)
        if (b.job[q].tiles) tiles_total += b.job[q].n_tiles;
    int tile_chunks = tiles_total > 0 ? (target_wgs + tiles_total - 1) / tiles_total : 1;
    tile_chunks = tile_chunks < 1 ? 1 : (tile_chunks > 4 ? 4 : tile_chunks);
    int total = 0;
    for (int q = 0; q < b.n_jobs; ++q) {
        SoftminJob &J = b.job[q];
        if (J.tiles) {  // block-sparse: workgroups per row tile = chunks of its range list
            J.chunk_cols = 0;
            J.n_chunks = J.range_cap > 1 ? tile_chunks : 1;
            J.wg_begin = total;
            total += J.n_tiles * J.n_chunks;
            continue;
        }
        int tiles = (J.n_cols + kColsPerTile - 1) / kColsPerTile;
        int tiles_per_chunk = (tiles + want_chunks - 1) / want_chunks;
        if (tiles_per_chunk < 1) tiles_per_chunk = 1;
        J.chunk_cols = tiles_per_chunk * kColsPerTile;
        J.n_chunks = (J.n_cols + J.chunk_cols - 1) / J.chunk_cols;
        if (J.n_chunks < 1) J.n_chunks = 1;
        J.wg_begin = total;
        total += J.row_tiles * J.n_chunks;
    }
    return total;
}

hipError_t launch_softmin(const SoftminBatch &b, int kp, int precision, int total_wgs,
                          hipStream_t s) {
    (void)precision;
    if (b.cost_p != 0.0f && b.cost_p != 2.0f) return launch_softmin_pcost(b, kp, total_wgs, s);
    dim3 grid(total_wgs), block(256);
    switch (kp) {
    case 4: hipLaunchKernelGGL(k_softmin_f32<4>, grid, block, 0, s, b); break;
    case 8: hipLaunchKernelGGL(k_softmin_f32<8>, grid, block, 0, s, b); break;
    case 16: hipLaunchKernelGGL(k_softmin_f32<16>, grid, block, 0, s, b); break;
    case 32: hipLaunchKernelGGL(k_softmin_f32<32>, grid, block, 0, s, b); break;
    case 64: hipLaunchKernelGGL(k_softmin_f32<64>, grid, block, 0, s, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int packed_width(int d) {
    int kp = 4;
    while (kp < d + 1) kp *= 2;
    return kp;
}

int packed_width_bf16(int d) {
    int kp = 16;
    while (kp < d + 4) kp *= 2;
    return kp <= 64 ? kp : 0;
}

}  // namespace skh
