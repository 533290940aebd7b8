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
// so the split error scales with the cluster radius |dy|, not with |y|.
// The shift re-reads the row k * x_i from memory at each cluster change (the
// register file holds only its bf16 split), which keeps the kernel at four
// workgroups per CU.
//
// Three more coordinates ride along in the contraction, so that the matrix
// cores deliver the exponent itself:
//   slots d, d+1, d+2 : the column offset u_j as three bf16 terms (hi, mid, lo:
//                       24 bits) against 1.0 in the row's hi plane;
//   slot KP-1         : 1.0 in the column's hi plane against w_i split over the
//                       row's hi and lo planes (16 bits), where w_i ~ shift_i - R_i
//                       moves the row's running reference R_i into the MFMA
//                       (shift_i = k <x_i, c_J>).
// The result is s_ij - R_i with R_i = shift_i - w_i known exactly, and each
// lane adds 2^{s_ij - R_i} for its 16 columns: one exp2 and one add per pair.
// Each problem has its own copy of the column hi plane whose slots d..d+2 are
// rewritten when its column potential changes (k_u_slots), so staging a tile
// is a plain copy, prefetched into registers one tile ahead.
// The reference changes only when the cluster changes (same level, re-rounded)
// or, for the whole wave at once, when a row's sum would leave [2^-4, 2^59)
// (first mass, overflow): then the larger of the block's maximum and the sum
// so far sets the new level and the block is re-summed from the accumulators.
// A row that holds mass keeps a sum >= 2^-4 (sums only grow; a cluster change
// re-rounds the level by far less), so once every row of a wave holds mass the
// overflow test runs only for blocks with a term above 2^40 (smaller terms cannot
// carry a sum to FP32 overflow over at most 2^23 blocks), and a block whose terms
// all lie below 2^T of the level (T = B.skip_log2: -48, lower for column sets
// beyond 2^20 points) is skipped
// after its products (it cannot move any row sum beyond rounding); the products
// of every pair are still computed.
//
// Padding and zero-weight columns use a finite sentinel (-1e30) rather than
// -inf so that the lo products stay finite (-inf * 0 would be NaN).
#include "skh_internal.h"

namespace skh {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kMasked = -1.0e30f;

static __device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
static __device__ __forceinline__ float xor32_sum(float v) {
    const unsigned u = __float_as_uint(v);
    const auto t = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}
static __device__ __forceinline__ float xor32_max(float v) {
    const unsigned u = __float_as_uint(v);
    const auto t = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return fmaxf(__uint_as_float(t[0]), __uint_as_float(t[1]));
}

// 64-column tiles and at most 128 registers per lane: four workgroups per CU.
template <int KP>
__global__ __launch_bounds__(256, 4) void k_softmin_bf16(const SoftminBatch B) {
    constexpr int TC = 64;  // columns staged per tile (a divisor of kColsPerTile)
    constexpr int H = KP / 2;        // dims per lane half
    constexpr int S = H / 8;         // k-steps of 16 (8 bf16 per lane)
    constexpr int RSB = KP * 2 + 16; // LDS row stride in bytes (padding against bank conflicts)
    constexpr int V16 = KP / 8;      // 16-byte chunks per packed column plane
    constexpr int NCH = (TC * V16 + 255) / 256;  // chunks per thread per plane and tile
    constexpr int NBT = TC / 32;                 // 32-column blocks per tile
    constexpr int NCE = NBT * KP;                  // centroid floats per tile
    constexpr int NCP = (NCE + 255) / 256;           // centroid floats per thread
    __shared__ __attribute__((aligned(16))) unsigned char lhi[TC * RSB];
    __shared__ __attribute__((aligned(16))) unsigned char llo[TC * RSB];
    __shared__ float lcent[NBT][KP];
    __shared__ __attribute__((aligned(8))) int lcl[NBT];

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
    const float *__restrict__ blk_cent = J.col_centroids;  // per 32-column block
    float2 *__restrict__ part = J.part;
    const int n_rows = J.n_rows, n_cols = J.n_cols;
    const int local = wg - J.wg_begin;
    const int d = B.d;
    const float kscale = B.kscale;

    // rows [rb, re) and the column ranges of this workgroup
    int rb, re, chunk, nranges, r0 = 0, rstep = 1;
    const int2 *rng = nullptr;
    int c_begin = 0, c_end = 0;
    if (J.tiles) {  // chunk c of a row tile takes its ranges c, c + n_chunks, ...
        const int4 t = J.tiles[local % J.n_tiles];
        rb = t.x;
        re = t.y;
        chunk = local / J.n_tiles;
        rng = J.ranges + (size_t)t.z * J.range_cap;
        nranges = J.range_count[t.z];
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

    // Row: k * x_i split into bf16 hi/lo in registers.  The FP32 row that the cluster
    // shift needs is read again from memory (L2) at each cluster change rather than held
    // in 32 more registers.
    const float *rowp = rows + (size_t)ic * KP + h * H;
    bf16x8 xh[S], xl[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const float4 v0 = *reinterpret_cast<const float4 *>(rowp + s * 8);
        const float4 v1 = *reinterpret_cast<const float4 *>(rowp + s * 8 + 4);
        const float xs[8] = {v0.x * kscale, v0.y * kscale, v0.z * kscale, v0.w * kscale,
                             v1.x * kscale, v1.y * kscale, v1.z * kscale, v1.w * kscale};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int dim = h * H + s * 8 + e;
            const float v = xs[e];
            const __bf16 hi = static_cast<__bf16>(v);
            const __bf16 lo = static_cast<__bf16>(v - static_cast<float>(hi));
            const bool aug = dim >= d && dim < d + 3;
            xh[s][e] = aug ? static_cast<__bf16>(1.0f) : hi;
            xl[s][e] = aug ? static_cast<__bf16>(0.0f) : lo;
        }
    }

    // running reference R (exact: R = shift - w) and the lane's sum relative to it
    float R = 0.0f, Sl = 0.0f, shift = 0.0f;
    int cur_cluster = -1;
    bool mass = false, all_mass = false;
    // w = w_hi + w_lo (16 significant bits) rides in slot KP-1 of both row planes;
    // returns the reference the contraction now subtracts
    auto set_ref = [&](float target) -> float {
        const __bf16 whi = static_cast<__bf16>(target);
        const __bf16 wlo = static_cast<__bf16>(target - static_cast<float>(whi));
        if (h == 1) {
            xh[S - 1][7] = whi;
            xl[S - 1][7] = wlo;
        }
        return shift - (static_cast<float>(whi) + static_cast<float>(wlo));
    };
    R = set_ref(0.0f);

    // Column tiles, walked range by range; the next tile is loaded into
    // registers while the current one is computed.  Range ends are multiples
    // of 32 (clusters are padded), so a 32-column block is either fully inside
    // the range or skipped.
    uint4 pfh[NCH], pfl[NCH];
    float pfc[NCP];
    int pfk = -1;
    auto next_tile = [&](int &r, int &a, int &e) -> bool {
        if (r >= 0 && a + TC < e) {
            a += TC;
            return true;
        }
        for (r = r < 0 ? r0 : r + rstep; r < nranges; r += rstep) {
            const int2 v = rng ? rng[r] : make_int2(c_begin, c_end);
            if (v.x < v.y) {
                a = v.x;
                e = v.y;
                return true;
            }
        }
        return false;
    };
    // Tile loads go through buffer descriptors based at the tile (scalar registers) with
    // 32-bit lane offsets; reads past the end of the column planes return zeros.  Columns
    // of a tile past its range end are staged but never used (ranges end on 32-column
    // blocks and only the blocks inside the range are computed).
    auto prefetch = [&](int a_, int e_) {
        const int a = __builtin_amdgcn_readfirstlane(a_);
        const int e = __builtin_amdgcn_readfirstlane(e_);
        const long long rem = (long long)(n_cols - a) * (KP * 2);
        const int nrec = rem > 0x7fffffff ? 0x7fffffff : (int)rem;
        const __amdgpu_buffer_rsrc_t rh = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<unsigned char *>(chi) + (size_t)a * (KP * 2), (short)0, nrec, 0x00020000);
        const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<unsigned char *>(clo) + (size_t)a * (KP * 2), (short)0, nrec, 0x00020000);
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const unsigned off = (unsigned)(tid + 256 * k) * 16u;
            if (TC * V16 % 256 == 0 || tid + 256 * k < TC * V16) {
                pfh[k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rh, off, 0, 0));
                pfl[k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rl, off, 0, 0));
            }
        }
        const int lim = e - a;
        const float *tc = blk_cent + (size_t)(a >> 5) * KP;
#pragma unroll
        for (int c = 0; c < NCP; ++c) {
            const int q = tid + 256 * c;
            pfc[c] = q < NCE && 32 * (q / KP) < lim ? tc[(unsigned)q] : 0.0f;
        }
        if (tid < NBT) pfk = 32 * tid < lim ? blk_cluster[(a >> 5) + tid] : -1;
    };

    int ri = -1, j0 = 0, jend = 0;
    bool have = next_tile(ri, j0, jend);
    if (have) prefetch(j0, jend);
    while (have) {
        __syncthreads();  // the previous tile is no longer read
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            const int idx = tid + 256 * k;
            const int c = idx / V16, v = idx - c * V16;
            if (TC * V16 % 256 != 0 && idx >= TC * V16) break;
            *reinterpret_cast<uint4 *>(lhi + c * RSB + v * 16) = pfh[k];
            *reinterpret_cast<uint4 *>(llo + c * RSB + v * 16) = pfl[k];
        }
#pragma unroll
        for (int c = 0; c < NCP; ++c) {
            const int q = tid + 256 * c;
            if (q < NCE) lcent[q / KP][q % KP] = pfc[c];
        }
        if (tid < NBT) lcl[tid] = pfk;
        const int cj0 = j0, cend = jend;
        const bool more = next_tile(ri, j0, jend);
        if (more) prefetch(j0, jend);
        __syncthreads();

        const int nblk = wave_active ? min(NBT, (cend - cj0 + 31) >> 5) : 0;
        static_assert(NBT == 2, "one int2 of cluster ids per tile");
        const int2 c2 = *reinterpret_cast<const int2 *>(lcl);
        const int cl0 = __builtin_amdgcn_readfirstlane(c2.x);
        const int cl1 = __builtin_amdgcn_readfirstlane(c2.y);
        for (int jb = 0; jb < nblk; ++jb) {
            const int cl = jb == 0 ? cl0 : cl1;
            if (cl != cur_cluster) {  // wave-uniform: new cluster shift, same reference level
                cur_cluster = cl;
                float r = 0.0f;
#pragma unroll
                for (int t = 0; t < H; t += 4) {
                    const float4 xv = *reinterpret_cast<const float4 *>(rowp + t);
                    r = fmaf(xv.x * kscale, lcent[jb][h * H + t], r);
                    r = fmaf(xv.y * kscale, lcent[jb][h * H + t + 1], r);
                    r = fmaf(xv.z * kscale, lcent[jb][h * H + t + 2], r);
                    r = fmaf(xv.w * kscale, lcent[jb][h * H + t + 3], r);
                }
                shift = xor32_sum(r);
                const float Rn = set_ref(shift - R);
                Sl = Sl > 0.0f ? Sl * fast_exp2(R - Rn) : 0.0f;
                R = Rn;
            }
            v16f acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                        0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const unsigned char *ph = lhi + (jb * 32 + li) * RSB + h * H * 2;
            const unsigned char *pl = llo + (jb * 32 + li) * RSB + h * H * 2;
            // operand reads one k-step ahead of the products; the scheduling fences keep
            // the compiler from hoisting every read of the block (register pressure)
            bf16x8 ah = *reinterpret_cast<const bf16x8 *>(ph);
            bf16x8 al = *reinterpret_cast<const bf16x8 *>(pl);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                bf16x8 nh = ah, nl = al;
                if (s + 1 < S) {
                    nh = *reinterpret_cast<const bf16x8 *>(ph + (s + 1) * 16);
                    nl = *reinterpret_cast<const bf16x8 *>(pl + (s + 1) * 16);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh[s], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh[s], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl[s], acc, 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                ah = nh;
                al = nl;
            }
            // acc[r] = s_ij - R.  Once every row of the wave holds mass (its sum is
            // >= 2^-4 relative to R), a block whose terms are all below 2^skip_log2
            // cannot change any row sum beyond FP32 rounding: its exponentials are
            // skipped (wave-uniform test on the block maximum).
            bool big = true;
            if (all_mass) {
                float mx = acc[0];
#pragma unroll
                for (int r = 1; r < 16; ++r) mx = fmaxf(mx, acc[r]);
                if (!__any(mx > B.skip_log2)) continue;
                // terms <= 2^40 cannot overflow a sum that holds mass (at most 2^23 blocks
                // per row add 2^44 each): the overflow test runs only for larger terms
                big = __any(mx > 40.0f);
            }
            // pairwise sum keeps the add chain short
            float ex[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) ex[r] = fast_exp2(acc[r]);
#pragma unroll
            for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
                for (int r = 0; r < w; ++r) ex[r] += ex[r + w];
            float Sn = Sl + ex[0];
            if (big && __any(!(Sn < 0x1p59f) || !mass)) {  // wave-uniform: look at whole rows
            const float Sc = xor32_sum(Sn);
            const bool need = !(Sc < 0x1p59f) || !(Sc >= 0x1p-4f);
            if (__any(need)) {  // wave-uniform: re-level the rows that need it
                float tmax = acc[0];
#pragma unroll
                for (int r = 1; r < 16; ++r) tmax = fmaxf(tmax, acc[r]);
                tmax = xor32_max(tmax);
                const float So = xor32_sum(Sl);
                const float lg = So > 0.0f ? __log2f(So) : -__builtin_huge_valf();
                const float top = fmaxf(tmax, lg);  // new level relative to R
                if (need && top > 0.5f * kMasked) {
                    const float Rn = set_ref(shift - (R + top));
                    const float dl = R - Rn;
                    float sb = 0.0f;
#pragma unroll
                    for (int r = 0; r < 16; ++r) sb += fast_exp2(acc[r] + dl);
                    Sn = (Sl > 0.0f ? Sl * fast_exp2(dl) : 0.0f) + sb;
                    R = Rn;
                }
            }
            mass = xor32_sum(Sn) >= 0x1p-4f;
            all_mass = !__any(!mass);
            }
            Sl = Sn;
        }
        have = more;
    }

    // both lane halves of a row share R: the row's partial is (R, sum of both halves)
    const float Sr = xor32_sum(Sl);
    const float M = Sr > 0.0f ? R : -__builtin_huge_valf();
    if (h == 0 && i < re) part[(size_t)chunk * n_rows + i] = make_float2(M, Sr);
}

// Column offsets u_j into slots d, d+1, d+2 of a packed hi plane, as three bf16
// terms (hi, mid, lo); non-finite or very negative offsets (no mass) become the
// finite sentinel.
__global__ __launch_bounds__(256) void k_u_slots(const float *__restrict__ u, int n, int kp, int d,
                                                 __hip_bfloat16 *__restrict__ hi) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float uu = u[i];
    if (!(uu > kMasked)) uu = kMasked;
    const __bf16 t1 = static_cast<__bf16>(uu);
    const float r1 = uu - static_cast<float>(t1);
    const __bf16 t2 = static_cast<__bf16>(r1);
    const float r2 = r1 - static_cast<float>(t2);
    const __bf16 t3 = static_cast<__bf16>(r2);
    __bf16 *row = reinterpret_cast<__bf16 *>(hi) + (size_t)i * kp;
    row[d] = t1;
    row[d + 1] = t2;
    row[d + 2] = t3;
}

hipError_t launch_u_slots(const float *u, int n, int kp, int d, __hip_bfloat16 *hi,
                          hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_u_slots, dim3((n + 255) / 256), dim3(256), 0, s, u, n, kp, d, hi);
    return hipGetLastError();
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
