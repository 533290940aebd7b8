// K-means coarse scale and the cluster-sorted layout (Section 2, coarse-to-fine
// strategy: the coarse measures are K-means clusterings of the two clouds).
//
// Lloyd iterations on the device:
//   assign   label_i = argmin_c |c|^2/2 - <x_i, c>     (ties -> lowest c)
//   sort     stable counting sort by label (per-block counts, one exclusive
//            scan over label-major counts, in-block ranks) -> permutation
//   update   c = alpha-weighted mean of its members, summed in FP64 in a fixed
//            order over the sorted members; an empty cluster keeps its centre
// Every step is deterministic (integer LDS atomics only count).
//
// The padded layout places every cluster at a multiple of 32 points so that a
// 32-column MFMA block never spans two clusters; padding points carry zero
// weight (log-weight -inf).
#include "skh_internal.h"

namespace skh {

constexpr int kT = 256;

typedef float v16f __attribute__((ext_vector_type(16)));

// Nearest centre of every point, ties to the lowest centre index.  The
// distance is ranked by 1/2 |c|^2 - <x, c> (the |x|^2 term is common to a row),
// computed on the matrix cores like the softmin's contraction: each wave keeps
// 32 rows as the B operand of v_mfma_f32_32x32x2f32 in VGPRs, with the unused
// last slot set to 1; tiles of centres (64 for wide points, 128 otherwise) are
// staged in LDS as -c with 1/2 |c|^2 in that slot, so the MFMA output is the
// ranking value itself.
// Each lane keeps the running minimum of its 16 centres per block; the two
// lane halves of a row combine once at the end.  Rows padded to KP have their
// slots past the coordinates at zero, so slot KP - 1 is free.
template <int KP>
__global__ __launch_bounds__(256) void k_kmeans_assign(const float *__restrict__ X, int n,
                                                       const float *__restrict__ C, int k,
                                                       int *__restrict__ label) {
    constexpr int H = KP / 2;       // k-steps per block; lane half h holds slots [h H, h H + H)
    constexpr int STRIDE = KP + 4;  // LDS row stride (floats)
    // centres per tile: 64 for wide points (17 KB of LDS, six workgroups per CU), else 128
    constexpr int TCN = KP >= 32 ? 64 : 128;
    __shared__ float tile[TCN * STRIDE];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, li = lane & 31;
    const int i = blockIdx.x * 128 + wave * 32 + li;
    const int ic = i < n ? i : n - 1;
    float xr[H];
#pragma unroll
    for (int s = 0; s < H; ++s) {
        const int slot = h * H + s;
        xr[s] = slot == KP - 1 ? 1.0f : X[(size_t)ic * KP + slot];
    }
    float best = __builtin_huge_valf();
    int bj = 0x7fffffff;
    for (int c0 = 0; c0 < k; c0 += TCN) {
        __syncthreads();
        for (int e = tid; e < TCN * KP; e += 256) {
            const int c = e / KP, dd = e - c * KP;
            tile[c * STRIDE + dd] = c0 + c < k ? -C[(size_t)(c0 + c) * KP + dd] : 0.0f;
        }
        __syncthreads();
        if (tid < TCN) {
            float sq = 0.0f;
#pragma unroll
            for (int dd = 0; dd < KP - 1; ++dd) sq = fmaf(tile[tid * STRIDE + dd], tile[tid * STRIDE + dd], sq);
            // a missing centre gets a value no real one can exceed
            tile[tid * STRIDE + KP - 1] = c0 + tid < k ? 0.5f * sq : 1.0e30f;
        }
        __syncthreads();
        const int nblk = min(TCN / 32, (k - c0 + 31) >> 5);
        for (int jb = 0; jb < nblk; ++jb) {
            v16f acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const float *tp = &tile[(jb * 32 + li) * STRIDE + h * H];
#pragma unroll
            for (int s = 0; s < H; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(tp[s], xr[s], acc, 0, 0, 0);
            // output register r of lane half h holds centre 8 (r / 4) + 4 h + r % 4 of the
            // block: increasing in r, so a strict comparison keeps the lowest index
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if (acc[r] < best) {
                    best = acc[r];
                    bj = c0 + jb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                }
            }
        }
    }
    const float ob = __shfl_xor(best, 32, 64);
    const int oj = __shfl_xor(bj, 32, 64);
    if (ob < best || (ob == best && oj < bj)) bj = oj;
    if (h == 0 && i < n) label[i] = bj;
}

// counts[c * nb + b] = number of points of block b (kT points) with label c.
__global__ __launch_bounds__(kT) void k_label_count(const int *__restrict__ label, int n, int k,
                                                    int nb, int *__restrict__ counts) {
    extern __shared__ int hist[];
    for (int c = threadIdx.x; c < k; c += kT) hist[c] = 0;
    __syncthreads();
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i < n) atomicAdd(&hist[label[i]], 1);
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += kT) counts[(size_t)c * nb + blockIdx.x] = hist[c];
}

// Stable scatter: position = offs[label * nb + block] + rank among earlier
// points of the block with the same label.
__global__ __launch_bounds__(kT) void k_label_scatter(const int *__restrict__ label, int n, int nb,
                                                      const int *__restrict__ offs,
                                                      int *__restrict__ perm,
                                                      int *__restrict__ sorted_label) {
    __shared__ int sl[kT];
    const int i = blockIdx.x * kT + threadIdx.x;
    const int lab = i < n ? label[i] : -1;
    sl[threadIdx.x] = lab;
    __syncthreads();
    if (i < n) {
        int r = 0;
        for (int t = 0; t < (int)threadIdx.x; ++t) r += (sl[t] == lab);
        const int pos = offs[(size_t)lab * nb + blockIdx.x] + r;
        perm[pos] = i;
        sorted_label[pos] = lab;
    }
}

// Exclusive scan of int arrays: three phases over blocks of 1024 elements.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kT) void k_scan_block_sums(const int *__restrict__ in, int64_t len,
                                                        int *__restrict__ sums) {
    __shared__ int sh[kT];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    int s = 0;
    for (int e = threadIdx.x; e < kScanBlock; e += kT)
        if (base + e < len) s += in[base + e];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kT / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = sh[0];
}

// One block: exclusive scan of nsum block sums in place; total in sums[nsum].
__global__ __launch_bounds__(kT) void k_scan_sums(int *sums, int nsum) {
    __shared__ int sh[kT];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nsum; b0 += kT) {
        const int idx = b0 + threadIdx.x;
        const int v = idx < nsum ? sums[idx] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kT; o <<= 1) {  // inclusive Hillis-Steele
            const int t = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (idx < nsum) sums[idx] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kT - 1) carry += sh[kT - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nsum] = carry;
}

__global__ __launch_bounds__(kT) void k_scan_apply(const int *__restrict__ in, int64_t len,
                                                   const int *__restrict__ sums,
                                                   int *__restrict__ out) {
    __shared__ int sh[kT];
    __shared__ int carry;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    if (threadIdx.x == 0) carry = sums[blockIdx.x];
    __syncthreads();
    for (int e0 = 0; e0 < kScanBlock; e0 += kT) {
        const int64_t idx = base + e0 + threadIdx.x;
        const int v = idx < len ? in[idx] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kT; o <<= 1) {
            const int t = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (idx < len) out[idx] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kT - 1) carry += sh[kT - 1];
        __syncthreads();
    }
}

int scan_sums_len(int64_t len) { return (int)((len + kScanBlock - 1) / kScanBlock) + 1; }

hipError_t launch_exclusive_scan(const int *in, int64_t len, int *sums, int *out, hipStream_t s) {
    const int nblk = (int)((len + kScanBlock - 1) / kScanBlock);
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_block_sums, dim3(nblk), dim3(kT), 0, s, in, len, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kT), 0, s, sums, nblk);
    hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(kT), 0, s, in, len, sums, out);
    return hipGetLastError();
}

// One block per cluster: alpha-weighted mean of the members (sorted range
// [off[c], off[c+1]) of perm), FP64 accumulation in a fixed order.  Members with
// zero weight do not move the centre; a cluster with no mass keeps its centre.
// Also writes the cluster mass (FP32 of the FP64 sum).
constexpr int kCU = 1024;  // threads of the centroid update: 16 waves walk one cluster

template <int KP>
__global__ __launch_bounds__(kCU) void k_centroid_update(const float *__restrict__ X,
                                                         const float *__restrict__ w,
                                                         const int *__restrict__ perm,
                                                         const int *__restrict__ off,
                                                         float *__restrict__ C,
                                                         float *__restrict__ cmass) {
    constexpr int NW = kCU / 64;
    __shared__ double sh[NW][KP];
    __shared__ double shm[NW];
    const int c = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int beg = off[c], end = off[c + 1];
    double acc = 0.0, m = 0.0;
    for (int p = beg + wave; p < end; p += NW) {
        const int i = perm[p];
        const double wi = w ? (double)w[i] : 1.0;
        if (lane < KP) acc += wi * (double)X[(size_t)i * KP + lane];
        m += wi;
    }
    if (lane < KP) sh[wave][lane] = acc;
    if (lane == 0) shm[wave] = m;
    __syncthreads();
    if (threadIdx.x < KP) {  // the waves' partial sums in a fixed order
        const int d = threadIdx.x;
        double mass = 0.0, sum = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            mass += shm[q];
            sum += sh[q][d];
        }
        if (mass > 0.0) C[(size_t)c * KP + d] = (float)(sum / mass);
        if (d == 0 && cmass) cmass[c] = (float)mass;
    }
}

// Radius of each cluster: max distance of a member to its centre.
template <int KP>
__global__ __launch_bounds__(kT) void k_cluster_radius(const float *__restrict__ X,
                                                       const int *__restrict__ perm,
                                                       const int *__restrict__ off,
                                                       const float *__restrict__ C,
                                                       float *__restrict__ radius) {
    __shared__ float sh[kT];
    const int c = blockIdx.x;
    float r2 = 0.0f;
    for (int p = off[c] + threadIdx.x; p < off[c + 1]; p += kT) {
        const int i = perm[p];
        float s = 0.0f;
#pragma unroll
        for (int d = 0; d < KP; ++d) {
            const float t = X[(size_t)i * KP + d] - C[(size_t)c * KP + d];
            s = fmaf(t, t, s);
        }
        r2 = fmaxf(r2, s);
    }
    sh[threadIdx.x] = r2;
    __syncthreads();
    for (int o = kT / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) radius[c] = sqrtf(sh[0]);
}

__global__ __launch_bounds__(kT) void k_init_centroids(const float *__restrict__ X, int n, int k,
                                                       int kp, float *__restrict__ C) {
    const int e = blockIdx.x * kT + threadIdx.x;
    if (e >= k * kp) return;
    const int c = e / kp, d = e % kp;
    const int64_t src = (int64_t)c * n / k;  // evenly strided distinct points
    C[e] = X[src * kp + d];
}

// Cluster offsets from the scanned label-major counts: off[c] = offs[c * nb].
__global__ __launch_bounds__(kT) void k_cluster_offsets(const int *__restrict__ offs, int k, int nb,
                                                        int n, int *__restrict__ off) {
    const int c = blockIdx.x * kT + threadIdx.x;
    if (c < k) off[c] = offs[(size_t)c * nb];
    if (c == k) off[k] = n;
}

// Padded sizes (multiple of 32) of each cluster.
__global__ __launch_bounds__(kT) void k_padded_sizes(const int *__restrict__ off, int k,
                                                     int *__restrict__ psize) {
    const int c = blockIdx.x * kT + threadIdx.x;
    if (c == k) psize[k] = 0;  // the scan below runs over k + 1 entries
    if (c >= k) return;
    const int s = off[c + 1] - off[c];
    psize[c] = (s + 31) & ~31;
}

// perm_pad[poff[c] + r] = perm[off[c] + r] for r < size, -1 on the padding;
// blk_cluster[(poff[c] + 32 t) / 32] = c.
__global__ __launch_bounds__(kT) void k_padded_layout(const int *__restrict__ perm,
                                                      const int *__restrict__ off,
                                                      const int *__restrict__ poff, int k,
                                                      int *__restrict__ perm_pad,
                                                      int *__restrict__ blk_cluster) {
    const int c = blockIdx.x;
    if (c >= k) return;
    const int beg = off[c], size = off[c + 1] - beg;
    const int pbeg = poff[c], psize = poff[c + 1] - pbeg;
    for (int r = threadIdx.x; r < psize; r += kT) perm_pad[pbeg + r] = r < size ? perm[beg + r] : -1;
    for (int t = threadIdx.x; t < psize / 32; t += kT) blk_cluster[pbeg / 32 + t] = c;
}

// Gathers one cloud into the padded cluster order.
//   Xf  : n_pad x KP FP32, centred coordinates (row operand and norms)
//   Yhi0/Yhi1/Ylo : n_pad x KP bf16, hi/lo split of x - c_{cluster} (column
//         operand); the two hi copies belong to the two problems that read the
//         cloud as columns and carry 1.0 in slot KP-1 (their offset slots are
//         filled per iteration)
//   hn, lw, wp : half squared norms, log weights (-inf on padding), weights (0 on padding)
template <int KP>
__global__ __launch_bounds__(kT) void k_pack_padded(
    const float *__restrict__ X, const float *__restrict__ w, const int *__restrict__ perm_pad,
    const int *__restrict__ blk_cluster, const float *__restrict__ C, int n_pad,
    float *__restrict__ Xf, __hip_bfloat16 *__restrict__ Yhi0, __hip_bfloat16 *__restrict__ Yhi1,
    __hip_bfloat16 *__restrict__ Ylo, float *__restrict__ hn, float *__restrict__ lw,
    float *__restrict__ wp) {
    // KP / 4 consecutive lanes share a point (4 coordinates each), so every load and
    // store of a wave covers whole contiguous rows
    constexpr int G = KP / 4;
    constexpr int PPB = kT / G;  // points per block
    const int t = threadIdx.x % G;
    const int p = blockIdx.x * PPB + threadIdx.x / G;
    const bool live = p < n_pad;
    const int pc = live ? p : n_pad - 1;  // every lane takes part in the reduction
    const int i = perm_pad[pc];
    const int c = blk_cluster[pc >> 5];
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i >= 0) v = *reinterpret_cast<const float4 *>(X + (size_t)i * KP + 4 * t);
    const float4 cc = *reinterpret_cast<const float4 *>(C + (size_t)c * KP + 4 * t);
    const float vv[4] = {v.x, v.y, v.z, v.w}, cv[4] = {cc.x, cc.y, cc.z, cc.w};
    __hip_bfloat16 hi[4], lo[4];
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        s += (double)vv[e] * (double)vv[e];
        const float dv = i >= 0 ? vv[e] - cv[e] : 0.0f;
        hi[e] = __float2bfloat16(dv);
        lo[e] = __float2bfloat16(dv - __bfloat162float(hi[e]));
        if (4 * t + e == KP - 1) hi[e] = __float2bfloat16(1.0f);
    }
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (!live) return;
    *reinterpret_cast<float4 *>(Xf + (size_t)p * KP + 4 * t) = v;
    *reinterpret_cast<uint2 *>(Yhi0 + (size_t)p * KP + 4 * t) = *reinterpret_cast<const uint2 *>(hi);
    *reinterpret_cast<uint2 *>(Yhi1 + (size_t)p * KP + 4 * t) = *reinterpret_cast<const uint2 *>(hi);
    *reinterpret_cast<uint2 *>(Ylo + (size_t)p * KP + 4 * t) = *reinterpret_cast<const uint2 *>(lo);
    if (t == 0) {
        hn[p] = (float)(0.5 * s);
        const float wi = i >= 0 ? (w ? w[i] : 1.0f) : 0.0f;
        wp[p] = wi;
        lw[p] = wi > 0.0f ? (float)log((double)wi) : -__builtin_huge_valf();
    }
}

__global__ __launch_bounds__(kT) void k_blk_centroids(const int *__restrict__ blk_cluster,
                                                      const float *__restrict__ C, int nblk, int kp,
                                                      float *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= (int64_t)nblk * kp) return;
    const int b = (int)(e / kp), t = (int)(e % kp);
    out[e] = C[(size_t)blk_cluster[b] * kp + t];
}

// out[perm_pad[p]] = in[p] for real points; in[p] = src[perm_pad[p]] (0 on padding).
__global__ __launch_bounds__(kT) void k_unpermute(const float *__restrict__ in,
                                                  const int *__restrict__ perm_pad, int n_pad,
                                                  float *__restrict__ out) {
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= n_pad) return;
    const int i = perm_pad[p];
    if (i >= 0) out[i] = in[p];
}
__global__ __launch_bounds__(kT) void k_permute(const float *__restrict__ src,
                                                const int *__restrict__ perm_pad, int n_pad,
                                                float *__restrict__ out) {
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= n_pad) return;
    const int i = perm_pad[p];
    out[p] = i >= 0 ? src[i] : 0.0f;
}

// Centres back in the caller's coordinates: out[c*d + t] = C[c*kp + t] + centre[t].
__global__ __launch_bounds__(kT) void k_unpack_centres(const float *__restrict__ C, int k, int d,
                                                       int kp, const float *__restrict__ centre,
                                                       float *__restrict__ out) {
    const int e = blockIdx.x * kT + threadIdx.x;
    if (e >= k * d) return;
    const int c = e / d, t = e % d;
    out[e] = (float)((double)C[(size_t)c * kp + t] + (double)centre[t]);
}

static inline unsigned blocks(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

hipError_t launch_unpack_centres(const float *C, int k, int d, int kp, const float *centre,
                                 float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_unpack_centres, dim3(blocks((int64_t)k * d)), dim3(kT), 0, s, C, k, d, kp,
                       centre, out);
    return hipGetLastError();
}

#define SKH_KP_DISPATCH(kp, KERNEL, ...)                                         \
    switch (kp) {                                                                \
    case 4: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                   \
    case 8: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                   \
    case 16: hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__); break;                 \
    case 32: hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__); break;                 \
    case 64: hipLaunchKernelGGL(KERNEL<64>, __VA_ARGS__); break;                 \
    default: return hipErrorInvalidValue;                                        \
    }

size_t kmeans_workspace_ints(int n, int k) {
    const int nb = (n + kT - 1) / kT;
    const int64_t len = (int64_t)k * nb;
    // label, sorted_label, perm, counts, offs, scan sums, off (k+1)
    return (size_t)n * 3 + (size_t)len * 2 + (size_t)scan_sums_len(len) + (size_t)(k + 1) + 64;
}

hipError_t run_kmeans(const float *X, const float *w, int n, int kp, int k, int iters, float *C,
                      float *cmass, float *radius, int *ws, int **perm_out, int **off_out,
                      hipStream_t s) {
    const int nb = (n + kT - 1) / kT;
    const int64_t len = (int64_t)k * nb;
    int *label = ws;
    int *slabel = label + n;
    int *perm = slabel + n;
    int *counts = perm + n;
    int *offs = counts + len;
    int *sums = offs + len;
    int *off = sums + scan_sums_len(len);
    hipLaunchKernelGGL(k_init_centroids, dim3(blocks((int64_t)k * kp)), dim3(kT), 0, s, X, n, k, kp,
                       C);
    for (int it = 0; it <= iters; ++it) {
        SKH_KP_DISPATCH(kp, k_kmeans_assign, dim3((n + 127) / 128), dim3(256), 0, s, X, n, C, k,
                        label);
        hipLaunchKernelGGL(k_label_count, dim3(nb), dim3(kT), k * sizeof(int), s, label, n, k, nb,
                           counts);
        hipError_t e = launch_exclusive_scan(counts, len, sums, offs, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_label_scatter, dim3(nb), dim3(kT), 0, s, label, n, nb, offs, perm,
                           slabel);
        hipLaunchKernelGGL(k_cluster_offsets, dim3(blocks(k + 1)), dim3(kT), 0, s, offs, k, nb, n,
                           off);
        // the last pass only sorts by the final centres (labels consistent with C)
        if (it < iters) {
            SKH_KP_DISPATCH(kp, k_centroid_update, dim3(k), dim3(kCU), 0, s, X, w, perm, off, C,
                            cmass);
        }
    }
    // the coarse points are the weighted means of the final clusters, with their masses
    SKH_KP_DISPATCH(kp, k_centroid_update, dim3(k), dim3(kCU), 0, s, X, w, perm, off, C, cmass);
    if (radius) SKH_KP_DISPATCH(kp, k_cluster_radius, dim3(k), dim3(kT), 0, s, X, perm, off, C, radius);
    *perm_out = perm;
    *off_out = off;
    return hipGetLastError();
}

hipError_t build_padded_layout(const int *perm, const int *off, int k, int *psize, int *poff,
                               int *scan_sums, hipStream_t s) {
    hipLaunchKernelGGL(k_padded_sizes, dim3(blocks(k + 1)), dim3(kT), 0, s, off, k, psize);
    return launch_exclusive_scan(psize, k + 1, scan_sums, poff, s);
}

hipError_t fill_padded_layout(const int *perm, const int *off, const int *poff, int k,
                              int *perm_pad, int *blk_cluster, hipStream_t s) {
    hipLaunchKernelGGL(k_padded_layout, dim3(k), dim3(kT), 0, s, perm, off, poff, k, perm_pad,
                       blk_cluster);
    return hipGetLastError();
}

hipError_t launch_pack_padded(const float *X, const float *w, const int *perm_pad,
                              const int *blk_cluster, const float *C, int n_pad, int kp, float *Xf,
                              __hip_bfloat16 *Yhi0, __hip_bfloat16 *Yhi1, __hip_bfloat16 *Ylo,
                              float *hn, float *lw, float *wp, hipStream_t s) {
    if (n_pad == 0) return hipSuccess;
    const int ppb = kT / (kp / 4);  // points per block
    SKH_KP_DISPATCH(kp, k_pack_padded, dim3((n_pad + ppb - 1) / ppb), dim3(kT), 0, s, X, w,
                    perm_pad, blk_cluster, C, n_pad, Xf, Yhi0, Yhi1, Ylo, hn, lw, wp);
    return hipGetLastError();
}

hipError_t launch_blk_centroids(const int *blk_cluster, const float *C, int nblk, int kp,
                                float *blk_cent, hipStream_t s) {
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_blk_centroids, dim3(blocks((int64_t)nblk * kp)), dim3(kT), 0, s,
                       blk_cluster, C, nblk, kp, blk_cent);
    return hipGetLastError();
}

hipError_t launch_unpermute(const float *in, const int *perm_pad, int n_pad, float *out,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_unpermute, dim3(blocks(n_pad)), dim3(kT), 0, s, in, perm_pad, n_pad, out);
    return hipGetLastError();
}

// L values per point: out[p][l] = src[perm_pad[p]][l] (0 on padding), and back:
// out[perm_pad[p]][l] = in[p][l] for real points.
__global__ __launch_bounds__(kT) void k_permute_rows(const float *__restrict__ src,
                                                     const int *__restrict__ perm_pad, int n_pad,
                                                     int L, float *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= (int64_t)n_pad * L) return;
    const int p = (int)(e / L), l = (int)(e - (int64_t)p * L);
    const int i = perm_pad[p];
    out[e] = i >= 0 ? src[(size_t)i * L + l] : 0.0f;
}
__global__ __launch_bounds__(kT) void k_unpermute_rows(const float *__restrict__ in,
                                                       const int *__restrict__ perm_pad, int n_pad,
                                                       int L, float *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= (int64_t)n_pad * L) return;
    const int p = (int)(e / L), l = (int)(e - (int64_t)p * L);
    const int i = perm_pad[p];
    if (i >= 0) out[(size_t)i * L + l] = in[e];
}

hipError_t launch_permute_rows(const float *src, const int *perm_pad, int n_pad, int L, float *out,
                               hipStream_t s) {
    if (n_pad == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_rows, dim3(blocks((int64_t)n_pad * L)), dim3(kT), 0, s, src,
                       perm_pad, n_pad, L, out);
    return hipGetLastError();
}

hipError_t launch_unpermute_rows(const float *in, const int *perm_pad, int n_pad, int L,
                                 float *out, hipStream_t s) {
    if (n_pad == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpermute_rows, dim3(blocks((int64_t)n_pad * L)), dim3(kT), 0, s, in,
                       perm_pad, n_pad, L, out);
    return hipGetLastError();
}

hipError_t launch_permute(const float *src, const int *perm_pad, int n_pad, float *out,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(blocks(n_pad)), dim3(kT), 0, s, src, perm_pad, n_pad, out);
    return hipGetLastError();
}

}  // namespace skh

namespace skh {

// Labels in [0, k) check: *bad |= 1 for any label out of range.
__global__ __launch_bounds__(kT) void k_check_labels(const int *__restrict__ lab, int n, int k,
                                                     int *__restrict__ bad) {
    const int i = blockIdx.x * kT + threadIdx.x;
    const int b = i < n && (lab[i] < 0 || lab[i] >= k);
    if (__any(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

hipError_t launch_check_labels(const int *lab, int n, int k, int *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_check_labels, dim3(blocks(n)), dim3(kT), 0, s, lab, n, k, bad);
    return hipGetLastError();
}

// Stable counting sort of labels already in ws[0, n) (the K-means workspace
// layout): perm (sorted position -> point) and off (k + 1).
hipError_t sort_labels(int n, int k, int *ws, int **perm_out, int **off_out, hipStream_t s) {
    const int nb = (n + kT - 1) / kT;
    const int64_t len = (int64_t)k * nb;
    int *label = ws;
    int *slabel = label + n;
    int *perm = slabel + n;
    int *counts = perm + n;
    int *offs = counts + len;
    int *sums = offs + len;
    int *off = sums + scan_sums_len(len);
    hipLaunchKernelGGL(k_label_count, dim3(nb), dim3(kT), k * sizeof(int), s, label, n, k, nb, counts);
    hipError_t e = launch_exclusive_scan(counts, len, sums, offs, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_label_scatter, dim3(nb), dim3(kT), 0, s, label, n, nb, offs, perm, slabel);
    hipLaunchKernelGGL(k_cluster_offsets, dim3(blocks(k + 1)), dim3(kT), 0, s, offs, k, nb, n, off);
    *perm_out = perm;
    *off_out = off;
    return hipGetLastError();
}

}  // namespace skh

namespace skh {

// The clustering of run_kmeans from given labels (in [0, k), checked by the
// caller): stable sort by label, weighted means and radii, no Lloyd iterations.
hipError_t clusters_from_labels(const float *X, const float *w, int n, int kp, int k,
                                const int *labels, float *C, float *cmass, float *radius, int *ws,
                                int **perm_out, int **off_out, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(ws, labels, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    int *perm, *off;
    e = sort_labels(n, k, ws, &perm, &off, s);
    if (e != hipSuccess) return e;
    SKH_KP_DISPATCH(kp, k_centroid_update, dim3(k), dim3(kCU), 0, s, X, w, perm, off, C, cmass);
    if (radius) SKH_KP_DISPATCH(kp, k_cluster_radius, dim3(k), dim3(kT), 0, s, X, perm, off, C, radius);
    *perm_out = perm;
    *off_out = off;
    return hipGetLastError();
}

}  // namespace skh
