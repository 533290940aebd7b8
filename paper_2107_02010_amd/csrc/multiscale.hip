// Coarse-to-fine support (Section 2, coarse-to-fine strategy, which cites
// Schmitzer's kernel truncation): a cluster block of the fine softmin is left
// out when the current dual vectors bound all its weights below e^{-theta};
// also the coarse measures of the K-means clusters.
//
// Truncation test for a row cluster I and a column cluster J, for the softmin
// whose rows carry potential f (scaled by 1/lambda inside the softmin) and
// whose columns carry g:
//
//   an entry (i, j) has normalised weight b_j exp((f_i/lam + g_j - C_ij)/eps) in
//   row i's sum, so the whole block is below b_j e^{-theta} when
//       max_I f / lam + max_J g - min_{i in I, j in J} C_ij  <  -theta eps,
//   with min C >= (max(0, |c_I - c_J| - r_I - r_J))^2 / 2 (centres c, radii r).
//
// The score takes the larger of (f/lam + g) and (f + g/lam) so that the
// (I, J) mask of one problem is the transpose of the (J, I) mask of the
// problem with rows and columns swapped.  The best-scoring block of every row
// cluster is always kept, so no row loses all of its columns.  Kept clusters
// that are adjacent in the padded column order merge into one range.
#include "skh_internal.h"

namespace skh {

constexpr int kT = 256;

static __device__ __forceinline__ float finf() { return __builtin_huge_valf(); }

// out[c] = max of pot over the members of cluster c with positive weight
// (padded order, cluster c at [poff[c], poff[c+1])); -inf when none.
__global__ __launch_bounds__(kT) void k_cluster_max(const float *__restrict__ pot,
                                                    const float *__restrict__ w,
                                                    const int *__restrict__ poff, int k,
                                                    float *__restrict__ out) {
    __shared__ float sh[kT];
    const int c = blockIdx.x;
    float v = -finf();
    for (int p = poff[c] + threadIdx.x; p < poff[c + 1]; p += kT)
        if (w[p] > 0.0f) v = fmaxf(v, pot[p]);
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kT / 2; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
}

hipError_t launch_cluster_max(const float *pot, const float *w, const int *poff, int k, float *out,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_cluster_max, dim3(k), dim3(kT), 0, s, pot, w, poff, k, out);
    return hipGetLastError();
}

// dist[I * kj + J] = |CI_I - CJ_J|  (centres packed with stride kp)
__global__ __launch_bounds__(kT) void k_centroid_dist(const float *__restrict__ CI, int ki,
                                                      const float *__restrict__ CJ, int kj, int kp,
                                                      float *__restrict__ dist) {
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= (int64_t)ki * kj) return;
    const int I = (int)(e / kj), J = (int)(e % kj);
    double s = 0.0;
    for (int t = 0; t < kp; ++t) {
        const double v = (double)CI[(size_t)I * kp + t] - (double)CJ[(size_t)J * kp + t];
        s += v * v;
    }
    dist[e] = (float)sqrt(s);
}

hipError_t launch_centroid_dist(const float *CI, int ki, const float *CJ, int kj, int kp,
                                float *dist, hipStream_t s) {
    const int64_t n = (int64_t)ki * kj;
    hipLaunchKernelGGL(k_centroid_dist, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, CI, ki,
                       CJ, kj, kp, dist);
    return hipGetLastError();
}

// One workgroup per row cluster I: the kept column ranges (padded order) and the
// number of real point pairs they hold (added to *pairs).  Thread t owns the
// column clusters [t CH, (t+1) CH).  A cluster is in a run when it is kept or
// empty (an empty cluster has no columns, so it never breaks a run); run starts
// and ends are found in parallel and the i-th start pairs with the i-th end.
constexpr int kBR = 256;

__global__ __launch_bounds__(kBR) void k_block_ranges(
    int ki, int kj, const float *__restrict__ rmax, const float *__restrict__ cmax,
    const float *__restrict__ dist, const float *__restrict__ rrad, const float *__restrict__ crad,
    const int *__restrict__ cpoff, const int *__restrict__ coff, const int *__restrict__ roff,
    float inv_lam, float theta_eps, int keep_all, int cap, int2 *__restrict__ ranges,
    int *__restrict__ count, unsigned long long *__restrict__ pairs) {
    const int I = blockIdx.x, t = threadIdx.x;
    __shared__ float sbs[kBR];
    __shared__ int sbj[kBR];
    __shared__ int sst[kBR], sen[kBR];
    __shared__ long long scols[kBR];
    const float fm = rmax[I];
    const long long rows_real = roff[I + 1] - roff[I];
    if (!(fm > -finf()) || rows_real == 0) {  // uniform over the workgroup
        if (t == 0) count[I] = 0;
        return;
    }
    const int CH = (kj + kBR - 1) / kBR;
    const int J0 = min(kj, t * CH), J1 = min(kj, J0 + CH);
    auto score = [&](int J) -> float {
        const float gm = cmax[J];
        if (!(gm > -finf())) return -finf();
        const float gap = fmaxf(0.0f, dist[(size_t)I * kj + J] - rrad[I] - crad[J]);
        return fmaxf(fm * inv_lam + gm, fm + gm * inv_lam) - 0.5f * gap * gap;
    };
    // the best block (first maximum in column order) is always kept
    float bs = -finf();
    int bj = -1;
    if (!keep_all)
        for (int J = J0; J < J1; ++J) {
            const float sc = score(J);
            if (sc > bs) {
                bs = sc;
                bj = J;
            }
        }
    sbs[t] = bs;
    sbj[t] = bj;
    __syncthreads();
    for (int o = kBR / 2; o >= 1; o >>= 1) {  // ties keep the lower thread: the lower J
        if (t < o && sbs[t + o] > sbs[t]) {
            sbs[t] = sbs[t + o];
            sbj[t] = sbj[t + o];
        }
        __syncthreads();
    }
    const int best = sbj[0];
    auto in_run = [&](int J) -> bool {
        if (cpoff[J + 1] == cpoff[J]) return true;  // empty
        return keep_all || J == best || score(J) >= -theta_eps;
    };
    // starts, ends and real columns of this thread's clusters
    int nst = 0, nen = 0;
    long long cols = 0;
    bool prev = J0 > 0 ? in_run(J0 - 1) : false;
    for (int J = J0; J < J1; ++J) {
        const bool cur = in_run(J);
        const bool next = J + 1 < kj ? in_run(J + 1) : false;
        nst += cur && !prev;
        nen += cur && !next;
        if (cur && cpoff[J + 1] > cpoff[J]) cols += coff[J + 1] - coff[J];
        prev = cur;
    }
    sst[t] = nst;
    sen[t] = nen;
    scols[t] = cols;
    __syncthreads();
    // exclusive scans of the start and end counts (Hillis-Steele), sum of columns
    for (int o = 1; o < kBR; o <<= 1) {
        const int a = t >= o ? sst[t - o] : 0, b = t >= o ? sen[t - o] : 0;
        const long long c = t >= o ? scols[t - o] : 0;
        __syncthreads();
        sst[t] += a;
        sen[t] += b;
        scols[t] += c;
        __syncthreads();
    }
    int rs = sst[t] - nst, re = sen[t] - nen;  // ranks of this thread's first start / end
    int2 *out = ranges + (size_t)I * cap;
    prev = J0 > 0 ? in_run(J0 - 1) : false;
    for (int J = J0; J < J1; ++J) {
        const bool cur = in_run(J);
        const bool next = J + 1 < kj ? in_run(J + 1) : false;
        if (cur && !prev) {
            if (rs < cap) out[rs].x = cpoff[J];
            ++rs;
        }
        if (cur && !next) {
            if (re < cap) out[re].y = cpoff[J + 1];
            ++re;
        }
        prev = cur;
    }
    if (t == kBR - 1) {
        count[I] = min(sst[kBR - 1], cap);
        atomicAdd(pairs, (unsigned long long)(rows_real * scols[kBR - 1]));
    }
}

hipError_t launch_block_ranges(int ki, int kj, const float *rmax, const float *cmax,
                               const float *dist, const float *rrad, const float *crad,
                               const int *cpoff, const int *coff, const int *roff, double lam,
                               double theta_eps, int keep_all, int cap, int2 *ranges, int *count,
                               unsigned long long *pairs, hipStream_t s) {
    if (ki <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_ranges, dim3(ki), dim3(kBR), 0, s, ki, kj, rmax, cmax, dist, rrad,
                       crad, cpoff, coff, roff, (float)(1.0 / lam), (float)theta_eps, keep_all, cap,
                       ranges, count, pairs);
    return hipGetLastError();
}

// Coarse measure of a clustered cloud: half squared norms and log masses of the
// centres (packed, stride kp).
__global__ __launch_bounds__(kT) void k_coarse_prep(const float *__restrict__ C,
                                                    const float *__restrict__ cmass, int k, int kp,
                                                    float *__restrict__ hn,
                                                    float *__restrict__ lw) {
    const int c = blockIdx.x * kT + threadIdx.x;
    if (c >= k) return;
    double s = 0.0;
    for (int t = 0; t < kp; ++t) s += (double)C[(size_t)c * kp + t] * (double)C[(size_t)c * kp + t];
    hn[c] = (float)(0.5 * s);
    lw[c] = cmass[c] > 0.0f ? (float)log((double)cmass[c]) : -finf();
}

hipError_t launch_coarse_prep(const float *C, const float *cmass, int k, int kp, float *hn,
                              float *lw, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse_prep, dim3((k + kT - 1) / kT), dim3(kT), 0, s, C, cmass, k, kp, hn,
                       lw);
    return hipGetLastError();
}

}  // namespace skh

namespace skh {

// Row tiles of the block-sparse softmin: cluster c (padded range
// [poff[c], poff[c+1])) splits into ceil(size / kRowsPerBlock) tiles.
__global__ __launch_bounds__(kT) void k_tile_counts(const int *__restrict__ poff, int k,
                                                    int *__restrict__ cnt) {
    const int c = blockIdx.x * kT + threadIdx.x;
    if (c < k) cnt[c] = (poff[c + 1] - poff[c] + kRowsPerBlock - 1) / kRowsPerBlock;
    if (c == k) cnt[k] = 0;
}

__global__ __launch_bounds__(kT) void k_tile_fill(const int *__restrict__ poff,
                                                  const int *__restrict__ toff, int k,
                                                  int4 *__restrict__ tiles) {
    const int c = blockIdx.x;
    const int n = toff[c + 1] - toff[c];
    for (int t = threadIdx.x; t < n; t += kT) {
        const int b = poff[c] + t * kRowsPerBlock;
        tiles[toff[c] + t] = make_int4(b, min(poff[c + 1], b + kRowsPerBlock), c, 0);
    }
}

hipError_t build_row_tiles(const int *poff, int k, int *cnt, int *toff, int *scan_sums,
                           int4 *tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_counts, dim3((k + 1 + kT - 1) / kT), dim3(kT), 0, s, poff, k, cnt);
    hipError_t e = launch_exclusive_scan(cnt, k + 1, scan_sums, toff, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_fill, dim3(k), dim3(kT), 0, s, poff, toff, k, tiles);
    return hipGetLastError();
}

}  // namespace skh
