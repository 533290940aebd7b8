// O(n + m) kernels around the softmin: bounding box and validation, packing,
// column offsets, the per-iteration merge + averaging step of the Algorithm,
// the marginal-error sums, and the FP64 sums of eq. (6).  All reductions are
// two-stage with a fixed order (no floating-point atomics), so results are
// bitwise reproducible run to run.
#include "skh_internal.h"

namespace skh {

static __device__ __forceinline__ float finf() { return __builtin_huge_valf(); }

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.6931471805599453094;
constexpr int kBBoxSeg = 2048;
constexpr int kThreads = 256;

template <class T>
static __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
static __device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
static __device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

int bbox_blocks(int64_t n) { return (int)((n + kBBoxSeg - 1) / kBBoxSeg); }

// Block b covers points [b*SEG, (b+1)*SEG).  pbad[2b] counts non-finite
// coordinates, pbad[2b+1] negative, NaN or infinite weights.
// The block reads its points' coordinates as one contiguous run: thread t < S
// (S = the largest multiple of d not above the block size) takes the elements
// t, t + S, t + 2S, ... of the run, all of coordinate t % d; the per-coordinate
// extremes are then combined over the threads t % d = k.
__global__ __launch_bounds__(kThreads) void k_bbox_partial(const float *__restrict__ x,
                                                           const float *__restrict__ w, int64_t n,
                                                           int d, float *plo, float *phi,
                                                           double *pmass, int *pbad) {
    __shared__ float tlo[kThreads], thi[kThreads];
    __shared__ double sm[4];
    __shared__ int sb[4][2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t beg = (int64_t)blockIdx.x * kBBoxSeg;
    const int64_t end = min(n, beg + kBBoxSeg);
    const int S = (kThreads / d) * d;
    int badc = 0, badw = 0;
    float lo = finf(), hi = -finf();
    if (tid < S) {
        for (int64_t e = beg * d + tid; e < end * d; e += S) {
            const float v = x[e];
            if (!isfinite(v)) {
                ++badc;
            } else {
                lo = fminf(lo, v);
                hi = fmaxf(hi, v);
            }
        }
    }
    tlo[tid] = lo;
    thi[tid] = hi;
    double ms = 0.0;
    if (w) {
        for (int64_t i = beg + tid; i < end; i += kThreads) {
            const float v = w[i];
            if (!(v >= 0.0f) || !isfinite(v))
                ++badw;
            else
                ms += (double)v;
        }
    }
    ms = wave_sum(ms);
    badc = wave_sum(badc);
    badw = wave_sum(badw);
    if (lane == 0) {
        sm[wave] = ms;
        sb[wave][0] = badc;
        sb[wave][1] = badw;
    }
    __syncthreads();
    if (tid < d) {
        float l = finf(), h = -finf();
        for (int t = tid; t < S; t += d) {
            l = fminf(l, tlo[t]);
            h = fmaxf(h, thi[t]);
        }
        plo[(size_t)blockIdx.x * 64 + tid] = l;
        phi[(size_t)blockIdx.x * 64 + tid] = h;
    }
    if (tid == 0) {
        pmass[blockIdx.x] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
        pbad[2 * blockIdx.x] = sb[0][0] + sb[1][0] + sb[2][0] + sb[3][0];
        pbad[2 * blockIdx.x + 1] = sb[0][1] + sb[1][1] + sb[2][1] + sb[3][1];
    }
}

hipError_t launch_bbox_partial(const float *x, const float *w, int64_t n, int d, float *plo,
                               float *phi, double *pmass, int *pbad, hipStream_t s) {
    const int nb = bbox_blocks(n);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kThreads), 0, s, x, w, n, d, plo, phi, pmass,
                       pbad);
    return hipGetLastError();
}

// One block.  lohi: [lo[64], hi[64], centre[64]] of the union of both clouds;
// mass[2]: FP64 weight sums per cloud; bad[4]: the two counters per cloud.
__global__ __launch_bounds__(64) void k_bbox_final(const float *plo, const float *phi,
                                                   const double *pmass, const int *pbad, int nb0,
                                                   int nb1, int d, float *lohi, double *mass,
                                                   int *bad) {
    const int t = threadIdx.x;
    if (t < d) {
        float lo = finf(), hi = -finf();
        for (int b = 0; b < nb0 + nb1; ++b) {
            lo = fminf(lo, plo[(size_t)b * 64 + t]);
            hi = fmaxf(hi, phi[(size_t)b * 64 + t]);
        }
        lohi[t] = lo;
        lohi[64 + t] = hi;
        lohi[128 + t] = (float)(0.5 * ((double)lo + (double)hi));
    }
    if (t == 0) {
        double m0 = 0.0, m1 = 0.0;
        long long c0 = 0, w0 = 0, c1 = 0, w1 = 0;
        for (int b = 0; b < nb0; ++b) {
            m0 += pmass[b];
            c0 += pbad[2 * b];
            w0 += pbad[2 * b + 1];
        }
        for (int b = nb0; b < nb0 + nb1; ++b) {
            m1 += pmass[b];
            c1 += pbad[2 * b];
            w1 += pbad[2 * b + 1];
        }
        mass[0] = m0;
        mass[1] = m1;
        bad[0] = (int)min(c0, (long long)INT32_MAX);
        bad[1] = (int)min(w0, (long long)INT32_MAX);
        bad[2] = (int)min(c1, (long long)INT32_MAX);
        bad[3] = (int)min(w1, (long long)INT32_MAX);
    }
}

hipError_t launch_bbox_final(const float *plo, const float *phi, const double *pmass,
                             const int *pbad, int nb0, int nb1, int d, float *lohi, double *mass,
                             int *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, s, plo, phi, pmass, pbad, nb0, nb1, d,
                       lohi, mass, bad);
    return hipGetLastError();
}

// kp consecutive lanes share a point (kp divides the wave), one coordinate each, so the
// loads and stores of a wave are contiguous; the FP64 half norm is reduced across them.
__global__ __launch_bounds__(kThreads) void k_pack(const float *__restrict__ x,
                                                   const float *__restrict__ w, int64_t n, int d,
                                                   int kp, const float *__restrict__ centre,
                                                   float *__restrict__ P, float *__restrict__ hn,
                                                   float *__restrict__ lw) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t i = e / kp;
    const int k = (int)(e - i * kp);
    const bool live = i < n;
    const int64_t ic = live ? i : n - 1;  // every lane takes part in the reduction
    float v = 0.0f;
    if (k < d) v = (float)((double)x[ic * d + k] - (double)centre[k]);
    double s = (double)v * (double)v;
    for (int o = kp / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (!live) return;
    P[e] = v;
    if (k == 0) {
        hn[i] = (float)(0.5 * s);
        if (lw) {
            const float wi = w ? w[i] : 1.0f;
            lw[i] = wi > 0.0f ? (float)log((double)wi) : -finf();
        }
    }
}

hipError_t launch_pack(const float *x, const float *w, int64_t n, int d, int kp,
                       const float *centre, float *P, float *hn, float *lw, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((n * kp + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, x, w, n, d, kp, centre, P, hn, lw);
    return hipGetLastError();
}

static __device__ __forceinline__ float col_offset(float lw, double h, float hn, double inv_eps) {
    if (!(lw > -finf())) return -finf();
    return (float)(kLog2e * ((double)lw + (h - (double)hn) * inv_eps));
}

__global__ __launch_bounds__(kThreads) void k_col_offsets(const float *__restrict__ lw,
                                                          const float *__restrict__ h,
                                                          const float *__restrict__ hn, int64_t n,
                                                          double inv_eps, float *__restrict__ u) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    u[i] = col_offset(lw[i], h ? (double)h[i] : 0.0, hn[i], inv_eps);
}

hipError_t launch_col_offsets(const float *lw, const float *h, const float *hn, int64_t n,
                              double eps, float *u, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_col_offsets, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, lw, h, hn, n, 1.0 / eps, u);
    return hipGetLastError();
}

// log2 sum over the chunk partials of one row; -inf when the row saw no mass.
static __device__ __forceinline__ double merge_l2(const float2 *part, int chunks, int64_t n,
                                                  int64_t i) {
    float M = -finf();
    for (int c = 0; c < chunks; ++c) M = fmaxf(M, part[(size_t)c * n + i].x);
    if (!(M > -finf())) return -(double)finf();
    double S = 0.0;
    for (int c = 0; c < chunks; ++c) {
        const float2 v = part[(size_t)c * n + i];
        if (v.x > -finf()) S += (double)v.y * exp2((double)v.x - (double)M);
    }
    return (double)M + log2(S);
}

__global__ __launch_bounds__(kThreads) void k_softmin_finish(const float2 *__restrict__ part,
                                                             int chunks, int64_t n,
                                                             const float *__restrict__ hn,
                                                             double eps, double lam,
                                                             float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double L2 = merge_l2(part, chunks, n, i);
    out[i] = (float)(lam * ((double)hn[i] - eps * kLn2 * L2));
}

hipError_t launch_softmin_finish(const float2 *part, int n_chunks, int64_t n, const float *hn,
                                 double eps, double lam, float *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_softmin_finish, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, part, n_chunks, n, hn, eps, lam, out);
    return hipGetLastError();
}

int finish_blocks(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

// Block-level FP64 sum of 4 values per thread into acc[blk*4 + 0..3].
static __device__ void block_sum4(double v[4], double *acc_blk) {
    __shared__ double sh[4][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
        for (int k = 0; k < 4; ++k) sh[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        acc_blk[k] = ((sh[0][k] + sh[1][k]) + sh[2][k]) + sh[3][k];
    }
}

// The averaging step of the Algorithm for one point of one cloud, after its two
// softmins: tilde = lam (hn - eps ln2 L2), pot <- (pot + tilde) / 2.
// With check != 0 also the marginal-error sums: the plan's row mass
// w_i exp((pot_i - tilde_i / lam) / eps) = w_i exp((pot_i - hn_i)/eps + ln2 L2)
// (eq. (4) summed over the other cloud) against its target w_i (balanced) or
// w_i exp(-pot_i / rho).
__global__ __launch_bounds__(kThreads) void k_iteration_finish(FinishSide sx, FinishSide sy,
                                                               int nbx, double eps, double lam,
                                                               double rho, int balanced,
                                                               double inv_eps_next, int check,
                                                               double *acc) {
    const bool is_x = (int)blockIdx.x < nbx;
    const FinishSide &S = is_x ? sx : sy;
    const int64_t i = (int64_t)(is_x ? blockIdx.x : blockIdx.x - nbx) * kThreads + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < S.n) {
        // a problem without partials belongs to a fixed loop: its vector is left as given
        const bool has_s = S.part_self != nullptr, has_c = S.part_cross != nullptr;
        const double hn = S.hn[i];
        const double L2s = has_s ? merge_l2(S.part_self, S.chunks_self, S.n, i) : 0.0;
        const double L2c = has_c ? merge_l2(S.part_cross, S.chunks_cross, S.n, i) : 0.0;
        const double ts = lam * (hn - eps * kLn2 * L2s);
        const double tc = lam * (hn - eps * kLn2 * L2c);
        const double ps = S.pot_self[i], pc = S.pot_cross[i];
        if (check) {
            const double wi = S.w[i];
            if (wi > 0.0) {
                if (has_c) {
                    const double rc = wi * exp((pc - hn) / eps + kLn2 * L2c);
                    const double tgc = balanced ? wi : wi * exp(-pc / rho);
                    v[0] = fabs(rc - tgc);
                    v[1] = tgc;
                }
                if (has_s) {
                    const double rs = wi * exp((ps - hn) / eps + kLn2 * L2s);
                    const double tgs = balanced ? wi : wi * exp(-ps / rho);
                    v[2] = fabs(rs - tgs);
                    v[3] = tgs;
                }
            }
        }
        const float lw = S.lw[i], hnf = S.hn[i];
        if (has_s) {
            const float ns = (float)(0.5 * (ps + ts));
            S.pot_self[i] = ns;
            S.u_self[i] = col_offset(lw, (double)ns, hnf, inv_eps_next);
        }
        if (has_c) {
            const float nc = (float)(0.5 * (pc + tc));
            S.pot_cross[i] = nc;
            S.u_cross[i] = col_offset(lw, (double)nc, hnf, inv_eps_next);
        }
    }
    if (check) block_sum4(v, acc + (size_t)blockIdx.x * 4);
}

hipError_t launch_iteration_finish(const FinishSide &sx, const FinishSide &sy, double eps,
                                   double lam, double rho, int balanced, double eps_next,
                                   int check, double *acc, hipStream_t s) {
    const int nbx = finish_blocks(sx.n), nby = finish_blocks(sy.n);
    hipLaunchKernelGGL(k_iteration_finish, dim3(nbx + nby), dim3(kThreads), 0, s, sx, sy, nbx, eps,
                       lam, rho, balanced, 1.0 / eps_next, check, acc);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_sum_partials(const double *__restrict__ part, int nb,
                                                           int W, double *__restrict__ out) {
    __shared__ double sh[kThreads];
    for (int w = 0; w < W; ++w) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += kThreads) s += part[(size_t)b * W + w];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int o = kThreads / 2; o >= 1; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[w] = sh[0];
        __syncthreads();
    }
}

hipError_t launch_sum_partials(const double *part, int nb, int W, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kThreads), 0, s, part, nb, W, out);
    return hipGetLastError();
}

// eq. (6) terms, FP64.  Balanced: w (pc - ps).  Unbalanced:
// w e^{-ps/rho} expm1(-(pc - ps)/rho)  (= w (e^{-pc/rho} - e^{-ps/rho})); the
// caller multiplies the sum by -(rho + eps/2).
__global__ __launch_bounds__(kThreads) void k_divergence_terms(
    const float *__restrict__ a, const float *__restrict__ f, const float *__restrict__ p, int64_t n,
    const float *__restrict__ b, const float *__restrict__ g, const float *__restrict__ q, int64_t m,
    int nbx, double rho, int balanced, double *part) {
    const bool is_x = (int)blockIdx.x < nbx;
    const int64_t i = (int64_t)(is_x ? blockIdx.x : blockIdx.x - nbx) * kThreads + threadIdx.x;
    const int64_t len = is_x ? n : m;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < len) {
        const double w = is_x ? a[i] : b[i];
        const double pc = is_x ? f[i] : g[i];
        const double ps = is_x ? p[i] : q[i];
        if (w > 0.0) v[0] = balanced ? w * (pc - ps) : w * exp(-ps / rho) * expm1(-(pc - ps) / rho);
    }
    block_sum4(v, part + (size_t)blockIdx.x * 4);
}

hipError_t launch_divergence_terms(const float *a, const float *f, const float *p, int64_t n,
                                   const float *b, const float *g, const float *q, int64_t m,
                                   double rho, int balanced, double *part, int *nb_out,
                                   hipStream_t s) {
    const int nbx = finish_blocks(n), nby = finish_blocks(m);
    *nb_out = nbx + nby;
    hipLaunchKernelGGL(k_divergence_terms, dim3(nbx + nby), dim3(kThreads), 0, s, a, f, p, n, b, g,
                       q, m, nbx, rho, balanced, part);
    return hipGetLastError();
}

// eq. (6) per pair of a batched solve: one workgroup per pair k sums its x points
// [xo[k], xo[k+1]) and y points [yo[k], yo[k+1]) in FP64 (fixed order per thread, then a
// tree); out[k] is the bracket of eq. (6) (balanced: the value itself).
__global__ __launch_bounds__(kThreads) void k_divergence_segments(
    const float *__restrict__ a, const float *__restrict__ f, const float *__restrict__ p,
    const int64_t *__restrict__ xo, const float *__restrict__ b, const float *__restrict__ g,
    const float *__restrict__ q, const int64_t *__restrict__ yo, double rho, int balanced,
    double *__restrict__ out) {
    __shared__ double red[kThreads];
    const int k = blockIdx.x;
    double v = 0.0;
    for (int side = 0; side < 2; ++side) {
        const int64_t lo = side ? yo[k] : xo[k], hi = side ? yo[k + 1] : xo[k + 1];
        const float *w = side ? b : a, *pc = side ? g : f, *ps = side ? q : p;
        for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
            const double wi = w[i];
            if (wi > 0.0) {
                const double c = pc[i], t = ps[i];
                v += balanced ? wi * (c - t) : wi * exp(-t / rho) * expm1(-(c - t) / rho);
            }
        }
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
}

hipError_t launch_divergence_segments(const float *a, const float *f, const float *p,
                                      const int64_t *xo, const float *b, const float *g,
                                      const float *q, const int64_t *yo, int K, double rho,
                                      int balanced, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_divergence_segments, dim3(K), dim3(kThreads), 0, s, a, f, p, xo, b, g, q,
                       yo, rho, balanced, out);
    return hipGetLastError();
}

}  // namespace skh
