// Transport plan applied to column values, and the weighted sums behind the
// gradient of S with respect to x.
//
// With the dual vectors (f, g) the plan is pi_ij = a_i b_j exp((f_i + g_j - C_ij)/eps)
// (eq. (4)).  For a row i and column values V_j (L of them) the kernel computes
//
//   W_i = sum_j 2^{s_ij - M_i},   P_il = sum_j 2^{s_ij - M_i} V_jl,
//   s_ij = k <x_i, y_j> + u_j,    u_j = log2(e) (log b_j + (g_j - |y_j|^2/2) / eps),
//
// with the running maximum M_i kept online exactly as in the softmin kernel,
// so that
//   sum_j pi_ij V_jl = a_i 2^{log2(e) (f_i - |x_i|^2/2) / eps + M_i} P_il.
//
// V is either a caller matrix (m x L, staged in LDS) or, for the gradient,
// the centred column coordinates themselves (L = d, read from the tile).
// s_ij comes from v_mfma_f32_32x32x2f32 as in the softmin; the accumulator
// layout of that instruction gives lane l (row i = l % 32) the columns
// j = 8 (r / 4) + 4 (l / 32) + (r % 4) of its 16 registers r, which is how
// each lane finds the V rows to weight.
#include "skh_internal.h"

namespace skh {

typedef float v16f __attribute__((ext_vector_type(16)));

static __device__ __forceinline__ float ninf() { return -__builtin_huge_valf(); }
static __device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

template <int KP, int LP>
__global__ __launch_bounds__(256) void k_plan_weighted(const PlanBatch B) {
    constexpr int H = KP / 2;
    constexpr int STRIDE = KP + 4;
    constexpr int V4 = KP / 4;
    // value rows: the matrix-core path reads one float per lane from rows 4 apart in the
    // two lane halves, so the stride keeps those 32 words apart in the banks
    constexpr int VSTRIDE = LP >= 32 ? LP + 8 : LP + 4;
    constexpr bool kMfmaValues = LP >= 32;
    constexpr int NT2 = kMfmaValues ? LP / 32 : 1;  // 32-wide value tiles
    // columns per LDS tile: 128, or 64 when 128 would take more than 40 KB of LDS, so
    // that four workgroups (four waves per SIMD) fit the 160 KB of a CU
    constexpr int TC = (STRIDE + VSTRIDE) * 4 * kColsPerTile > 40 * 1024 ? 64 : kColsPerTile;
    __shared__ __attribute__((aligned(16))) float tile[TC * STRIDE];
    __shared__ __attribute__((aligned(16))) float vtile[TC * VSTRIDE];

    const int wg = blockIdx.x;
    int q = 0;
#pragma unroll
    for (int t = 1; t < kMaxJobs; ++t)
        if (t < B.n_jobs && wg >= B.job[t].wg_begin) q = t;
    const PlanJob &J = B.job[q];
    const float *__restrict__ rows = J.rows;
    const float *__restrict__ cols = J.cols;
    const float *__restrict__ u = J.u;
    const float *__restrict__ V = J.V;
    float *__restrict__ part = J.part;
    const int n_rows = J.n_rows, n_cols = J.n_cols, L = J.L;
    const int row_tiles = J.row_tiles, chunk_cols = J.chunk_cols;
    const int local = wg - J.wg_begin;
    const int d = B.d;
    const float kscale = B.kscale;
    int rb, re, chunk, nranges;
    const int2 *rng = nullptr;
    int c_begin = 0, c_end = 0;
    int r0 = 0, rstep = 1;
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
        const int rt = local % row_tiles;
        chunk = local / row_tiles;
        rb = rt * kRowsPerBlock;
        re = min(n_rows, rb + kRowsPerBlock);
        c_begin = chunk * chunk_cols;
        c_end = min(n_cols, c_begin + chunk_cols);
        nranges = 1;
    }

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, li = lane & 31;
    const int i = rb + wave * 32 + li;
    const int ic = i < re ? i : re - 1;

    float xr[H];
    {
        const float *rp = rows + (size_t)ic * KP + h * H;
#pragma unroll
        for (int s = 0; s < H; ++s) xr[s] = rp[s];
#pragma unroll
        for (int s = 0; s < H; ++s) xr[s] = (h * H + s == d) ? 1.0f : xr[s] * kscale;
    }

    float m = ninf(), wsum = 0.0f;
    float vacc[kMfmaValues ? 1 : LP];
#pragma unroll
    for (int l = 0; l < (kMfmaValues ? 1 : LP); ++l) vacc[l] = 0.0f;
    v16f pacc[NT2];
#pragma unroll
    for (int t = 0; t < NT2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) pacc[t][r] = 0.0f;

    for (int ri = r0; ri < nranges; ri += rstep) {
    if (rng) {
        c_begin = rng[ri].x;
        c_end = rng[ri].y;
    }
    for (int j0 = c_begin; j0 < c_end; j0 += TC) {
        __syncthreads();
        for (int e = tid; e < TC * V4; e += 256) {
            const int c = e / V4, v = e - c * V4;
            const int j = j0 + c;
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < c_end) val = *reinterpret_cast<const float4 *>(cols + (size_t)j * KP + v * 4);
            *reinterpret_cast<float4 *>(&tile[c * STRIDE + v * 4]) = val;
        }
        for (int e = tid; e < TC * LP; e += 256) {
            const int c = e / LP, l = e - c * LP;
            const int j = j0 + c;
            float val = 0.0f;
            if (j < c_end && l < L) val = V ? V[(size_t)j * L + l] : cols[(size_t)j * KP + l];
            vtile[c * VSTRIDE + l] = val;
        }
        __syncthreads();
        if (tid < TC) {  // augmented coordinate: the column offset
            const int j = j0 + tid;
            tile[tid * STRIDE + d] = j < c_end ? u[j] : ninf();
        }
        __syncthreads();
        const int nblk = min(TC / 32, (c_end - j0 + 31) >> 5);
        for (int jb = 0; jb < nblk; ++jb) {
            v16f acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                        0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const float *tp = &tile[(jb * 32 + li) * STRIDE + h * H];
#pragma unroll
            for (int s = 0; s < H; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(tp[s], xr[s], acc, 0, 0, 0);
            float tmax = acc[0];
#pragma unroll
            for (int r = 1; r < 16; ++r) tmax = fmaxf(tmax, acc[r]);
            if constexpr (kMfmaValues) {
                // One level per row: both lane halves feed the same K-reduction below.
                // Register r of lane (row li, half h) holds the weight of column
                // c_r(h) = 8 (r / 4) + 4 h + r % 4, which is exactly the B operand
                // (K index h, column li) of a v_mfma_f32_32x32x2f32 summing over the
                // column pair {c_r(0), c_r(1)}; A is V at those columns for 32 values.
                // The products run with every lane active (no branch around them): a
                // block of masked columns (u_j = -inf, the same for every row) uses
                // base 0, so its weights are exactly 0.
                tmax = fmaxf(tmax, __shfl_xor(tmax, 32, 64));
                const float mn = fmaxf(m, tmax);
                if (mn > m) {
                    const float sc = fast_exp2(m - mn);  // 0 while m = -inf
                    wsum *= sc;
#pragma unroll
                    for (int t = 0; t < NT2; ++t)
#pragma unroll
                        for (int r = 0; r < 16; ++r) pacc[t][r] *= sc;
                    m = mn;
                }
                const float base = m > ninf() ? m : 0.0f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float w = fast_exp2(acc[r] - base);
                    wsum += w;
                    const int jl = jb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
#pragma unroll
                    for (int t = 0; t < NT2; ++t)
                        pacc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            vtile[jl * VSTRIDE + 32 * t + li], w, pacc[t], 0, 0, 0);
                }
            } else {
                const float mn = fmaxf(m, tmax);
                if (mn > ninf()) {
                    const float sc = fast_exp2(m - mn);
                    wsum *= sc;
#pragma unroll
                    for (int l = 0; l < LP; ++l) vacc[l] *= sc;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float w = fast_exp2(acc[r] - mn);
                        wsum += w;
                        const int jl = jb * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                        const float *vr = &vtile[jl * VSTRIDE];
#pragma unroll
                        for (int l = 0; l < LP; l += 4) {
                            const float4 vv = *reinterpret_cast<const float4 *>(vr + l);
                            vacc[l] = fmaf(w, vv.x, vacc[l]);
                            if (l + 1 < LP) vacc[l + 1] = fmaf(w, vv.y, vacc[l + 1]);
                            if (l + 2 < LP) vacc[l + 2] = fmaf(w, vv.z, vacc[l + 2]);
                            if (l + 3 < LP) vacc[l + 3] = fmaf(w, vv.w, vacc[l + 3]);
                        }
                    }
                    m = mn;
                }
            }
        }
    }

    }  // ranges

    const int RW = L + 2;
    float *rec = part + ((size_t)chunk * n_rows + ic) * RW;
    if constexpr (kMfmaValues) {
        // the level is row-uniform and each value sum is complete in one lane:
        // lane (li, h) holds values 32 t + 8 (r / 4) + 4 h + r % 4 of row li
        const float W = wsum + __shfl_xor(wsum, 32, 64);
        if (i < re) {
#pragma unroll
            for (int t = 0; t < NT2; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int l = 32 * t + 8 * (r >> 2) + 4 * h + (r & 3);
                    if (l < L) rec[2 + l] = pacc[t][r];
                }
            if (h == 0) {
                rec[0] = m;
                rec[1] = W;
            }
        }
    } else {
        // merge the two lane halves of each row
        const float m2 = __shfl_xor(m, 32, 64);
        const float M = fmaxf(m, m2);
        const float s1 = M > ninf() ? fast_exp2(m - M) : 0.0f;
        const float s2 = M > ninf() ? fast_exp2(m2 - M) : 0.0f;
        const float w2 = __shfl_xor(wsum, 32, 64);
        const float W = wsum * s1 + w2 * s2;
        // partial record: [M, W, P_0 .. P_{L-1}]
#pragma unroll
        for (int l = 0; l < LP; ++l) {
            const float o = __shfl_xor(vacc[l], 32, 64);
            const float val = vacc[l] * s1 + o * s2;
            if (h == 0 && i < re && l < L) rec[2 + l] = val;
        }
        if (h == 0 && i < re) {
            rec[0] = M;
            rec[1] = W;
        }
    }
}

int plan_plan_batch(PlanBatch &b, int target_wgs) {
    int row_tiles_total = 0;
    for (int q = 0; q < b.n_jobs; ++q) {
        PlanJob &J = b.job[q];
        J.row_tiles = (J.n_rows + kRowsPerBlock - 1) / kRowsPerBlock;
        row_tiles_total += J.row_tiles;
    }
    bool sparse = false;
    for (int q = 0; q < b.n_jobs; ++q) sparse = sparse || b.job[q].tiles != nullptr;
    if (sparse) {  // block-sparse: each row tile's range list over up to kMaxPlanTileChunks
        int tiles_total = 0;
        for (int q = 0; q < b.n_jobs; ++q) tiles_total += b.job[q].n_tiles;
        int c = tiles_total > 0 ? (target_wgs + tiles_total - 1) / tiles_total : 1;
        c = c < 1 ? 1 : (c > kMaxPlanTileChunks ? kMaxPlanTileChunks : c);
        int total = 0;
        for (int q = 0; q < b.n_jobs; ++q) {
            PlanJob &J = b.job[q];
            J.chunk_cols = 0;
            J.n_chunks = J.range_cap > 1 ? c : 1;
            J.wg_begin = total;
            total += J.n_tiles * J.n_chunks;
        }
        return total;
    }
    int want_chunks = row_tiles_total > 0 ? (target_wgs + row_tiles_total - 1) / row_tiles_total : 1;
    if (want_chunks < 1) want_chunks = 1;
    // each chunk holds L + 2 floats per row and the merge walks them per row
    if (want_chunks > 64) want_chunks = 64;
    int total = 0;
    for (int q = 0; q < b.n_jobs; ++q) {
        PlanJob &J = b.job[q];
        const int tiles = (J.n_cols + kColsPerTile - 1) / kColsPerTile;
        int per = (tiles + want_chunks - 1) / want_chunks;
        if (per < 1) per = 1;
        J.chunk_cols = per * kColsPerTile;
        J.n_chunks = (J.n_cols + J.chunk_cols - 1) / J.chunk_cols;
        if (J.n_chunks < 1) J.n_chunks = 1;
        J.wg_begin = total;
        total += J.row_tiles * J.n_chunks;
    }
    return total;
}

int plan_value_width(int L) {
    int lp = 4;
    while (lp < L) lp *= 2;
    return lp <= 64 ? lp : 0;
}

template <int KP>
static hipError_t launch_kp(const PlanBatch &b, int lp, dim3 grid, hipStream_t s) {
    switch (lp) {
    case 4: hipLaunchKernelGGL((k_plan_weighted<KP, 4>), grid, dim3(256), 0, s, b); break;
    case 8: hipLaunchKernelGGL((k_plan_weighted<KP, 8>), grid, dim3(256), 0, s, b); break;
    case 16: hipLaunchKernelGGL((k_plan_weighted<KP, 16>), grid, dim3(256), 0, s, b); break;
    case 32: hipLaunchKernelGGL((k_plan_weighted<KP, 32>), grid, dim3(256), 0, s, b); break;
    case 64: hipLaunchKernelGGL((k_plan_weighted<KP, 64>), grid, dim3(256), 0, s, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_plan_weighted(const PlanBatch &b, int kp, int lp, int total_wgs, hipStream_t s) {
    dim3 grid(total_wgs);
    switch (kp) {
    case 4: return launch_kp<4>(b, lp, grid, s);
    case 8: return launch_kp<8>(b, lp, grid, s);
    case 16: return launch_kp<16>(b, lp, grid, s);
    case 32: return launch_kp<32>(b, lp, grid, s);
    case 64: return launch_kp<64>(b, lp, grid, s);
    default: return hipErrorInvalidValue;
    }
}

// Merges chunk records [M, W, P_0..P_{L-1}] of one job into
//   out_il = scale_i 2^{c_i + M_i} P_il,  c_i = log2(e) (pot_i - hn_i) / eps,
// scale_i = w_i (or 1), and mass_i = scale_i 2^{c_i + M_i} W_i when mass != NULL.
// One factor 2^{M_c - M} per chunk; the value sums (LP >= L of them) stay in registers.
template <int LP>
__global__ __launch_bounds__(256) void k_plan_finish(const float *__restrict__ part, int chunks,
                                                     int n, int L, const float *__restrict__ hn,
                                                     const float *__restrict__ pot,
                                                     const float *__restrict__ w, double eps,
                                                     float *__restrict__ out,
                                                     float *__restrict__ mass) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int RW = L + 2;
    float M = ninf();
    for (int c = 0; c < chunks; ++c) M = fmaxf(M, part[((size_t)c * n + i) * RW]);
    const double scale = w ? (double)w[i] : 1.0;
    double base = 0.0;
    if (M > ninf())
        base = scale * exp2(1.4426950408889634074 * ((double)pot[i] - (double)hn[i]) / eps + (double)M);
    double acc[LP], W = 0.0;
#pragma unroll
    for (int l = 0; l < LP; ++l) acc[l] = 0.0;
    for (int c = 0; c < chunks; ++c) {
        const float *rec = part + ((size_t)c * n + i) * RW;
        if (!(rec[0] > ninf())) continue;
        const double f = exp2((double)rec[0] - (double)M);
#pragma unroll
        for (int l = 0; l < LP; ++l)
            if (l < L) acc[l] += (double)rec[2 + l] * f;
        W += (double)rec[1] * f;
    }
#pragma unroll
    for (int l = 0; l < LP; ++l)
        if (l < L) out[(size_t)i * L + l] = (float)(base * acc[l]);
    if (mass) mass[i] = (float)(base * W);
}

hipError_t launch_plan_finish(const float *part, int chunks, int n, int L, const float *hn,
                              const float *pot, const float *w, double eps, float *out,
                              float *mass, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const dim3 grid((n + 255) / 256), block(256);
    switch (plan_value_width(L)) {
    case 4: hipLaunchKernelGGL(k_plan_finish<4>, grid, block, 0, s, part, chunks, n, L, hn, pot, w, eps, out, mass); break;
    case 8: hipLaunchKernelGGL(k_plan_finish<8>, grid, block, 0, s, part, chunks, n, L, hn, pot, w, eps, out, mass); break;
    case 16: hipLaunchKernelGGL(k_plan_finish<16>, grid, block, 0, s, part, chunks, n, L, hn, pot, w, eps, out, mass); break;
    case 32: hipLaunchKernelGGL(k_plan_finish<32>, grid, block, 0, s, part, chunks, n, L, hn, pot, w, eps, out, mass); break;
    case 64: hipLaunchKernelGGL(k_plan_finish<64>, grid, block, 0, s, part, chunks, n, L, hn, pot, w, eps, out, mass); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// grad_i = (m1_i x_i - P1_i) - (m2_i x_i - P2_i), x centred (packed, stride kp);
// P1 = sum_j pi_ij y_j, m1 = sum_j pi_ij, P2 = sum_k pi^aa_ik x_k, m2 = sum_k pi^aa_ik.
__global__ __launch_bounds__(256) void k_grad_combine(const float *__restrict__ X, int n, int d,
                                                      int kp, const float *__restrict__ P1,
                                                      const float *__restrict__ m1,
                                                      const float *__restrict__ P2,
                                                      const float *__restrict__ m2,
                                                      float *__restrict__ grad) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n * d) return;
    const int i = e / d, t = e % d;
    const double x = X[(size_t)i * kp + t];
    const double g1 = (double)m1[i] * x - (double)P1[e];
    const double g2 = (double)m2[i] * x - (double)P2[e];
    grad[e] = (float)(g1 - g2);
}

hipError_t launch_grad_combine(const float *X, int n, int d, int kp, const float *P1,
                               const float *m1, const float *P2, const float *m2, float *grad,
                               hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_combine, dim3((unsigned)(((int64_t)n * d + 255) / 256)), dim3(256), 0,
                       s, X, n, d, kp, P1, m1, P2, m2, grad);
    return hipGetLastError();
}

// dS/d alpha_i from the dual vectors (envelope theorem on the dual of eq. (3) for
// the three OT terms of eq. (5); the mass terms cancel):
//   (rho + eps)(e^{-p_i/rho} - e^{-f_i/rho}) = -(rho + eps) e^{-p_i/rho} expm1(-(f_i - p_i)/rho),
// f_i - p_i when balanced (rho <= 0).  FP64 arithmetic, FP32 result; (g, q) give dS/d beta.
__global__ __launch_bounds__(256) void k_grad_weights(const float *__restrict__ f,
                                                      const float *__restrict__ p, int64_t n,
                                                      double eps, double rho,
                                                      float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double fi = f[i], pi = p[i];
    const double v = rho > 0.0 ? -(rho + eps) * exp(-pi / rho) * expm1(-(fi - pi) / rho) : fi - pi;
    out[i] = (float)v;
}

hipError_t launch_grad_weights(const float *f, const float *p, int64_t n, double eps, double rho,
                               float *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f, p, n,
                       eps, rho, out);
    return hipGetLastError();
}

// Label transfer (Section 3): the subject augmented with the mirror flips of its fibres
// (Section 2: tractograms are augmented with the flips of all fibres, the simplest
// encoding of unoriented curves).  Rows [0, n) copy x; row n + i is fibre i with its P
// points in reverse order (each point d / P coordinates); the weights are repeated.
__global__ __launch_bounds__(256) void k_flip_augment(const float *__restrict__ x,
                                                      const float *__restrict__ a, int64_t n,
                                                      int d, int P, float *__restrict__ xa,
                                                      float *__restrict__ aa) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * d) return;
    const int64_t i = e / d;
    const int t = (int)(e - i * d);
    const int D0 = d / P;
    const int pt = t / D0, c = t - pt * D0;
    const float v = x[e];
    xa[e] = v;
    xa[(n + i) * d + (int64_t)(P - 1 - pt) * D0 + c] = v;
    if (t == 0) {
        aa[i] = a[i];
        aa[n + i] = a[i];
    }
}

// One-hot atlas labels: V[j][l] = 1 if labels[j] == l (m x L, labels checked beforehand).
__global__ __launch_bounds__(256) void k_one_hot(const int *__restrict__ labels, int64_t m, int L,
                                                 float *__restrict__ V) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= m * L) return;
    const int64_t j = e / L;
    V[e] = labels[j] == (int)(e - j * L) ? 1.0f : 0.0f;
}

// Soft labels of eq. (7) per subject fibre: with flips the two versions add up (the plan
// keeps mass on the better-oriented one); score_i = sum_l Lab_il (FP64 sum), the fraction
// of the fibre's weight the plan transports (close to 0 for an outlier).
__global__ __launch_bounds__(256) void k_label_fold(const float *__restrict__ aug, int64_t n,
                                                    int L, int flips, float *__restrict__ lab,
                                                    float *__restrict__ score) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int l = 0; l < L; ++l) {
        float v = aug[i * L + l];
        if (flips) v += aug[(n + i) * L + l];
        if (lab) lab[i * L + l] = v;
        s += (double)v;
    }
    if (score) score[i] = (float)s;
}

hipError_t launch_flip_augment(const float *x, const float *a, int64_t n, int d, int P, float *xa,
                               float *aa, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_flip_augment, dim3((unsigned)((n * d + 255) / 256)), dim3(256), 0, s, x, a,
                       n, d, P, xa, aa);
    return hipGetLastError();
}

hipError_t launch_one_hot(const int *labels, int64_t m, int L, float *V, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_one_hot, dim3((unsigned)((m * L + 255) / 256)), dim3(256), 0, s, labels, m,
                       L, V);
    return hipGetLastError();
}

hipError_t launch_label_fold(const float *aug, int64_t n, int L, int flips, float *lab, float *score,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_label_fold, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, aug, n, L,
                       flips, lab, score);
    return hipGetLastError();
}

}  // namespace skh
