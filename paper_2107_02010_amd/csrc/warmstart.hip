// Kernels of the learned warm start: a permutation-equivariant set encoder that
// maps the K-means clusters of the two clouds (the coarse scale of the
// coarse-to-fine strategy, Section 2) to the dual values of each cluster, so the
// Algorithm's loop can start near its fixed point instead of at the largest
// scale.  The network is an addition to the method; the Algorithm still decides
// the fixed point.
//
// Network (weights row-major, out x in, one flat FP32 vector):
//   h   = relu(relu(relu(X W1^T + b1) W2^T + b2) W3^T + b3)      tokens x 256
//   P_s = sum_{t in s} w_t h_t / sum_{t in s} w_t                 per segment s
//   a4  = relu(h W4[:, :256]^T + P_alpha W4[:, 256:512]^T
//               + P_beta W4[:, 512:]^T + b4)                      tokens x 256
//   y   = a4 W5^T + b5                                            tokens x 2
// A batch holds several cloud pairs; pair p owns segments 2p (alpha tokens) and
// 2p + 1 (beta tokens), contiguous in token order.
//
// Dense layers run on the matrix cores: one strided GEMM kernel (64 x 64 output
// tile per workgroup, four waves of 32 x 32, K staged through LDS in steps of
// 16) serves the forward products and both backward products (dX = dY W and
// dW = dY^T X) through its strides.  FP32 operands use v_mfma_f32_32x32x2f32
// (training); the BF16 variant rounds the staged operands to bfloat16 and uses
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation (inference).  Every sum over
// tokens is a fixed-order loop or a two-stage reduction: results do not depend
// on scheduling.
#include <algorithm>
#include <cmath>

#include "skh_internal.h"

namespace skh {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {
constexpr int kTile = 64;
constexpr int kKs = 16;
constexpr int kPad = kTile + 4;
}  // namespace

// C[m, n] = epilogue(sum_k A(m, k) B(k, n)), A(m, k) = A[m a_m + k a_k],
// B(k, n) = B[k b_k + n b_n].  Epilogue, in order: + bias[n];
// + rs[m] G[grp[m] / grp_div, n] (rs NULL: 1); relu; zero where mask[m, n] <= 0.
template <bool BF16>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ float As[kKs][kPad];  // [k][m]
    __shared__ float Bs[kKs][kPad];  // [k][n]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int li = lane & 31, hk = lane >> 5;
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const bool a_kfast = g.a_k == 1, b_nfast = g.b_n == 1;
    v16f acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += kKs) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + 256 * j;
            const int am = a_kfast ? (e >> 4) : (e & 63), ak = a_kfast ? (e & 15) : (e >> 6);
            const int gm = m0 + am, gk = k0 + ak;
            As[ak][am] = (gm < g.M && gk < g.K) ? g.A[(int64_t)gm * g.a_m + (int64_t)gk * g.a_k] : 0.f;
            const int bn = b_nfast ? (e & 63) : (e >> 4), bk = b_nfast ? (e >> 6) : (e & 15);
            const int gn = n0 + bn, gkb = k0 + bk;
            Bs[bk][bn] = (gn < g.N && gkb < g.K) ? g.B[(int64_t)gkb * g.b_k + (int64_t)gn * g.b_n] : 0.f;
        }
        __syncthreads();
        if constexpr (!BF16) {
#pragma unroll
            for (int s = 0; s < kKs / 2; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[2 * s + hk][wm * 32 + li],
                                                           Bs[2 * s + hk][wn * 32 + li], acc, 0, 0, 0);
        } else {
            bf16x8 a, b;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                a[t] = (__bf16)As[8 * hk + t][wm * 32 + li];
                b[t] = (__bf16)Bs[8 * hk + t][wn * 32 + li];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int n = n0 + wn * 32 + li;
    if (n >= g.N) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 32 + 8 * (r >> 2) + 4 * hk + (r & 3);
        if (m >= g.M) continue;
        float v = acc[r];
        if (g.bias) v += g.bias[n];
        if (g.G) {
            const float t = g.G[(int64_t)(g.grp[m] / g.grp_div) * g.ldg + n];
            v += g.rs ? g.rs[m] * t : t;
        }
        if (g.relu) v = fmaxf(v, 0.f);
        if (g.mask && !(g.mask[(int64_t)m * g.ldm + n] > 0.f)) v = 0.f;
        g.C[(int64_t)m * g.ldc + n] = v;
    }
}

hipError_t launch_gemm(const GemmArgs &g, bool bf16, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const dim3 grid((g.N + kTile - 1) / kTile, (g.M + kTile - 1) / kTile);
    if (bf16)
        hipLaunchKernelGGL(k_gemm<true>, grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL(k_gemm<false>, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// Column sums of an M x N row-major matrix (stride ld), two stages: chunk c of
// rows sums into part[c * N + n], then out[n] = sum over chunks in order.
constexpr int kColChunks = 64;

__global__ __launch_bounds__(256) void k_colsum_part(const float *__restrict__ A, int M, int N,
                                                     int64_t ld, float *__restrict__ part) {
    const int n = blockIdx.x * 64 + (threadIdx.x & 63);
    const int rg = threadIdx.x >> 6;  // 4 row groups
    const int c = blockIdx.y;
    const int rows = (M + kColChunks - 1) / kColChunks;
    const int mb = c * rows, me = min(M, mb + rows);
    __shared__ float sh[4][64];
    float s = 0.f;
    if (n < N)
        for (int m = mb + rg; m < me; m += 4) s += A[(int64_t)m * ld + n];
    sh[rg][threadIdx.x & 63] = s;
    __syncthreads();
    if (rg == 0 && n < N)
        part[(int64_t)c * N + n] = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) +
                                   (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_colsum_final(const float *__restrict__ part, int N,
                                                      float *__restrict__ out) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int c = 0; c < kColChunks; ++c) s += part[(int64_t)c * N + n];
    out[n] = s;
}

size_t colsum_part_len(int N) { return (size_t)kColChunks * N; }

hipError_t launch_colsum(const float *A, int M, int N, int64_t ld, float *part, float *out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, kColChunks), dim3(256), 0, s, A, M, N, ld,
                       part);
    hipLaunchKernelGGL(k_colsum_final, dim3((N + 255) / 256), dim3(256), 0, s, part, N, out);
    return hipGetLastError();
}

// Segment sums of the 256-wide rows of X: segment s covers tokens
// [off[s * stride], off[(s + 1) * stride]).  With w: weighted by w_t and, when
// normalise, divided by the segment's weight (wsum[s] receives that weight).
// Block (s, q) handles features 64 q .. 64 q + 63 with four row groups.
__global__ __launch_bounds__(256) void k_segsum(const float *__restrict__ X, const int *__restrict__ off,
                                                int stride, const float *__restrict__ w, int normalise,
                                                float *__restrict__ out, double *__restrict__ wsum) {
    const int sg = blockIdx.x, q = blockIdx.y;
    const int f = q * 64 + (threadIdx.x & 63), rg = threadIdx.x >> 6;
    const int tb = off[sg * stride], te = off[(sg + 1) * stride];
    float s = 0.f;
    for (int t = tb + rg; t < te; t += 4) {
        const float v = X[(int64_t)t * kWsWidth + f];
        s = w ? fmaf(w[t], v, s) : s + v;
    }
    __shared__ float sh[4][64];
    sh[rg][threadIdx.x & 63] = s;
    __syncthreads();
    if (rg != 0) return;
    float tot = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
    if (w && normalise) {
        double W = 0.0;
        for (int t = tb; t < te; ++t) W += (double)w[t];
        tot = W > 0.0 ? (float)((double)tot / W) : 0.f;
        if (q == 0 && threadIdx.x == 0 && wsum) wsum[sg] = W;
    }
    out[(int64_t)sg * kWsWidth + f] = tot;
}

hipError_t launch_segsum(const float *X, const int *off, int stride, int n_seg, const float *w,
                         int normalise, float *out, double *wsum, hipStream_t s) {
    if (n_seg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_segsum, dim3(n_seg, kWsWidth / 64), dim3(256), 0, s, X, off, stride, w,
                       normalise, out, wsum);
    return hipGetLastError();
}

// Per token: its segment index, the pooling share w_t / W_seg and the loss
// weight w_t / (W_alpha + W_beta of its pair) / n_pairs.
__global__ __launch_bounds__(256) void k_token_index(const int *__restrict__ off, int n_seg,
                                                     const float *__restrict__ w,
                                                     const double *__restrict__ wsum, int T,
                                                     int *__restrict__ seg, float *__restrict__ share,
                                                     float *__restrict__ lw) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= T) return;
    int lo = 0, hi = n_seg - 1;  // last segment with off[s] <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    seg[t] = lo;
    const double W = wsum[lo];
    share[t] = W > 0.0 ? (float)((double)w[t] / W) : 0.f;
    const int p = lo >> 1;
    const double Wp = wsum[2 * p] + wsum[2 * p + 1];
    const int n_pairs = n_seg >> 1;
    if (lw) lw[t] = Wp > 0.0 ? (float)((double)w[t] / Wp / n_pairs) : 0.f;
}

hipError_t launch_token_index(const int *off, int n_seg, const float *w, const double *wsum, int T,
                              int *seg, float *share, float *lw, hipStream_t s) {
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_token_index, dim3((T + 255) / 256), dim3(256), 0, s, off, n_seg, w, wsum,
                       T, seg, share, lw);
    return hipGetLastError();
}

// Output layer, one wave per token: y_t = a4_t W5^T + b5.  With a target:
// r = y - target, dy_t = 2 lw_t r and the token's loss lw_t |r|^2 (FP64).
__global__ __launch_bounds__(256) void k_head(const float *__restrict__ a4, const float *__restrict__ W5,
                                              const float *__restrict__ b5, int T,
                                              const float *__restrict__ target,
                                              const float *__restrict__ lw, float *__restrict__ y,
                                              float *__restrict__ dy, double *__restrict__ tl) {
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= T) return;
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int i = 0; i < kWsWidth / 64; ++i) {
        const int f = lane + 64 * i;
        const float v = a4[(int64_t)t * kWsWidth + f];
        s0 = fmaf(v, W5[f], s0);
        s1 = fmaf(v, W5[kWsWidth + f], s1);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
    }
    if (lane != 0) return;
    const float y0 = s0 + b5[0], y1 = s1 + b5[1];
    if (y) {
        y[2 * t] = y0;
        y[2 * t + 1] = y1;
    }
    if (target) {
        const float r0 = y0 - target[2 * t], r1 = y1 - target[2 * t + 1];
        const float l = lw[t];
        dy[2 * t] = 2.f * l * r0;
        dy[2 * t + 1] = 2.f * l * r1;
        tl[t] = (double)l * ((double)r0 * r0 + (double)r1 * r1);
    }
}

hipError_t launch_head(const float *a4, const float *W5, const float *b5, int T, const float *target,
                       const float *lw, float *y, float *dy, double *tl, hipStream_t s) {
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_head, dim3((T + 3) / 4), dim3(256), 0, s, a4, W5, b5, T, target, lw, y, dy,
                       tl);
    return hipGetLastError();
}

// da4[t, f] = (dy_t0 W5[0, f] + dy_t1 W5[1, f]) [a4[t, f] > 0]
__global__ __launch_bounds__(256) void k_head_bwd(const float *__restrict__ dy,
                                                  const float *__restrict__ W5,
                                                  const float *__restrict__ a4, int T,
                                                  float *__restrict__ da4) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)T * kWsWidth) return;
    const int t = (int)(e / kWsWidth), f = (int)(e % kWsWidth);
    const float v = fmaf(dy[2 * t], W5[f], dy[2 * t + 1] * W5[kWsWidth + f]);
    da4[e] = a4[e] > 0.f ? v : 0.f;
}

hipError_t launch_head_bwd(const float *dy, const float *W5, const float *a4, int T, float *da4,
                           hipStream_t s) {
    const int64_t n = (int64_t)T * kWsWidth;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_head_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dy, W5, a4, T,
                       da4);
    return hipGetLastError();
}

// Deterministic FP64 sum of n values: one block, fixed strided order.
__global__ __launch_bounds__(256) void k_sum_f64(const double *__restrict__ v, int n,
                                                 double *__restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += v[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

hipError_t launch_sum_f64(const double *v, int n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, s, v, n, out);
    return hipGetLastError();
}

// Adam with bias correction (Kingma & Ba): c1 = 1 - beta1^step, c2 = 1 - beta2^step.
__global__ __launch_bounds__(256) void k_adam(int64_t n, float *__restrict__ theta,
                                              const float *__restrict__ grad, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float b1, float b2,
                                              float c1, float c2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(int64_t n, float *theta, const float *grad, float *m, float *v, double lr,
                       double b1, double b2, int step, double eps, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // the hyper-parameters are rounded to FP32 once; the bias corrections use those values
    const float b1f = (float)b1, b2f = (float)b2;
    const double c1 = 1.0 - std::pow((double)b1f, (double)step);
    const double c2 = 1.0 - std::pow((double)b2f, (double)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, theta, grad, m,
                       v, (float)lr, b1f, b2f, (float)c1, (float)c2, (float)eps);
    return hipGetLastError();
}

// Tokens of one clustered cloud (centres C: k x kp in centred coordinates):
//   [C_c / scale (d values, zero up to 60), log(k m_c / M), r_c / scale,
//    side == 0, side == 1],  token weight m_c.
// A massless cluster gets log-mass -30 and weight 0.
__global__ __launch_bounds__(256) void k_tokens(const float *__restrict__ C, const float *__restrict__ cm,
                                                const float *__restrict__ rad, int k, int kp, int d,
                                                double total, double inv_scale, int side,
                                                float *__restrict__ tok, float *__restrict__ tw) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)k * kWsIn) return;
    const int c = (int)(e / kWsIn), f = (int)(e % kWsIn);
    float v = 0.f;
    if (f < d) {
        v = (float)((double)C[(size_t)c * kp + f] * inv_scale);
    } else if (f == kWsIn - 4) {
        const double mc = cm[c];
        v = mc > 0.0 && total > 0.0 ? (float)std::log((double)k * mc / total) : -30.f;
    } else if (f == kWsIn - 3) {
        v = (float)((double)rad[c] * inv_scale);
    } else if (f == kWsIn - 2) {
        v = side == 0 ? 1.f : 0.f;
    } else if (f == kWsIn - 1) {
        v = side == 1 ? 1.f : 0.f;
    }
    tok[e] = v;
    if (f == 0) tw[c] = cm[c];
}

hipError_t launch_tokens(const float *C, const float *cm, const float *rad, int k, int kp, int d,
                         double total, double scale, int side, float *tok, float *tw, hipStream_t s) {
    const int64_t n = (int64_t)k * kWsIn;
    hipLaunchKernelGGL(k_tokens, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, cm, rad, k, kp,
                       d, total, 1.0 / scale, side, tok, tw);
    return hipGetLastError();
}

// Cluster-mean targets: out[c, j] = scale * sum_{i in c} w_i pot_j[i] / sum_{i in c} w_i
// over the points of cluster c (sorted order perm[off[c] .. off[c+1])), FP64
// sums in point order; zero for a massless cluster.
__global__ __launch_bounds__(256) void k_cluster_means(const int *__restrict__ perm,
                                                       const int *__restrict__ off,
                                                       const float *__restrict__ w,
                                                       const float *__restrict__ p0,
                                                       const float *__restrict__ p1, int k,
                                                       double scale, float *__restrict__ out) {
    const int c = blockIdx.x;
    __shared__ double sh[3][256];
    double sw = 0.0, s0 = 0.0, s1 = 0.0;
    for (int i = off[c] + threadIdx.x; i < off[c + 1]; i += 256) {
        const int pt = perm[i];
        const double wi = w[pt];
        if (wi > 0.0) {
            sw += wi;
            s0 += wi * (double)p0[pt];
            s1 += wi * (double)p1[pt];
        }
    }
    sh[0][threadIdx.x] = sw;
    sh[1][threadIdx.x] = s0;
    sh[2][threadIdx.x] = s1;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double W = sh[0][0];
        out[2 * c] = W > 0.0 ? (float)(scale * sh[1][0] / W) : 0.f;
        out[2 * c + 1] = W > 0.0 ? (float)(scale * sh[2][0] / W) : 0.f;
    }
}

hipError_t launch_cluster_means(const int *perm, const int *off, const float *w, const float *p0,
                                const float *p1, int k, double scale, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_cluster_means, dim3(k), dim3(256), 0, s, perm, off, w, p0, p1, k, scale,
                       out);
    return hipGetLastError();
}

// Broadcast of per-cluster predictions to the points: pot_j[i] = scale pred[lab_i, j].
__global__ __launch_bounds__(256) void k_expand(const int *__restrict__ lab, int64_t n,
                                                const float *__restrict__ pred, int k, double scale,
                                                float *__restrict__ p0, float *__restrict__ p1,
                                                int *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = lab[i];
    float v0 = __builtin_nanf(""), v1 = v0;
    if (c >= 0 && c < k) {
        v0 = (float)(scale * (double)pred[2 * c]);
        v1 = (float)(scale * (double)pred[2 * c + 1]);
    }
    p0[i] = v0;
    p1[i] = v1;
    if (!isfinite(v0) || !isfinite(v1)) atomicOr(bad, 1);
}

hipError_t launch_expand(const int *lab, int64_t n, const float *pred, int k, double scale, float *p0,
                         float *p1, int *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_expand, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, lab, n, pred, k,
                       scale, p0, p1, bad);
    return hipGetLastError();
}

// Labels in point order from the cluster-sorted permutation.
__global__ __launch_bounds__(256) void k_labels_from_perm(const int *__restrict__ perm,
                                                          const int *__restrict__ off, int k,
                                                          int *__restrict__ lab) {
    const int c = blockIdx.x;
    for (int i = off[c] + threadIdx.x; i < off[c + 1]; i += 256) lab[perm[i]] = c;
}

hipError_t launch_labels_from_perm(const int *perm, const int *off, int k, int *lab, hipStream_t s) {
    hipLaunchKernelGGL(k_labels_from_perm, dim3(k), dim3(256), 0, s, perm, off, k, lab);
    return hipGetLastError();
}

// Non-finite check of starting potentials: sets *bad when any value is NaN or infinite.
__global__ __launch_bounds__(256) void k_nonfinite(const float *__restrict__ v, int64_t n,
                                                   int *__restrict__ bad) {
    int b = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        b |= !isfinite(v[i]);
    if (__any(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

hipError_t launch_nonfinite(const float *v, int64_t n, int *bad, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)blocks), dim3(256), 0, s, v, n, bad);
    return hipGetLastError();
}

}  // namespace skh
