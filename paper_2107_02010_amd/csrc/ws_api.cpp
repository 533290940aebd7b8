// C ABI of the learned warm start (declared in include/skh.h): cluster tokens,
// network forward, loss gradient, Adam, training targets and the broadcast of
// predictions to starting dual vectors.  All arithmetic runs in the kernels of
// warmstart.hip and kmeans.hip; this file checks arguments, carves workspace
// and sequences launches on the context's stream.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_util.h"
#include "skh.h"
#include "skh_internal.h"

using namespace skh_host;

namespace {

constexpr int kW = skh::kWsWidth;
constexpr int kIn = skh::kWsIn;

struct NetPtrs {
    float *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4, *W5, *b5;
};

NetPtrs net_ptrs(float *t) {
    NetPtrs p;
    p.W1 = t;
    p.b1 = p.W1 + kW * kIn;
    p.W2 = p.b1 + kW;
    p.b2 = p.W2 + kW * kW;
    p.W3 = p.b2 + kW;
    p.b3 = p.W3 + kW * kW;
    p.W4 = p.b3 + kW;
    p.b4 = p.W4 + kW * 3 * kW;
    p.W5 = p.b4 + kW;
    p.b5 = p.W5 + 2 * kW;
    return p;
}

static_assert(kW * kIn + kW + 2 * (kW * kW + kW) + kW * 3 * kW + kW + 2 * kW + 2 == SKH_WS_N_PARAMS,
              "parameter count");

// Batch geometry checked on the host: seg (2P + 1 offsets) -> T.
int check_segments(skh_ctx *ctx, int32_t n_pairs, const int32_t *seg, int *T) {
    if (n_pairs < 1 || n_pairs > SKH_WS_MAX_PAIRS)
        return fail(ctx, SKH_EINVAL, "n_pairs must be in [1, SKH_WS_MAX_PAIRS]");
    if (!seg) return fail(ctx, SKH_EINVAL, "NULL seg");
    if (seg[0] != 0) return fail(ctx, SKH_EINVAL, "seg[0] must be 0");
    for (int s = 0; s < 2 * n_pairs; ++s)
        if (seg[s + 1] <= seg[s]) return fail(ctx, SKH_EINVAL, "every segment must be non-empty");
    *T = seg[2 * n_pairs];
    if (*T > (1 << 22)) return fail(ctx, SKH_EINVAL, "too many tokens");
    return SKH_OK;
}

// Device activations of one batch (workspace slot 2).
struct Acts {
    int *off = nullptr, *seg = nullptr;
    double *wsum = nullptr, *tl = nullptr, *loss = nullptr;
    float *a1 = nullptr, *a2 = nullptr, *h = nullptr, *a4 = nullptr;
    float *pooled = nullptr, *ctxv = nullptr, *share = nullptr, *lw = nullptr;
    float *dy = nullptr, *d1 = nullptr, *d2 = nullptr, *Dp = nullptr, *dP = nullptr, *part = nullptr;
};

int carve_acts(skh_ctx *ctx, int P, int T, bool train, Acts &A) {
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[2] : nullptr);
        A.off = c.take<int>(2 * P + 1);
        A.seg = c.take<int>(T);
        A.wsum = c.take<double>(2 * P);
        A.a1 = c.take<float>((size_t)T * kW);
        A.a2 = c.take<float>((size_t)T * kW);
        A.h = c.take<float>((size_t)T * kW);
        A.a4 = c.take<float>((size_t)T * kW);
        A.pooled = c.take<float>((size_t)2 * P * kW);
        A.ctxv = c.take<float>((size_t)P * kW);
        A.share = c.take<float>(T);
        A.lw = c.take<float>(T);
        if (train) {
            A.tl = c.take<double>(T);
            A.loss = c.take<double>(1);
            A.dy = c.take<float>((size_t)T * 2);
            A.d1 = c.take<float>((size_t)T * kW);
            A.d2 = c.take<float>((size_t)T * kW);
            A.Dp = c.take<float>((size_t)P * kW);
            A.dP = c.take<float>((size_t)2 * P * kW);
            A.part = c.take<float>(skh::colsum_part_len(3 * kW));
        }
        if (!pass) {
            int rc = ensure_ws(ctx, 2, c.off);
            if (rc) return rc;
        }
    }
    return SKH_OK;
}

skh::GemmArgs gemm(const float *A, int64_t a_m, int64_t a_k, const float *B, int64_t b_k,
                   int64_t b_n, float *C, int64_t ldc, int M, int N, int K) {
    skh::GemmArgs g{};
    g.A = A;
    g.a_m = a_m;
    g.a_k = a_k;
    g.B = B;
    g.b_k = b_k;
    g.b_n = b_n;
    g.C = C;
    g.ldc = ldc;
    g.M = M;
    g.N = N;
    g.K = K;
    g.grp_div = 1;
    return g;
}

// Uploads the segment offsets (through the pinned buffer; synchronises).
int upload_segments(skh_ctx *ctx, const int32_t *seg, int n_seg, int *dev) {
    const size_t bytes = (size_t)(n_seg + 1) * sizeof(int);
    if (bytes > kHostBytes) return fail(ctx, SKH_EINVAL, "too many segments");
    std::memcpy(ctx->host, seg, bytes);
    SKH_HIP(hipMemcpyAsync(dev, ctx->host, bytes, hipMemcpyHostToDevice, ctx->stream));
    SKH_HIP(hipStreamSynchronize(ctx->stream));
    return SKH_OK;
}

// Forward pass to a4 (and the token bookkeeping), weights W.
int forward_hidden(skh_ctx *ctx, const NetPtrs &W, int P, int T, const float *X, const float *w,
                   bool bf16, Acts &A) {
    hipStream_t s = ctx->stream;
    skh::GemmArgs g = gemm(X, kIn, 1, W.W1, 1, kIn, A.a1, kW, T, kW, kIn);
    g.bias = W.b1;
    g.relu = 1;
    SKH_HIP(skh::launch_gemm(g, bf16, s));
    g = gemm(A.a1, kW, 1, W.W2, 1, kW, A.a2, kW, T, kW, kW);
    g.bias = W.b2;
    g.relu = 1;
    SKH_HIP(skh::launch_gemm(g, bf16, s));
    g = gemm(A.a2, kW, 1, W.W3, 1, kW, A.h, kW, T, kW, kW);
    g.bias = W.b3;
    g.relu = 1;
    SKH_HIP(skh::launch_gemm(g, bf16, s));
    // pooled context of every cloud, then token bookkeeping
    SKH_HIP(skh::launch_segsum(A.h, A.off, 1, 2 * P, w, 1, A.pooled, A.wsum, s));
    SKH_HIP(skh::launch_token_index(A.off, 2 * P, w, A.wsum, T, A.seg, A.share, A.lw, s));
    // per-pair context: [P_alpha, P_beta] W4[:, 256:]^T + b4
    g = gemm(A.pooled, 2 * kW, 1, W.W4 + kW, 1, 3 * kW, A.ctxv, kW, P, kW, 2 * kW);
    g.bias = W.b4;
    SKH_HIP(skh::launch_gemm(g, bf16, s));
    // a4 = relu(h W4[:, :256]^T + context of the token's pair)
    g = gemm(A.h, kW, 1, W.W4, 1, 3 * kW, A.a4, kW, T, kW, kW);
    g.G = A.ctxv;
    g.ldg = kW;
    g.grp = A.seg;
    g.grp_div = 2;
    g.relu = 1;
    SKH_HIP(skh::launch_gemm(g, bf16, s));
    return SKH_OK;
}

// dW = dY^T X for dY (T x O, row stride ldy) and X (T x I, row stride ldx) into
// C (O x I, row stride ldc), and db = column sums of dY.
int weight_grad(skh_ctx *ctx, const float *dY, int64_t ldy, int O, const float *X, int64_t ldx, int I,
                int T, float *C, int64_t ldc, float *db, float *part) {
    hipStream_t s = ctx->stream;
    skh::GemmArgs g = gemm(dY, 1, ldy, X, ldx, 1, C, ldc, O, I, T);
    SKH_HIP(skh::launch_gemm(g, false, s));
    if (db) SKH_HIP(skh::launch_colsum(dY, T, O, ldy, part, db, s));
    return SKH_OK;
}

}  // namespace

extern "C" {

int skh_ws_forward(skh_ctx *ctx, const float *theta, int32_t n_pairs, const int32_t *seg,
                   const float *tokens, const float *tok_w, int32_t precision, float *out) {
    if (!ctx) return SKH_EINVAL;
    if (!theta || !tokens || !tok_w || !out) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (precision != SKH_FP32 && precision != SKH_BF16_SPLIT)
        return fail(ctx, SKH_EINVAL, "unknown precision");
    int T = 0;
    int rc = check_segments(ctx, n_pairs, seg, &T);
    if (rc) return rc;
    DeviceGuard guard(ctx->device);
    Acts A;
    rc = carve_acts(ctx, n_pairs, T, false, A);
    if (rc) return rc;
    rc = upload_segments(ctx, seg, 2 * n_pairs, A.off);
    if (rc) return rc;
    const NetPtrs W = net_ptrs(const_cast<float *>(theta));
    rc = forward_hidden(ctx, W, n_pairs, T, tokens, tok_w, precision == SKH_BF16_SPLIT, A);
    if (rc) return rc;
    SKH_HIP(skh::launch_head(A.a4, W.W5, W.b5, T, nullptr, nullptr, out, nullptr, nullptr,
                             ctx->stream));
    return SKH_OK;
}

int skh_ws_loss_grad(skh_ctx *ctx, const float *theta, int32_t n_pairs, const int32_t *seg,
                     const float *tokens, const float *tok_w, const float *target, double *loss,
                     float *grad) {
    if (!ctx) return SKH_EINVAL;
    if (!theta || !tokens || !tok_w || !target || !grad)
        return fail(ctx, SKH_EINVAL, "NULL argument");
    int T = 0;
    int rc = check_segments(ctx, n_pairs, seg, &T);
    if (rc) return rc;
    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    Acts A;
    rc = carve_acts(ctx, n_pairs, T, true, A);
    if (rc) return rc;
    rc = upload_segments(ctx, seg, 2 * n_pairs, A.off);
    if (rc) return rc;
    const int P = n_pairs;
    const NetPtrs W = net_ptrs(const_cast<float *>(theta));
    const NetPtrs G = net_ptrs(grad);
    rc = forward_hidden(ctx, W, P, T, tokens, tok_w, false, A);
    if (rc) return rc;
    // output layer, loss and dy
    SKH_HIP(skh::launch_head(A.a4, W.W5, W.b5, T, target, A.lw, nullptr, A.dy, A.tl, s));
    SKH_HIP(skh::launch_sum_f64(A.tl, T, A.loss, s));
    rc = weight_grad(ctx, A.dy, 2, 2, A.a4, kW, kW, T, G.W5, kW, G.b5, A.part);
    if (rc) return rc;
    // da4 -> d1
    SKH_HIP(skh::launch_head_bwd(A.dy, W.W5, A.a4, T, A.d1, s));
    // W4: token part from h, context part from the pooled vectors
    rc = weight_grad(ctx, A.d1, kW, kW, A.h, kW, kW, T, G.W4, 3 * kW, nullptr, A.part);
    if (rc) return rc;
    SKH_HIP(skh::launch_segsum(A.d1, A.off, 2, P, nullptr, 0, A.Dp, nullptr, s));
    rc = weight_grad(ctx, A.Dp, kW, kW, A.pooled, 2 * kW, 2 * kW, P, G.W4 + kW, 3 * kW, G.b4,
                     A.part);
    if (rc) return rc;
    // gradient of the pooled vectors: dP[pair] = Dp[pair] W4[:, 256:]  (P x 512 = 2P x 256)
    skh::GemmArgs g = gemm(A.Dp, kW, 1, W.W4 + kW, 3 * kW, 1, A.dP, 2 * kW, P, 2 * kW, kW);
    SKH_HIP(skh::launch_gemm(g, false, s));
    // dh3 = (da4 W4[:, :256] + share_t dP[seg_t]) [h > 0] -> d2
    g = gemm(A.d1, kW, 1, W.W4, 3 * kW, 1, A.d2, kW, T, kW, kW);
    g.G = A.dP;
    g.ldg = kW;
    g.grp = A.seg;
    g.grp_div = 1;
    g.rs = A.share;
    g.mask = A.h;
    g.ldm = kW;
    SKH_HIP(skh::launch_gemm(g, false, s));
    rc = weight_grad(ctx, A.d2, kW, kW, A.a2, kW, kW, T, G.W3, kW, G.b3, A.part);
    if (rc) return rc;
    // da2 = (dh3 W3) [a2 > 0] -> d1
    g = gemm(A.d2, kW, 1, W.W3, kW, 1, A.d1, kW, T, kW, kW);
    g.mask = A.a2;
    g.ldm = kW;
    SKH_HIP(skh::launch_gemm(g, false, s));
    rc = weight_grad(ctx, A.d1, kW, kW, A.a1, kW, kW, T, G.W2, kW, G.b2, A.part);
    if (rc) return rc;
    // da1 = (da2 W2) [a1 > 0] -> d2
    g = gemm(A.d1, kW, 1, W.W2, kW, 1, A.d2, kW, T, kW, kW);
    g.mask = A.a1;
    g.ldm = kW;
    SKH_HIP(skh::launch_gemm(g, false, s));
    rc = weight_grad(ctx, A.d2, kW, kW, tokens, kIn, kIn, T, G.W1, kIn, G.b1, A.part);
    if (rc) return rc;
    double *hl = static_cast<double *>(ctx->host);
    SKH_HIP(hipMemcpyAsync(hl, A.loss, sizeof(double), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipStreamSynchronize(s));
    if (loss) *loss = *hl;
    return SKH_OK;
}

int skh_ws_adam(skh_ctx *ctx, int64_t n, float *theta, const float *grad, float *m, float *v,
                int32_t step, double lr, double beta1, double beta2, double eps) {
    if (!ctx) return SKH_EINVAL;
    if (!theta || !grad || !m || !v) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || step < 1) return fail(ctx, SKH_EINVAL, "n and step must be >= 1");
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
        !(eps >= 0.0))
        return fail(ctx, SKH_EINVAL, "bad Adam hyper-parameter");
    DeviceGuard guard(ctx->device);
    SKH_HIP(skh::launch_adam(n, theta, grad, m, v, lr, beta1, beta2, step, eps, ctx->stream));
    return SKH_OK;
}

int skh_ws_tokens(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                  const float *b, int64_t m, int32_t d, int32_t n_clusters, int32_t kmeans_iters,
                  int32_t cap_tokens, float *tokens, float *tok_w, int32_t *labels_x,
                  int32_t *labels_y, int32_t *k_out) {
    if (!ctx) return SKH_EINVAL;
    if (!x || !a || !y || !b || !tokens || !tok_w || !labels_x || !labels_y || !k_out)
        return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || m < 1 || n > (1 << 28) || m > (1 << 28))
        return fail(ctx, SKH_EINVAL, "n and m must be in [1, 2^28]");
    if (d < 1 || d > kIn - 4) return fail(ctx, SKH_EINVAL, "tokens need 1 <= d <= 60");
    if (n_clusters < 0 || kmeans_iters < 0) return fail(ctx, SKH_EINVAL, "negative count");
    const int kx = n_clusters > 0 ? (int)std::min<int64_t>(std::min(n_clusters, 4096), n) : kmeans_k(n);
    const int ky = n_clusters > 0 ? (int)std::min<int64_t>(std::min(n_clusters, 4096), m) : kmeans_k(m);
    if (kx + ky > cap_tokens) return fail(ctx, SKH_EINVAL, "cap_tokens too small");
    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    const int kp = skh::packed_width(d);
    const int nbx = skh::bbox_blocks(n), nby = skh::bbox_blocks(m);
    float *Xp, *Yp, *hnx, *hny, *plo, *phi, *lohi, *Cx, *Cy, *cmx, *cmy, *rx, *ry;
    double *pmass, *mass;
    int *pbad, *bad, *kwx, *kwy;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[0] : nullptr);
        Xp = c.take<float>((size_t)n * kp);
        Yp = c.take<float>((size_t)m * kp);
        hnx = c.take<float>(n);
        hny = c.take<float>(m);
        plo = c.take<float>((size_t)(nbx + nby) * 64);
        phi = c.take<float>((size_t)(nbx + nby) * 64);
        pmass = c.take<double>(nbx + nby);
        pbad = c.take<int>(2 * (nbx + nby));
        lohi = c.take<float>(192);
        mass = c.take<double>(2);
        bad = c.take<int>(4);
        Cx = c.take<float>((size_t)kx * kp);
        Cy = c.take<float>((size_t)ky * kp);
        cmx = c.take<float>(kx);
        cmy = c.take<float>(ky);
        rx = c.take<float>(kx);
        ry = c.take<float>(ky);
        kwx = c.take<int>(skh::kmeans_workspace_ints((int)n, kx));
        kwy = c.take<int>(skh::kmeans_workspace_ints((int)m, ky));
        if (!pass) {
            int rc = ensure_ws(ctx, 0, c.off);
            if (rc) return rc;
        }
    }
    // joint bounding box: validation, centre and diagonal (as the solver)
    SKH_HIP(skh::launch_bbox_partial(x, a, n, d, plo, phi, pmass, pbad, s));
    SKH_HIP(skh::launch_bbox_partial(y, b, m, d, plo + (size_t)nbx * 64, phi + (size_t)nbx * 64,
                                     pmass + nbx, pbad + 2 * nbx, s));
    SKH_HIP(skh::launch_bbox_final(plo, phi, pmass, pbad, nbx, nby, d, lohi, mass, bad, s));
    char *hb = static_cast<char *>(ctx->host);
    SKH_HIP(hipMemcpyAsync(hb, lohi, 128 * sizeof(float), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipMemcpyAsync(hb + 512, mass, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipMemcpyAsync(hb + 528, bad, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipStreamSynchronize(s));
    const float *hlo = reinterpret_cast<const float *>(hb);
    const double *hmass = reinterpret_cast<const double *>(hb + 512);
    const int *hbad = reinterpret_cast<const int *>(hb + 528);
    if (hbad[1] || hbad[3]) return fail(ctx, SKH_EINVAL, "negative, NaN or infinite weight");
    if (hbad[0] || hbad[2]) return fail(ctx, SKH_ENONFINITE, "non-finite coordinate");
    if (!(hmass[0] > 0.0) || !(hmass[1] > 0.0))
        return fail(ctx, SKH_EINVAL, "total weight must be positive");
    double s2 = 0.0;
    for (int k = 0; k < d; ++k) {
        const double t = (double)hlo[64 + k] - (double)hlo[k];
        s2 += t * t;
    }
    const double diam = s2 > 0.0 ? std::sqrt(s2) : 1.0;
    const double Mx = hmass[0], My = hmass[1];
    SKH_HIP(skh::launch_pack(x, a, n, d, kp, lohi + 128, Xp, hnx, nullptr, s));
    SKH_HIP(skh::launch_pack(y, b, m, d, kp, lohi + 128, Yp, hny, nullptr, s));
    int *px, *ox, *py, *oy;
    SKH_HIP(skh::run_kmeans(Xp, a, (int)n, kp, kx, kmeans_iters, Cx, cmx, rx, kwx, &px, &ox, s));
    SKH_HIP(skh::run_kmeans(Yp, b, (int)m, kp, ky, kmeans_iters, Cy, cmy, ry, kwy, &py, &oy, s));
    SKH_HIP(skh::launch_tokens(Cx, cmx, rx, kx, kp, d, Mx, diam, 0, tokens, tok_w, s));
    SKH_HIP(skh::launch_tokens(Cy, cmy, ry, ky, kp, d, My, diam, 1, tokens + (size_t)kx * kIn,
                               tok_w + kx, s));
    SKH_HIP(skh::launch_labels_from_perm(px, ox, kx, labels_x, s));
    SKH_HIP(skh::launch_labels_from_perm(py, oy, ky, labels_y, s));
    SKH_HIP(hipStreamSynchronize(s));
    k_out[0] = kx;
    k_out[1] = ky;
    return SKH_OK;
}

int skh_ws_targets(skh_ctx *ctx, const int32_t *labels, int64_t n, int32_t k, const float *w,
                   const float *pot_cross, const float *pot_self, double scale, float *out) {
    if (!ctx) return SKH_EINVAL;
    if (!labels || !w || !pot_cross || !pot_self || !out) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || n > (1 << 28) || k < 1 || k > 4096) return fail(ctx, SKH_EINVAL, "bad n or k");
    if (!std::isfinite(scale)) return fail(ctx, SKH_EINVAL, "scale must be finite");
    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    int *kws, *bad;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[0] : nullptr);
        kws = c.take<int>(skh::kmeans_workspace_ints((int)n, k));
        bad = c.take<int>(1);
        if (!pass) {
            int rc = ensure_ws(ctx, 0, c.off);
            if (rc) return rc;
        }
    }
    SKH_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    SKH_HIP(skh::launch_check_labels(labels, (int)n, k, bad, s));
    int *hb = static_cast<int *>(ctx->host);
    SKH_HIP(hipMemcpyAsync(hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipStreamSynchronize(s));
    if (*hb) return fail(ctx, SKH_EINVAL, "label out of [0, k)");
    SKH_HIP(hipMemcpyAsync(kws, labels, n * sizeof(int), hipMemcpyDeviceToDevice, s));
    int *perm, *off;
    SKH_HIP(skh::sort_labels((int)n, k, kws, &perm, &off, s));
    SKH_HIP(skh::launch_cluster_means(perm, off, w, pot_cross, pot_self, k, scale, out, s));
    return SKH_OK;
}

int skh_ws_expand(skh_ctx *ctx, const int32_t *labels, int64_t n, int32_t k, const float *pred,
                  double scale, float *pot_cross, float *pot_self) {
    if (!ctx) return SKH_EINVAL;
    if (!labels || !pred || !pot_cross || !pot_self) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || n > (1 << 28) || k < 1 || k > 4096) return fail(ctx, SKH_EINVAL, "bad n or k");
    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    int *bad;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[0] : nullptr);
        bad = c.take<int>(1);
        if (!pass) {
            int rc = ensure_ws(ctx, 0, c.off);
            if (rc) return rc;
        }
    }
    // an out-of-range label or a non-finite prediction yields NaN starting
    // values, which the checked warm start of the solver turns into a cold start
    SKH_HIP(skh::launch_expand(labels, n, pred, k, scale, pot_cross, pot_self, bad, s));
    return SKH_OK;
}

}  // extern "C"
