// Host driver and C ABI of libskh (declared in include/skh.h).
//
// The driver runs the symmetric, averaged Sinkhorn loop with eps-scaling
// (Algorithm) on one device stream: per iteration one softmin launch covering
// the four problems (alpha<->alpha, beta<->beta, alpha->beta, beta->alpha)
// and one O(n + m) launch that merges, averages and prepares the next column
// offsets.  The host synchronises only for the bounding box (scale list and
// validation), for the periodic marginal-error check in converged mode, and
// for the final FP64 value of eq. (6).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "skh.h"
#include "skh_internal.h"
#include "host_util.h"

thread_local std::string g_create_err;

// Device scratch of the allocation-free softmin entry (skh_softmin_noalloc): a fixed
// array in the code object, so that entry never allocates.  Each device holds its own
// copy from module load until the process ends.  In host code the name `scratch` is a
// host-side stand-in, not a device address: host code uses only the address
// hipGetSymbolAddress returns on each device (scratch_address), never the name.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// The scratch array's address on `device`, looked up once per device (with that
// device current) and kept for every later context of the device.
int scratch_address(int device, void **out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return SKH_EHIP;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SKH_EHIP;
        }
        addr[device] = p;
    }
    *out = addr[device];
    return SKH_OK;
}

}  // namespace

namespace {
using namespace skh_host;

struct Clustered {
    int n = 0, k = 0, n_pad_max = 0, n_pad = 0, max_tiles = 0, n_tiles = 0;
    float *C = nullptr, *cmass = nullptr, *radius = nullptr;  // k x kp, k, k
    float *hnC = nullptr, *lwC = nullptr;                     // coarse measure: k, k
    int *kws = nullptr;                                       // K-means workspace
    int *psize = nullptr, *poff = nullptr, *ssum = nullptr;   // k + 1, k + 1, scan sums
    int *tcnt = nullptr, *toff = nullptr;                     // k + 1 each (row tiles)
    int4 *tiles = nullptr;                                    // max_tiles
    int *perm_pad = nullptr, *blk = nullptr;                  // n_pad_max, n_pad_max / 32
    float *Xf = nullptr;                                      // n_pad_max x kp
    __hip_bfloat16 *Yhi[2] = {nullptr, nullptr};              // n_pad_max x kp, per problem
    __hip_bfloat16 *Ylo = nullptr;                            // n_pad_max x kp
    float *blkcent = nullptr;                                 // (n_pad_max / 32) x kp
    float *hn = nullptr, *lw = nullptr, *wp = nullptr;        // n_pad_max
    int *perm = nullptr, *off = nullptr;                      // inside kws, set by K-means
    std::vector<int> h_poff;                                  // host copies
    std::vector<float> h_mass, h_rad;

    void carve(Carver &c, int n_, int kp, int k_req) {
        n = n_;
        k = k_req > 0 ? std::min(std::min(k_req, n_), 4096) : kmeans_k(n_);
        n_pad_max = n_ + 31 * k;
        max_tiles = n_pad_max / kRowTile + k + 1;
        C = c.take<float>((size_t)k * kp);
        cmass = c.take<float>(k);
        radius = c.take<float>(k);
        hnC = c.take<float>(k);
        lwC = c.take<float>(k);
        kws = c.take<int>(skh::kmeans_workspace_ints(n_, k));
        psize = c.take<int>(k + 1);
        poff = c.take<int>(k + 1);
        ssum = c.take<int>(skh::scan_sums_len(k + 1));
        tcnt = c.take<int>(k + 1);
        toff = c.take<int>(k + 1);
        tiles = c.take<int4>(max_tiles);
        perm_pad = c.take<int>(n_pad_max);
        blk = c.take<int>(n_pad_max / 32 + 1);
        Xf = c.take<float>((size_t)n_pad_max * kp);
        Yhi[0] = c.take<__hip_bfloat16>((size_t)n_pad_max * kp);
        Yhi[1] = c.take<__hip_bfloat16>((size_t)n_pad_max * kp);
        Ylo = c.take<__hip_bfloat16>((size_t)n_pad_max * kp);
        blkcent = c.take<float>((size_t)(n_pad_max / 32 + 1) * kp);
        hn = c.take<float>(n_pad_max);
        lw = c.take<float>(n_pad_max);
        wp = c.take<float>(n_pad_max);
    }
};

// K-means of a packed cloud and the padded cluster sizes (poff[k] = n_pad).
int cluster_start(skh_ctx *ctx, Clustered &cl, const float *X, const float *w, int kp, int iters,
                  hipStream_t s, const int *labels = nullptr) {
    if (labels)
        SKH_HIP(skh::clusters_from_labels(X, w, cl.n, kp, cl.k, labels, cl.C, cl.cmass, cl.radius,
                                          cl.kws, &cl.perm, &cl.off, s));
    else
        SKH_HIP(skh::run_kmeans(X, w, cl.n, kp, cl.k, iters, cl.C, cl.cmass, cl.radius, cl.kws,
                                &cl.perm, &cl.off, s));
    SKH_HIP(skh::build_padded_layout(cl.perm, cl.off, cl.k, cl.psize, cl.poff, cl.ssum, s));
    return SKH_OK;
}

// Gathers the cloud into the padded order once cl.n_pad is known on the host.
int cluster_finish(skh_ctx *ctx, Clustered &cl, const float *X, const float *w, int kp,
                   hipStream_t s) {
    if (cl.n_pad < cl.n || cl.n_pad > cl.n_pad_max)
        return fail(ctx, SKH_EHIP, "inconsistent padded cluster layout");
    SKH_HIP(skh::fill_padded_layout(cl.perm, cl.off, cl.poff, cl.k, cl.perm_pad, cl.blk, s));
    SKH_HIP(skh::launch_pack_padded(X, w, cl.perm_pad, cl.blk, cl.C, cl.n_pad, kp, cl.Xf,
                                    cl.Yhi[0], cl.Yhi[1], cl.Ylo, cl.hn, cl.lw, cl.wp, s));
    SKH_HIP(skh::launch_blk_centroids(cl.blk, cl.C, cl.n_pad / 32, kp, cl.blkcent, s));
    return SKH_OK;
}

}  // namespace

extern "C" {

void skh_params_default(skh_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->blur = 0.05;
    p->cost_p = 2.0;
    p->reach = INFINITY;
    p->scaling = 0.9;
    p->diameter = 0.0;
    p->tol = 0.0;
    p->extra_iters = 0;
    p->max_iters = 1000;
    p->check_every = 5;
    p->precision = SKH_FP32;
    p->init = 0;
    p->timing = 0;
    p->multiscale = 0;
    p->jump_scale = 0.0;
    p->trunc_theta = 20.0;
    p->start_scale = 0.0;
    p->n_clusters = 0;
    p->kmeans_iters = kKmeansIters;
}

int skh_create(skh_ctx **out, int device, void *hip_stream) {
    if (!out) {
        g_create_err = "out is NULL";
        return SKH_EINVAL;
    }
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        g_create_err = "invalid HIP device " + std::to_string(device);
        return SKH_EHIP;
    }
    DeviceGuard guard(device);
    skh_ctx *ctx = new skh_ctx();
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cus = prop.multiProcessorCount;
    if (hipHostMalloc(&ctx->host, kHostBytes, hipHostMallocDefault) != hipSuccess) {
        g_create_err = "pinned host allocation failed";
        delete ctx;
        return SKH_EHIP;
    }
    if (scratch_address(device, &ctx->scratch) != SKH_OK) {
        g_create_err = "hipGetSymbolAddress of the device scratch array failed";
        (void)hipHostFree(ctx->host);
        delete ctx;
        return SKH_EHIP;
    }
    *out = ctx;
    return SKH_OK;
}

void skh_destroy(skh_ctx *ctx) {
    if (!ctx) return;
    {
        DeviceGuard guard(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (int k = 0; k < 4; ++k)
            if (ctx->ws[k]) (void)hipFree(ctx->ws[k]);
        if (ctx->host) (void)hipHostFree(ctx->host);
        for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    }
    delete ctx;
}

int skh_set_stream(skh_ctx *ctx, void *hip_stream) {
    if (!ctx) return SKH_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return SKH_OK;
}

const char *skh_last_error(const skh_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int skh_set_workspace_limit(skh_ctx *ctx, size_t bytes) {
    if (!ctx) return SKH_EINVAL;
    ctx->ws_limit = bytes;
    if (bytes && ws_total(ctx) > bytes) {  // release what the new limit does not cover
        DeviceGuard guard(ctx->device);
        SKH_HIP(hipStreamSynchronize(ctx->stream));
        for (int k = 0; k < 4; ++k) {
            if (ctx->ws[k]) SKH_HIP(hipFree(ctx->ws[k]));
            ctx->ws[k] = nullptr;
            ctx->ws_bytes[k] = 0;
        }
    }
    return SKH_OK;
}

int skh_workspace_bytes(const skh_ctx *ctx, size_t *out) {
    if (!ctx || !out) return SKH_EINVAL;
    *out = ws_total(ctx);
    return SKH_OK;
}

}  // extern "C"

namespace {

// Where one call of the softmin entry takes its device workspace: the context's
// growing workspace (slot by slot), or consecutive pieces of the fixed scratch array
// (the allocation-free entry, which must not allocate).
struct SoftminRegions {
    skh_ctx *ctx;
    bool fixed;
    size_t used = 0;
    int get(int slot, size_t bytes, void **out) {
        if (!fixed) {
            const int rc = ensure_ws(ctx, slot, bytes);
            if (rc) return rc;
            *out = ctx->ws[slot];
            return SKH_OK;
        }
        const size_t off = (used + 255) & ~size_t(255);
        if (!ctx->scratch || off + bytes > kScratchBytes)
            return fail(ctx, SKH_EINVAL, "internal: scratch region out of range");
        *out = static_cast<char *>(ctx->scratch) + off;
        used = off + bytes;
        return SKH_OK;
    }
};

int softmin_impl(skh_ctx *ctx, const float *x, int64_t n, const float *y, int64_t m, int32_t d,
                 const float *w, const float *h, double eps, double lam, int32_t precision,
                 float *out, bool no_alloc) {
    if (!ctx) return SKH_EINVAL;
    if (!x || !y || !w || !h || !out) return fail(ctx, SKH_EINVAL, "NULL array argument");
    if (n < 1 || m < 1) return fail(ctx, SKH_EINVAL, "n and m must be >= 1");
    if (n > kMaxPoints || m > kMaxPoints) return fail(ctx, SKH_EINVAL, "n or m too large");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ctx, SKH_EINVAL, "eps must be > 0");
    if (!(lam > 0.0) || lam > 1.0) return fail(ctx, SKH_EINVAL, "lam must be in (0, 1]");
    if (precision != SKH_FP32 && precision != SKH_BF16_SPLIT)
        return fail(ctx, SKH_EINVAL, "unknown precision");
    const bool split = precision == SKH_BF16_SPLIT;
    const int kp = split ? skh::packed_width_bf16(d) : skh::packed_width(d);
    if (!kp) return fail(ctx, SKH_EINVAL, "the BF16 split path needs d <= 60");
    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    const int nbx = skh::bbox_blocks(n), nby = skh::bbox_blocks(m);

    // Phase A (bounding box, packing, clustering of the columns on the split path) and
    // phase B (column offsets, softmin partials) carve their buffers in two passes: the
    // first, with no base, measures.
    float *Xp, *Yp, *hnx, *hny, *lwy, *plo, *phi, *lohi;
    double *pmass, *mass;
    int *pbad, *bad;
    Clustered cy;
    auto carve_a = [&](Carver &c) {
        Xp = c.take<float>((size_t)n * kp);
        Yp = c.take<float>((size_t)m * kp);
        hnx = c.take<float>(n);
        hny = c.take<float>(m);
        lwy = c.take<float>(m);
        plo = c.take<float>((size_t)(nbx + nby) * 64);
        phi = c.take<float>((size_t)(nbx + nby) * 64);
        pmass = c.take<double>(nbx + nby);
        pbad = c.take<int>(2 * (nbx + nby));
        lohi = c.take<float>(192);
        mass = c.take<double>(2);
        bad = c.take<int>(4);
        if (split) cy.carve(c, (int)m, kp, 0);
    };
    skh::SoftminBatch batch{};
    batch.n_jobs = 1;
    batch.d = d;
    batch.kscale = (float)(kLog2e / eps);
    batch.job[0].n_rows = (int)n;
    float *u, *hperm;
    float2 *part;
    auto carve_b = [&](Carver &c, int m_cols) {
        u = c.take<float>(m_cols);
        hperm = c.take<float>(m_cols);
        part = c.take<float2>((size_t)batch.job[0].n_chunks * n);
    };
    SoftminRegions regions{ctx, no_alloc};
    Carver ma(nullptr);
    carve_a(ma);
    if (no_alloc) {  // the whole call must fit the scratch array: checked before any work
        const int m_cols_max = split ? cy.n_pad_max : (int)m;
        batch.job[0].n_cols = m_cols_max;
        skh::plan_softmin_batch(batch, target_wgs_softmin(ctx, split));
        Carver mb(nullptr);
        carve_b(mb, m_cols_max);
        const size_t need = ((ma.off + 255) & ~size_t(255)) + mb.off;
        if (need > kScratchBytes)
            return fail(ctx, SKH_EINVAL,
                        "skh_softmin_noalloc: this problem needs " + std::to_string(need) +
                            " bytes of scratch, more than the fixed " +
                            std::to_string(kScratchBytes) + " bytes");
    }
    void *base_a = nullptr;
    {
        const int rc = regions.get(0, ma.off, &base_a);
        if (rc) return rc;
        Carver c(base_a);
        carve_a(c);
    }
    SKH_HIP(skh::launch_bbox_partial(x, nullptr, n, d, plo, phi, pmass, pbad, s));
    SKH_HIP(skh::launch_bbox_partial(y, w, m, d, plo + (size_t)nbx * 64, phi + (size_t)nbx * 64,
                                     pmass + nbx, pbad + 2 * nbx, s));
    SKH_HIP(skh::launch_bbox_final(plo, phi, pmass, pbad, nbx, nby, d, lohi, mass, bad, s));
    SKH_HIP(skh::launch_pack(x, nullptr, n, d, kp, lohi + 128, Xp, hnx, nullptr, s));
    SKH_HIP(skh::launch_pack(y, w, m, d, kp, lohi + 128, Yp, hny, lwy, s));
    const float *cols_u_lw = lwy, *cols_hn = hny, *h_cols = h;
    int m_cols = (int)m;
    if (split) {
        int rc = cluster_start(ctx, cy, Yp, w, kp, kKmeansIters, s);
        if (rc) return rc;
        SKH_HIP(hipMemcpyAsync(ctx->host, cy.poff + cy.k, sizeof(int), hipMemcpyDeviceToHost, s));
        SKH_HIP(hipStreamSynchronize(s));
        cy.n_pad = *static_cast<int *>(ctx->host);
        rc = cluster_finish(ctx, cy, Yp, w, kp, s);
        if (rc) return rc;
        cols_u_lw = cy.lw;
        cols_hn = cy.hn;
        m_cols = cy.n_pad;
    }

    // Phase B: column offsets, the softmin, the merge.
    batch.job[0].n_cols = m_cols;
    const int wgs = skh::plan_softmin_batch(batch, target_wgs_softmin(ctx, split));
    {
        Carver mb(nullptr);
        carve_b(mb, m_cols);
        void *base_b = nullptr;
        const int rc = regions.get(1, mb.off, &base_b);
        if (rc) return rc;
        Carver c(base_b);
        carve_b(c, m_cols);
    }
    if (split) {
        SKH_HIP(skh::launch_permute(h, cy.perm_pad, cy.n_pad, hperm, s));
        h_cols = hperm;
    }
    SKH_HIP(skh::launch_col_offsets(cols_u_lw, h_cols, cols_hn, m_cols, eps, u, s));
    skh::SoftminJob &J = batch.job[0];
    J.rows = Xp;
    J.u = u;
    J.part = part;
    if (split) {
        SKH_HIP(skh::launch_u_slots(u, m_cols, kp, d, cy.Yhi[0], s));
        J.cols_hi = cy.Yhi[0];
        J.cols_lo = cy.Ylo;
        J.col_blk_cluster = cy.blk;
        J.col_centroids = cy.blkcent;
        SKH_HIP(skh::launch_softmin_bf16(batch, kp, wgs, s));
    } else {
        J.cols = Yp;
        SKH_HIP(skh::launch_softmin(batch, kp, precision, wgs, s));
    }
    SKH_HIP(skh::launch_softmin_finish(part, J.n_chunks, n, hnx, eps, lam, out, s));
    return SKH_OK;
}

}  // namespace

extern "C" {

int skh_softmin(skh_ctx *ctx, const float *x, int64_t n, const float *y, int64_t m, int32_t d,
                const float *w, const float *h, double eps, double lam, int32_t precision,
                float *out) {
    return softmin_impl(ctx, x, n, y, m, d, w, h, eps, lam, precision, out, false);
}

int skh_softmin_noalloc(skh_ctx *ctx, const float *x, int64_t n, const float *y, int64_t m,
                        int32_t d, const float *w, const float *h, double eps, double lam,
                        int32_t precision, float *out) {
    return softmin_impl(ctx, x, n, y, m, d, w, h, eps, lam, precision, out, true);
}

// Independent problems solved together (block-diagonal softmins): pair k owns the
// points [x_off[k], x_off[k+1]) of x and [y_off[k], y_off[k+1]) of y (host offsets).
struct Segments {
    int K;
    const int64_t *x_off, *y_off;
    double *S;  // host, K values of eq. (6)
};

// The cross plan applied to column values after a multiscale loop, over the kept
// cluster blocks of the final potentials: out_i = (pi V)_i / a_i (eq. (4), eq. (7)).
struct PostPlan {
    const float *V;  // m x L, caller order (device)
    int L;
    float *out;      // n x L, caller order (device)
};

static int solve(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                 const float *b, int64_t m, int32_t d, const skh_params *params, double *S_out,
                 float *f, float *g, float *p, float *q, skh_stats *stats, const Segments *seg,
                 const PostPlan *pp = nullptr);

int skh_sinkhorn_divergence(skh_ctx *ctx, const float *x, const float *a, int64_t n,
                            const float *y, const float *b, int64_t m, int32_t d,
                            const skh_params *params, double *S_out, float *f, float *g, float *p,
                            float *q, skh_stats *stats) {
    return solve(ctx, x, a, n, y, b, m, d, params, S_out, f, g, p, q, stats, nullptr);
}

int skh_sinkhorn_divergence_batched(skh_ctx *ctx, const float *x, const float *a,
                                    const int64_t *x_off, const float *y, const float *b,
                                    const int64_t *y_off, int32_t K, int32_t d,
                                    const skh_params *params, double *S_out, float *f, float *g,
                                    float *p, float *q, skh_stats *stats) {
    if (!ctx) return SKH_EINVAL;
    if (!x_off || !y_off || !S_out) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (K < 1) return fail(ctx, SKH_EINVAL, "K must be >= 1");
    if (x_off[0] != 0 || y_off[0] != 0) return fail(ctx, SKH_EINVAL, "offsets must start at 0");
    for (int k = 0; k < K; ++k)
        if (x_off[k + 1] <= x_off[k] || y_off[k + 1] <= y_off[k])
            return fail(ctx, SKH_EINVAL, "every pair needs at least one point on each side");
    const Segments seg{K, x_off, y_off, S_out};
    double S = 0.0;
    return solve(ctx, x, a, x_off[K], y, b, y_off[K], d, params, &S, f, g, p, q, stats, &seg);
}

static int solve(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                 const float *b, int64_t m, int32_t d, const skh_params *params, double *S_out,
                 float *f, float *g, float *p, float *q, skh_stats *stats, const Segments *seg,
                 const PostPlan *pp) {
    if (!ctx) return SKH_EINVAL;
    const auto t_start = std::chrono::steady_clock::now();
    if (!x || !a || !y || !b || !params) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || m < 1) return fail(ctx, SKH_EINVAL, "n and m must be >= 1");
    if (n > kMaxPoints || m > kMaxPoints) return fail(ctx, SKH_EINVAL, "n or m too large");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    skh_params P = *params;
    if (!(P.blur > 0.0) || !std::isfinite(P.blur)) return fail(ctx, SKH_EINVAL, "blur must be > 0");
    if (!(P.scaling > 0.0 && P.scaling < 1.0))
        return fail(ctx, SKH_EINVAL, "scaling must be in (0, 1)");
    if (std::isnan(P.reach) || std::isnan(P.diameter) || std::isnan(P.tol) ||
        std::isnan(P.jump_scale) || std::isnan(P.trunc_theta))
        return fail(ctx, SKH_EINVAL, "NaN parameter");
    if (P.extra_iters < 0 || P.max_iters < 0 || P.kmeans_iters < 0 || P.n_clusters < 0)
        return fail(ctx, SKH_EINVAL, "negative count parameter");
    if (P.precision != SKH_FP32 && P.precision != SKH_BF16_SPLIT)
        return fail(ctx, SKH_EINVAL, "unknown precision");
    for (int k = 0; k < 4; ++k)
        if (P.reserved[k]) return fail(ctx, SKH_EINVAL, "reserved params must be zero");
    const int fixed = P.fixed;
    if (fixed & ~(SKH_FIX_P | SKH_FIX_Q | SKH_FIX_CROSS))
        return fail(ctx, SKH_EINVAL, "unknown fixed bits");
    if ((fixed & SKH_FIX_CROSS) && P.multiscale)
        return fail(ctx, SKH_EINVAL, "a fixed cross loop needs a dense solve");
    if (((fixed & SKH_FIX_P) && !p) || ((fixed & SKH_FIX_Q) && !q) ||
        ((fixed & SKH_FIX_CROSS) && (!f || !g)))
        return fail(ctx, SKH_EINVAL, "fixed dual vectors must be given");
    if (P.init != SKH_INIT_COLD && P.init != SKH_INIT_GIVEN && P.init != SKH_INIT_WARM)
        return fail(ctx, SKH_EINVAL, "unknown init mode");
    if (std::isnan(P.start_scale)) return fail(ctx, SKH_EINVAL, "NaN parameter");
    if ((P.labels_x == nullptr) != (P.labels_y == nullptr))
        return fail(ctx, SKH_EINVAL, "labels_x and labels_y go together");
    if (P.init && (!f || !g || !p || !q))
        return fail(ctx, SKH_EINVAL, "init requires f, g, p and q");
    const bool split = P.precision == SKH_BF16_SPLIT;
    const bool ms = P.multiscale != 0;
    const bool clustered = split || ms;
    const int kp = split ? skh::packed_width_bf16(d) : skh::packed_width(d);
    if (!kp) return fail(ctx, SKH_EINVAL, "the BF16 split path needs d <= 60");
    const int check_every = P.check_every < 1 ? 1 : P.check_every;
    const bool balanced = is_balanced(P.reach);
    // cost |x - y|^p / p: eps = sigma^p, rho = reach^p (p = 2 unless given)
    const double pc = P.cost_p == 0.0 ? 2.0 : P.cost_p;
    if (!(pc >= 1.0 && pc <= 2.0)) return fail(ctx, SKH_EINVAL, "cost_p must be in [1, 2]");
    if (pc != 2.0 && (split || ms))
        return fail(ctx, SKH_EINVAL, "cost_p != 2 runs on the dense FP32 path only");
    auto powp = [pc](double v) { return pc == 2.0 ? v * v : std::pow(v, pc); };
    const double rho = balanced ? 0.0 : powp(P.reach);
    if (seg && (split || ms || pc != 2.0))
        return fail(ctx, SKH_EINVAL, "batched problems run on the dense FP32 path with p = 2");
    const int pp_lp = pp ? skh::plan_value_width(pp->L) : 0;
    if (pp && (!ms || pc != 2.0 || (P.fixed & SKH_FIX_CROSS) || pp->L < 1 || !pp_lp))
        return fail(ctx, SKH_EINVAL, "post-solve plan: multiscale, p = 2, 1 <= L <= 64");
    // batched: row tiles of each pair against that pair's column range, per problem
    // (0: rows x / cols x, 1: y / y, 2: y / x, 3: x / y)
    std::vector<int4> seg_tiles[4];
    std::vector<int2> seg_ranges[4];
    if (seg) {
        const int64_t *ro[4] = {seg->x_off, seg->y_off, seg->y_off, seg->x_off};
        const int64_t *co[4] = {seg->x_off, seg->y_off, seg->x_off, seg->y_off};
        for (int j = 0; j < 4; ++j) {
            for (int k = 0; k < seg->K; ++k) {
                for (int64_t r = ro[j][k]; r < ro[j][k + 1]; r += kRowTile)
                    seg_tiles[j].push_back(
                        make_int4((int)r, (int)std::min<int64_t>(r + kRowTile, ro[j][k + 1]), k, 0));
                seg_ranges[j].push_back(make_int2((int)co[j][k], (int)co[j][k + 1]));
            }
        }
    }

    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    const int nbx = skh::bbox_blocks(n), nby = skh::bbox_blocks(m);

    // ---- Phase A: bounding box, validation, packing, clustering ----
    float *Xp, *Yp, *hnx, *hny, *lwx, *lwy, *plo, *phi, *lohi;
    float *dist[4] = {nullptr, nullptr, nullptr, nullptr};  // xx, yy, yx, xy
    double *pmass, *mass;
    int *pbad, *bad, *wbad;
    Clustered cx, cy;
    int4 *seg_dtiles[4] = {nullptr, nullptr, nullptr, nullptr};
    int2 *seg_dranges[4] = {nullptr, nullptr, nullptr, nullptr};
    int *seg_ones = nullptr;
    int64_t *seg_xoff = nullptr, *seg_yoff = nullptr;
    double *seg_out = nullptr;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[0] : nullptr);
        Xp = c.take<float>((size_t)n * kp);
        Yp = c.take<float>((size_t)m * kp);
        hnx = c.take<float>(n);
        hny = c.take<float>(m);
        lwx = c.take<float>(n);
        lwy = c.take<float>(m);
        plo = c.take<float>((size_t)(nbx + nby) * 64);
        phi = c.take<float>((size_t)(nbx + nby) * 64);
        pmass = c.take<double>(nbx + nby);
        pbad = c.take<int>(2 * (nbx + nby));
        lohi = c.take<float>(192);
        mass = c.take<double>(2);
        bad = c.take<int>(4);
        wbad = c.take<int>(1);
        if (clustered) {
            cx.carve(c, (int)n, kp, P.n_clusters);
            cy.carve(c, (int)m, kp, P.n_clusters);
        }
        if (seg) {
            for (int j = 0; j < 4; ++j) {
                seg_dtiles[j] = c.take<int4>(seg_tiles[j].size());
                seg_dranges[j] = c.take<int2>(seg_ranges[j].size());
            }
            seg_ones = c.take<int>(seg->K);
            seg_xoff = c.take<int64_t>(seg->K + 1);
            seg_yoff = c.take<int64_t>(seg->K + 1);
            seg_out = c.take<double>(seg->K);
        }
        if (ms) {
            dist[0] = c.take<float>((size_t)cx.k * cx.k);
            dist[1] = c.take<float>((size_t)cy.k * cy.k);
            dist[2] = c.take<float>((size_t)cy.k * cx.k);
            dist[3] = c.take<float>((size_t)cx.k * cy.k);
        }
        if (!pass) {
            int rc = ensure_ws(ctx, 0, c.off);
            if (rc) return rc;
        }
    }
    SKH_HIP(skh::launch_bbox_partial(x, a, n, d, plo, phi, pmass, pbad, s));
    SKH_HIP(skh::launch_bbox_partial(y, b, m, d, plo + (size_t)nbx * 64, phi + (size_t)nbx * 64,
                                     pmass + nbx, pbad + 2 * nbx, s));
    SKH_HIP(skh::launch_bbox_final(plo, phi, pmass, pbad, nbx, nby, d, lohi, mass, bad, s));
    std::vector<int> seg_one_h;
    if (seg) {
        for (int j = 0; j < 4; ++j) {
            SKH_HIP(hipMemcpyAsync(seg_dtiles[j], seg_tiles[j].data(),
                                   seg_tiles[j].size() * sizeof(int4), hipMemcpyHostToDevice, s));
            SKH_HIP(hipMemcpyAsync(seg_dranges[j], seg_ranges[j].data(),
                                   seg_ranges[j].size() * sizeof(int2), hipMemcpyHostToDevice, s));
        }
        seg_one_h.assign(seg->K, 1);
        SKH_HIP(hipMemcpyAsync(seg_ones, seg_one_h.data(), seg->K * sizeof(int),
                               hipMemcpyHostToDevice, s));
        SKH_HIP(hipMemcpyAsync(seg_xoff, seg->x_off, (seg->K + 1) * sizeof(int64_t),
                               hipMemcpyHostToDevice, s));
        SKH_HIP(hipMemcpyAsync(seg_yoff, seg->y_off, (seg->K + 1) * sizeof(int64_t),
                               hipMemcpyHostToDevice, s));
    }
    char *hb = static_cast<char *>(ctx->host);
    SKH_HIP(hipMemcpyAsync(hb, lohi, 128 * sizeof(float), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipMemcpyAsync(hb + 512, mass, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipMemcpyAsync(hb + 528, bad, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    if (P.init == SKH_INIT_WARM) {  // the checked start: every starting value must be finite
        SKH_HIP(hipMemsetAsync(wbad, 0, sizeof(int), s));
        SKH_HIP(skh::launch_nonfinite(f, n, wbad, s));
        SKH_HIP(skh::launch_nonfinite(g, m, wbad, s));
        SKH_HIP(skh::launch_nonfinite(p, n, wbad, s));
        SKH_HIP(skh::launch_nonfinite(q, m, wbad, s));
        SKH_HIP(hipMemcpyAsync(hb + 544, wbad, sizeof(int), hipMemcpyDeviceToHost, s));
    }
    SKH_HIP(hipStreamSynchronize(s));
    int warm_fallback = 0;
    if (P.init == SKH_INIT_WARM && *reinterpret_cast<const int *>(hb + 544)) {
        P.init = SKH_INIT_COLD;
        warm_fallback = 1;
    }
    const float *hlo = reinterpret_cast<const float *>(hb);
    const float *hhi = hlo + 64;
    const double *hmass = reinterpret_cast<const double *>(hb + 512);
    const int *hbad = reinterpret_cast<const int *>(hb + 528);
    if (hbad[1] || hbad[3]) return fail(ctx, SKH_EINVAL, "negative, NaN or infinite weight");
    if (hbad[0] || hbad[2]) return fail(ctx, SKH_ENONFINITE, "non-finite coordinate");
    if (!(hmass[0] > 0.0) || !(hmass[1] > 0.0))
        return fail(ctx, SKH_EINVAL, "total weight must be positive");

    double diam = P.init && P.start_scale > 0.0 ? P.start_scale : P.diameter;
    if (!(diam > 0.0)) {
        double s2 = 0.0;
        for (int k = 0; k < d; ++k) {
            const double t = (double)hhi[k] - (double)hlo[k];
            s2 += t * t;
        }
        diam = std::sqrt(s2);
    }
    const std::vector<double> sig = scale_list(diam, P.blur, P.scaling);
    const int L = (int)sig.size();
    const int total = L + P.extra_iters;
    const int cap = total + (P.tol > 0.0 ? P.max_iters : 0);
    auto sigma_at = [&](int it) { return it < L ? sig[it] : P.blur; };

    SKH_HIP(skh::launch_pack(x, a, n, d, kp, lohi + 128, Xp, hnx, lwx, s));
    SKH_HIP(skh::launch_pack(y, b, m, d, kp, lohi + 128, Yp, hny, lwy, s));
    if (pc != 2.0) {  // no |x|^2/2 expansion terms for this cost
        SKH_HIP(hipMemsetAsync(hnx, 0, sizeof(float) * n, s));
        SKH_HIP(hipMemsetAsync(hny, 0, sizeof(float) * m, s));
    }
    // point sets of the fine loop: caller order (dense FP32) or cluster order
    int64_t nn = n, mm = m;
    const float *rowx = Xp, *rowy = Yp, *hnX = hnx, *hnY = hny, *lwX = lwx, *lwY = lwy, *wX = a,
                *wY = b;
    int t_jump = 0;
    if (clustered) {
        const int kmi = P.kmeans_iters;
        if (P.labels_x) {  // given clusterings: check the labels before sorting by them
            SKH_HIP(hipMemsetAsync(wbad, 0, sizeof(int), s));
            SKH_HIP(skh::launch_check_labels(P.labels_x, (int)n, cx.k, wbad, s));
            SKH_HIP(skh::launch_check_labels(P.labels_y, (int)m, cy.k, wbad, s));
            SKH_HIP(hipMemcpyAsync(hb + 544, wbad, sizeof(int), hipMemcpyDeviceToHost, s));
            SKH_HIP(hipStreamSynchronize(s));
            if (*reinterpret_cast<const int *>(hb + 544))
                return fail(ctx, SKH_EINVAL, "cluster label out of range");
        }
        int rc = cluster_start(ctx, cx, Xp, a, kp, kmi, s, P.labels_x);
        if (rc) return rc;
        rc = cluster_start(ctx, cy, Yp, b, kp, kmi, s, P.labels_y);
        if (rc) return rc;
        Clustered *cl2[2] = {&cx, &cy};
        for (Clustered *cl : cl2) {
            cl->h_poff.resize(cl->k + 1);
            cl->h_mass.resize(cl->k);
            cl->h_rad.resize(cl->k);
            SKH_HIP(hipMemcpyAsync(cl->h_poff.data(), cl->poff, (cl->k + 1) * sizeof(int),
                                   hipMemcpyDeviceToHost, s));
            SKH_HIP(hipMemcpyAsync(cl->h_mass.data(), cl->cmass, cl->k * sizeof(float),
                                   hipMemcpyDeviceToHost, s));
            SKH_HIP(hipMemcpyAsync(cl->h_rad.data(), cl->radius, cl->k * sizeof(float),
                                   hipMemcpyDeviceToHost, s));
        }
        SKH_HIP(hipStreamSynchronize(s));
        for (Clustered *cl : cl2) {
            cl->n_pad = cl->h_poff[cl->k];
            rc = cluster_finish(ctx, *cl, cl == &cx ? Xp : Yp, cl == &cx ? a : b, kp, s);
            if (rc) return rc;
        }
        nn = cx.n_pad;
        mm = cy.n_pad;
        rowx = cx.Xf;
        rowy = cy.Xf;
        hnX = cx.hn;
        hnY = cy.hn;
        lwX = cx.lw;
        lwY = cy.lw;
        wX = cx.wp;
        wY = cy.wp;
        if (ms) {
            for (Clustered *cl : cl2) {
                SKH_HIP(skh::launch_coarse_prep(cl->C, cl->cmass, cl->k, kp, cl->hnC, cl->lwC, s));
                SKH_HIP(skh::build_row_tiles(cl->poff, cl->k, cl->tcnt, cl->toff, cl->ssum,
                                             cl->tiles, s));
                int nt = 0;
                for (int c = 0; c < cl->k; ++c)
                    nt += (cl->h_poff[c + 1] - cl->h_poff[c] + kRowTile - 1) / kRowTile;
                cl->n_tiles = nt;
            }
            SKH_HIP(skh::launch_centroid_dist(cx.C, cx.k, cx.C, cx.k, kp, dist[0], s));
            SKH_HIP(skh::launch_centroid_dist(cy.C, cy.k, cy.C, cy.k, kp, dist[1], s));
            SKH_HIP(skh::launch_centroid_dist(cy.C, cy.k, cx.C, cx.k, kp, dist[2], s));
            SKH_HIP(skh::launch_centroid_dist(cx.C, cx.k, cy.C, cy.k, kp, dist[3], s));
            // coarse phase while sigma is above the jump scale (never for a warm start)
            if (!P.init && P.jump_scale >= 0.0) {
                double thr = P.jump_scale;
                if (!(thr > 0.0)) {  // mass-weighted RMS cluster radius of both clouds
                    double num = 0.0, den = 0.0;
                    for (Clustered *cl : cl2)
                        for (int c = 0; c < cl->k; ++c) {
                            num += (double)cl->h_mass[c] * cl->h_rad[c] * cl->h_rad[c];
                            den += cl->h_mass[c];
                        }
                    thr = den > 0.0 ? std::sqrt(num / den) : 0.0;
                }
                while (t_jump < L - 1 && sig[t_jump] > thr) ++t_jump;
            }
        }
    }

    // ---- Phase B: loop buffers ----
    skh::SoftminBatch batch{};
    batch.n_jobs = 4;
    batch.d = d;
    batch.cost_p = (float)pc;
    // job 0: a~^{aa} (rows x, cols x); job 1: b~^{bb} (rows y, cols y);
    // job 2: a~^{a->b} (rows y, cols x); job 3: b~^{b->a} (rows x, cols y).
    const int64_t nr[4] = {nn, mm, mm, nn}, nc[4] = {nn, mm, nn, mm};
    Clustered *rowc[4] = {&cx, &cy, &cy, &cx}, *colc[4] = {&cx, &cy, &cx, &cy};
    // problems of a fixed loop get no rows: no workgroups, no updates
    const bool skip_job[4] = {(fixed & SKH_FIX_P) != 0, (fixed & SKH_FIX_Q) != 0,
                              (fixed & SKH_FIX_CROSS) != 0, (fixed & SKH_FIX_CROSS) != 0};
    for (int k = 0; k < 4; ++k) {
        batch.job[k].n_rows = skip_job[k] ? 0 : (int)nr[k];
        batch.job[k].n_cols = (int)nc[k];
        if (ms) {
            batch.job[k].n_tiles = skip_job[k] ? 0 : rowc[k]->n_tiles;
            batch.job[k].range_cap = colc[k]->k / 2 + 2;
            batch.job[k].tiles = rowc[k]->tiles;  // marks block-sparse mode for planning
        }
        if (seg) {  // one range per pair: its own columns
            batch.job[k].n_tiles = skip_job[k] ? 0 : (int)seg_tiles[k].size();
            batch.job[k].range_cap = 1;
            batch.job[k].tiles = seg_dtiles[k];
            batch.job[k].ranges = seg_dranges[k];
            batch.job[k].range_count = seg_ones;
        }
    }
    const int wgs = skh::plan_softmin_batch(batch, target_wgs_softmin(ctx, split));
    const int fbx = skh::finish_blocks(nn), fby = skh::finish_blocks(mm);
    // coarse loop and jump batches (multiscale)
    skh::SoftminBatch cbatch{}, jbatch{};
    int cwgs = 0, jwgs = 0;
    const int kx = cx.k, ky = cy.k;
    if (ms && t_jump > 0) {
        cbatch.n_jobs = 4;
        cbatch.d = d;
        jbatch.n_jobs = 4;
        jbatch.d = d;
        const int64_t cr[4] = {kx, ky, ky, kx}, cc[4] = {kx, ky, kx, ky};
        for (int k = 0; k < 4; ++k) {
            cbatch.job[k].n_rows = skip_job[k] ? 0 : (int)cr[k];
            cbatch.job[k].n_cols = (int)cc[k];
            jbatch.job[k].n_rows = skip_job[k] ? 0 : (int)nr[k];
            jbatch.job[k].n_cols = (int)cc[k];
        }
        cwgs = skh::plan_softmin_batch(cbatch, target_wgs(ctx));
        jwgs = skh::plan_softmin_batch(jbatch, target_wgs(ctx));
    }
    float *u[4];
    float2 *part[4];
    double *acc, *sums;
    float *pot[4] = {f, g, p, q};
    const int64_t plen[4] = {nn, mm, nn, mm};
    int2 *ranges[4] = {nullptr, nullptr, nullptr, nullptr};
    int *rcount[4] = {nullptr, nullptr, nullptr, nullptr};
    float *cmax[4] = {nullptr, nullptr, nullptr, nullptr};  // f, g, p, q maxima per cluster
    unsigned long long *pairs_ctr = nullptr;
    float *pp_V = nullptr, *pp_part = nullptr, *pp_out = nullptr;
    float *uc[4], *cpot[4], *ju[4];
    float2 *cpart[4], *jpart[4];
    double *cacc = nullptr;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[1] : nullptr);
        for (int k = 0; k < 4; ++k) u[k] = c.take<float>(nc[k]);
        for (int k = 0; k < 4; ++k) part[k] = c.take<float2>((size_t)batch.job[k].n_chunks * nr[k]);
        acc = c.take<double>((size_t)(fbx + fby) * 4);
        sums = c.take<double>(8);
        for (int k = 0; k < 4; ++k) {
            float *t = c.take<float>(plen[k]);
            if (pass && (clustered || !pot[k])) pot[k] = t;
        }
        if (ms) {
            const int kk[4] = {kx, ky, kx, ky};
            for (int k = 0; k < 4; ++k) {
                ranges[k] = c.take<int2>((size_t)rowc[k]->k * batch.job[k].range_cap);
                rcount[k] = c.take<int>(rowc[k]->k);
                cmax[k] = c.take<float>(kk[k]);
            }
            pairs_ctr = c.take<unsigned long long>(1);
            if (pp) {
                pp_V = c.take<float>((size_t)cy.n_pad * pp->L);
                pp_part = c.take<float>((size_t)skh::kMaxPlanTileChunks * cx.n_pad * (pp->L + 2));
                pp_out = c.take<float>((size_t)cx.n_pad * pp->L);
            }
            if (t_jump > 0) {
                const int64_t cr[4] = {kx, ky, ky, kx}, cc[4] = {kx, ky, kx, ky};
                for (int k = 0; k < 4; ++k) {
                    uc[k] = c.take<float>(cc[k]);
                    cpot[k] = c.take<float>(kk[k]);
                    cpart[k] = c.take<float2>((size_t)cbatch.job[k].n_chunks * cr[k]);
                    ju[k] = c.take<float>(cc[k]);
                    jpart[k] = c.take<float2>((size_t)jbatch.job[k].n_chunks * nr[k]);
                }
                cacc = c.take<double>((size_t)(skh::finish_blocks(kx) + skh::finish_blocks(ky)) * 4);
            }
        }
        if (!pass) {
            int rc = ensure_ws(ctx, 1, c.off);
            if (rc) return rc;
        }
    }
    float *F = pot[0], *G = pot[1], *Pp = pot[2], *Q = pot[3];
    {
        // given values (init, or a fixed loop) are read from the caller; the rest start at 0
        const bool given[4] = {P.init || (fixed & SKH_FIX_CROSS), P.init || (fixed & SKH_FIX_CROSS),
                               P.init || (fixed & SKH_FIX_P), P.init || (fixed & SKH_FIX_Q)};
        const float *src[4] = {f, g, p, q};
        const Clustered *cl[4] = {&cx, &cy, &cx, &cy};
        for (int k = 0; k < 4; ++k) {
            if (given[k]) {
                if (clustered)
                    SKH_HIP(skh::launch_permute(src[k], cl[k]->perm_pad, cl[k]->n_pad, pot[k], s));
            } else {
                SKH_HIP(hipMemsetAsync(pot[k], 0, plen[k] * sizeof(float), s));
            }
        }
    }
    if (ms) SKH_HIP(hipMemsetAsync(pairs_ctr, 0, sizeof(unsigned long long), s));

    // ---- Coarse phase: the loop on the K-means centres, then the jump ----
    double pairs = 0.0, dense_pairs = 0.0;
    double pairs_per_iter = (skip_job[0] ? 0.0 : (double)n * n) +
                            (skip_job[1] ? 0.0 : (double)m * m) +
                            (skip_job[2] ? 0.0 : 2.0 * (double)n * m);
    if (seg) {
        pairs_per_iter = 0.0;
        for (int k = 0; k < seg->K; ++k) {
            const double nk = (double)(seg->x_off[k + 1] - seg->x_off[k]);
            const double mk = (double)(seg->y_off[k + 1] - seg->y_off[k]);
            pairs_per_iter += (skip_job[0] ? 0.0 : nk * nk) + (skip_job[1] ? 0.0 : mk * mk) +
                              (skip_job[2] ? 0.0 : 2.0 * nk * mk);
        }
    }
    if (ms && t_jump > 0) {
        float *Fc = cpot[0], *Gc = cpot[1], *Pc = cpot[2], *Qc = cpot[3];
        for (int k = 0; k < 4; ++k) SKH_HIP(hipMemsetAsync(cpot[k], 0, (k % 2 ? ky : kx) * sizeof(float), s));
        const double e0 = powp(sigma_at(0));
        SKH_HIP(skh::launch_col_offsets(cx.lwC, Pc, cx.hnC, kx, e0, uc[0], s));
        SKH_HIP(skh::launch_col_offsets(cy.lwC, Qc, cy.hnC, ky, e0, uc[1], s));
        SKH_HIP(skh::launch_col_offsets(cx.lwC, Fc, cx.hnC, kx, e0, uc[2], s));
        SKH_HIP(skh::launch_col_offsets(cy.lwC, Gc, cy.hnC, ky, e0, uc[3], s));
        const float *crow[4] = {cx.C, cy.C, cy.C, cx.C}, *ccol[4] = {cx.C, cy.C, cx.C, cy.C};
        for (int k = 0; k < 4; ++k) {
            cbatch.job[k].rows = crow[k];
            cbatch.job[k].cols = ccol[k];
            cbatch.job[k].u = uc[k];
            cbatch.job[k].part = cpart[k];
        }
        skh::FinishSide csx{}, csy{};
        csx.part_self = skip_job[0] ? nullptr : cpart[0];
        csx.part_cross = cpart[3];
        csx.chunks_self = cbatch.job[0].n_chunks;
        csx.chunks_cross = cbatch.job[3].n_chunks;
        csx.n = kx;
        csx.hn = cx.hnC;
        csx.lw = cx.lwC;
        csx.w = cx.cmass;
        csx.pot_self = Pc;
        csx.pot_cross = Fc;
        csx.u_self = uc[0];
        csx.u_cross = uc[2];
        csy.part_self = skip_job[1] ? nullptr : cpart[1];
        csy.part_cross = cpart[2];
        csy.chunks_self = cbatch.job[1].n_chunks;
        csy.chunks_cross = cbatch.job[2].n_chunks;
        csy.n = ky;
        csy.hn = cy.hnC;
        csy.lw = cy.lwC;
        csy.w = cy.cmass;
        csy.pot_self = Qc;
        csy.pot_cross = Gc;
        csy.u_self = uc[1];
        csy.u_cross = uc[3];
        const double cpairs = (skip_job[0] ? 0.0 : (double)kx * kx) +
                              (skip_job[1] ? 0.0 : (double)ky * ky) + 2.0 * (double)kx * ky;
        for (int it = 0; it < t_jump; ++it) {
            const double sigma = sigma_at(it), eps = powp(sigma), sn = sigma_at(it + 1);
            cbatch.kscale = (float)(kLog2e / eps);
            SKH_HIP(skh::launch_softmin(cbatch, kp, SKH_FP32, cwgs, s));
            SKH_HIP(skh::launch_iteration_finish(csx, csy, eps, damping(sigma, P.reach, pc), rho,
                                                 balanced ? 1 : 0, powp(sn), 0, cacc, s));
            pairs += cpairs;
        }
        // jump: one softmin of the fine points against the other cloud's coarse
        // measure, at the scale of the last coarse iteration
        const double sj = sigma_at(t_jump - 1), ej = powp(sj), lj = damping(sj, P.reach, pc);
        SKH_HIP(skh::launch_col_offsets(cx.lwC, Pc, cx.hnC, kx, ej, ju[0], s));
        SKH_HIP(skh::launch_col_offsets(cy.lwC, Qc, cy.hnC, ky, ej, ju[1], s));
        SKH_HIP(skh::launch_col_offsets(cx.lwC, Fc, cx.hnC, kx, ej, ju[2], s));
        SKH_HIP(skh::launch_col_offsets(cy.lwC, Gc, cy.hnC, ky, ej, ju[3], s));
        const float *jrow[4] = {rowx, rowy, rowy, rowx};
        for (int k = 0; k < 4; ++k) {
            jbatch.job[k].rows = jrow[k];
            jbatch.job[k].cols = ccol[k];
            jbatch.job[k].u = ju[k];
            jbatch.job[k].part = jpart[k];
        }
        jbatch.kscale = (float)(kLog2e / ej);
        SKH_HIP(skh::launch_softmin(jbatch, kp, SKH_FP32, jwgs, s));
        const float *jhn[4] = {hnX, hnY, hnY, hnX};
        float *jout[4] = {Pp, Q, G, F};
        for (int k = 0; k < 4; ++k)
            if (!skip_job[k])
                SKH_HIP(skh::launch_softmin_finish(jpart[k], jbatch.job[k].n_chunks, nr[k], jhn[k],
                                                   ej, lj, jout[k], s));
        pairs += (skip_job[0] ? 0.0 : (double)n * kx) + (skip_job[1] ? 0.0 : (double)m * ky) +
                 (double)m * kx + (double)n * ky;
    }

    // ---- Fine phase ----
    {
        const double e0 = powp(sigma_at(t_jump));
        SKH_HIP(skh::launch_col_offsets(lwX, Pp, hnX, nn, e0, u[0], s));
        SKH_HIP(skh::launch_col_offsets(lwY, Q, hnY, mm, e0, u[1], s));
        SKH_HIP(skh::launch_col_offsets(lwX, F, hnX, nn, e0, u[2], s));
        SKH_HIP(skh::launch_col_offsets(lwY, G, hnY, mm, e0, u[3], s));
    }
    // split path: the column offsets also live in the slots of each problem's hi plane
    auto refresh_slots = [&]() -> int {
        if (!split) return SKH_OK;
        for (int k = 0; k < 4; ++k)
            SKH_HIP(skh::launch_u_slots(u[k], (int)nc[k], kp, d, colc[k]->Yhi[k / 2], s));
        return SKH_OK;
    };
    {
        int rc = refresh_slots();
        if (rc) return rc;
    }
    const float *rowp[4] = {rowx, rowy, rowy, rowx}, *colp[4] = {Xp, Yp, Xp, Yp};
    for (int k = 0; k < 4; ++k) {
        skh::SoftminJob &J = batch.job[k];
        J.rows = rowp[k];
        J.u = u[k];
        J.part = part[k];
        if (split) {
            J.cols_hi = colc[k]->Yhi[k / 2];  // problems 0, 1: self; 2, 3: cross
            J.cols_lo = colc[k]->Ylo;
            J.col_blk_cluster = colc[k]->blk;
            J.col_centroids = colc[k]->blkcent;
        } else {
            J.cols = clustered ? colc[k]->Xf : colp[k];
        }
        if (ms) {
            J.tiles = rowc[k]->tiles;
            J.ranges = ranges[k];
            J.range_count = rcount[k];
        }
    }
    skh::FinishSide sx{}, sy{};
    sx.part_self = skip_job[0] ? nullptr : part[0];
    sx.part_cross = skip_job[3] ? nullptr : part[3];
    sx.chunks_self = batch.job[0].n_chunks;
    sx.chunks_cross = batch.job[3].n_chunks;
    sx.n = nn;
    sx.hn = hnX;
    sx.lw = lwX;
    sx.w = wX;
    sx.pot_self = Pp;
    sx.pot_cross = F;
    sx.u_self = u[0];
    sx.u_cross = u[2];
    sy.part_self = skip_job[1] ? nullptr : part[1];
    sy.part_cross = skip_job[2] ? nullptr : part[2];
    sy.chunks_self = batch.job[1].n_chunks;
    sy.chunks_cross = batch.job[2].n_chunks;
    sy.n = mm;
    sy.hn = hnY;
    sy.lw = lwY;
    sy.w = wY;
    sy.pot_self = Q;
    sy.pot_cross = G;
    sy.u_self = u[1];
    sy.u_cross = u[3];

    if (P.timing) {
        int rc = ensure_events(ctx, 2 * (size_t)cap);
        if (rc) return rc;
    }
    double err = -1.0, eps = powp(P.blur);
    int it = t_jump, checks = 0, launches = 0;
    bool converged = false;
    for (; it < cap; ++it) {
        const double sigma = sigma_at(it);
        eps = powp(sigma);
        const double lam = damping(sigma, P.reach, pc);
        const double sn = sigma_at(it + 1);
        if (ms) {  // cluster-block truncation from the current dual vectors
            SKH_HIP(skh::launch_cluster_max(F, wX, cx.poff, kx, cmax[0], s));
            SKH_HIP(skh::launch_cluster_max(G, wY, cy.poff, ky, cmax[1], s));
            SKH_HIP(skh::launch_cluster_max(Pp, wX, cx.poff, kx, cmax[2], s));
            SKH_HIP(skh::launch_cluster_max(Q, wY, cy.poff, ky, cmax[3], s));
            const int keep_all = P.trunc_theta > 0.0 ? 0 : 1;
            const double te = P.trunc_theta * eps;
            // rows x / cols x (p), rows y / cols y (q), rows y / cols x (g, f), rows x / cols y (f, g)
            if (!skip_job[0])
                SKH_HIP(skh::launch_block_ranges(kx, kx, cmax[2], cmax[2], dist[0], cx.radius,
                                                 cx.radius, cx.poff, cx.off, cx.off, lam, te,
                                                 keep_all, batch.job[0].range_cap, ranges[0],
                                                 rcount[0], pairs_ctr, s));
            if (!skip_job[1])
                SKH_HIP(skh::launch_block_ranges(ky, ky, cmax[3], cmax[3], dist[1], cy.radius,
                                                 cy.radius, cy.poff, cy.off, cy.off, lam, te,
                                                 keep_all, batch.job[1].range_cap, ranges[1],
                                                 rcount[1], pairs_ctr, s));
            SKH_HIP(skh::launch_block_ranges(ky, kx, cmax[1], cmax[0], dist[2], cy.radius, cx.radius,
                                             cx.poff, cx.off, cy.off, lam, te, keep_all,
                                             batch.job[2].range_cap, ranges[2], rcount[2],
                                             pairs_ctr, s));
            SKH_HIP(skh::launch_block_ranges(kx, ky, cmax[0], cmax[1], dist[3], cx.radius, cy.radius,
                                             cy.poff, cy.off, cx.off, lam, te, keep_all,
                                             batch.job[3].range_cap, ranges[3], rcount[3],
                                             pairs_ctr, s));
        } else {
            pairs += pairs_per_iter;
        }
        dense_pairs += pairs_per_iter;
        batch.kscale = (float)(kLog2e / eps);
        if (P.timing) SKH_HIP(hipEventRecord(ctx->events[2 * launches], s));
        if (split)
            SKH_HIP(skh::launch_softmin_bf16(batch, kp, wgs, s));
        else
            SKH_HIP(skh::launch_softmin(batch, kp, P.precision, wgs, s));
        if (P.timing) SKH_HIP(hipEventRecord(ctx->events[2 * launches + 1], s));
        ++launches;
        bool check = (it == cap - 1);
        if (P.tol > 0.0 && it >= total && ((it - total + 1) % check_every == 0)) check = true;
        SKH_HIP(skh::launch_iteration_finish(sx, sy, eps, lam, rho, balanced ? 1 : 0, powp(sn),
                                             check ? 1 : 0, acc, s));
        {
            int rc = refresh_slots();
            if (rc) return rc;
        }
        if (check) {
            SKH_HIP(skh::launch_sum_partials(acc, fbx, 4, sums, s));
            SKH_HIP(skh::launch_sum_partials(acc + (size_t)fbx * 4, fby, 4, sums + 4, s));
            SKH_HIP(hipMemcpyAsync(hb + 1024, sums, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
            SKH_HIP(hipStreamSynchronize(s));
            ++checks;
            const double *hs = reinterpret_cast<const double *>(hb + 1024);
            err = 0.0;
            for (int k = 0; k < 4; ++k) {
                const double num = hs[2 * k], den = hs[2 * k + 1];
                const double e = den > 0.0 ? num / den : 0.0;
                if (!std::isfinite(num) || !std::isfinite(den))
                    return fail(ctx, SKH_ENONFINITE, "non-finite marginal error");
                if (e > err) err = e;
            }
            if (P.tol > 0.0 && err <= P.tol) {
                converged = true;
                ++it;
                break;
            }
        }
    }

    // eq. (6) at eps = blur^p, FP64 on the device.
    int nbd = 0;
    SKH_HIP(skh::launch_divergence_terms(wX, F, Pp, nn, wY, G, Q, mm, rho, balanced ? 1 : 0, acc,
                                         &nbd, s));
    SKH_HIP(skh::launch_sum_partials(acc, nbd, 4, sums, s));
    SKH_HIP(hipMemcpyAsync(hb + 1024, sums, sizeof(double), hipMemcpyDeviceToHost, s));
    if (ms) SKH_HIP(hipMemcpyAsync(hb + 1088, pairs_ctr, sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, s));
    if (clustered) {
        float *outs[4] = {f, g, p, q};
        const Clustered *cl[4] = {&cx, &cy, &cx, &cy};
        for (int k = 0; k < 4; ++k)
            if (outs[k])
                SKH_HIP(skh::launch_unpermute(pot[k], cl[k]->perm_pad, cl[k]->n_pad, outs[k], s));
    }
    std::vector<double> seg_S;
    if (seg) {
        SKH_HIP(skh::launch_divergence_segments(wX, F, Pp, seg_xoff, wY, G, Q, seg_yoff, seg->K, rho,
                                                balanced ? 1 : 0, seg_out, s));
        seg_S.resize(seg->K);
        SKH_HIP(hipMemcpyAsync(seg_S.data(), seg_out, seg->K * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    }
    SKH_HIP(hipStreamSynchronize(s));
    double S = *reinterpret_cast<const double *>(hb + 1024);
    if (ms) pairs += (double)*reinterpret_cast<const unsigned long long *>(hb + 1088);
    const double eps_blur = powp(P.blur);
    if (!balanced) S = -(rho + 0.5 * eps_blur) * S;
    if (S_out) *S_out = S;
    if (seg)
        for (int k = 0; k < seg->K; ++k)
            seg->S[k] = balanced ? seg_S[k] : -(rho + 0.5 * eps_blur) * seg_S[k];
    if (pp) {
        // kept blocks of the cross problem (rows x, columns y) at the final potentials:
        // every entry of pi / (alpha beta) in a dropped block is below e^{-theta}, since
        // f_i + g_j - C_ij <= max_I f + max_J g - gap^2 / 2 (damping 1: the plan of
        // eq. (4) carries f and g undamped)
        SKH_HIP(skh::launch_cluster_max(F, wX, cx.poff, kx, cmax[0], s));
        SKH_HIP(skh::launch_cluster_max(G, wY, cy.poff, ky, cmax[1], s));
        SKH_HIP(skh::launch_block_ranges(kx, ky, cmax[0], cmax[1], dist[3], cx.radius, cy.radius,
                                         cy.poff, cy.off, cx.off, 1.0,
                                         P.trunc_theta * eps_blur, P.trunc_theta > 0.0 ? 0 : 1,
                                         batch.job[3].range_cap, ranges[3], rcount[3], pairs_ctr,
                                         s));
        SKH_HIP(skh::launch_permute_rows(pp->V, cy.perm_pad, (int)cy.n_pad, pp->L, pp_V, s));
        skh::PlanBatch pb{};
        pb.n_jobs = 1;
        pb.d = d;
        pb.kscale = (float)(kLog2e / eps_blur);
        skh::PlanJob &PJ = pb.job[0];
        PJ.rows = cx.Xf;
        PJ.cols = cy.Xf;
        PJ.u = u[3];  // offsets of g on the y columns at eps = blur^2
        PJ.V = pp_V;
        PJ.part = pp_part;
        PJ.n_rows = (int)cx.n_pad;
        PJ.n_cols = (int)cy.n_pad;
        PJ.L = pp->L;
        PJ.tiles = cx.tiles;
        PJ.n_tiles = cx.n_tiles;
        PJ.ranges = ranges[3];
        PJ.range_count = rcount[3];
        PJ.range_cap = batch.job[3].range_cap;
        const int pwgs = skh::plan_plan_batch(pb, ctx->num_cus * 32);
        SKH_HIP(skh::launch_plan_weighted(pb, kp, pp_lp, pwgs, s));
        SKH_HIP(skh::launch_plan_finish(pp_part, PJ.n_chunks, (int)cx.n_pad, pp->L, cx.hn, F,
                                        nullptr, eps_blur, pp_out, nullptr, s));
        SKH_HIP(skh::launch_unpermute_rows(pp_out, cx.perm_pad, (int)cx.n_pad, pp->L, pp->out, s));
    }
    double ms_softmin = 0.0;
    if (P.timing) {
        for (int k = 0; k < launches; ++k) {
            float t_ms = 0.0f;
            SKH_HIP(hipEventElapsedTime(&t_ms, ctx->events[2 * k], ctx->events[2 * k + 1]));
            ms_softmin += t_ms;
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->softmin_launches = launches;
        stats->coarse_iters = t_jump;
        stats->ms_softmin = ms_softmin;
        stats->iters = it;
        stats->n_scales = L;
        stats->converged = converged ? 1 : 0;
        stats->checks = checks;
        stats->diameter = diam;
        stats->warm_fallback = warm_fallback;
        stats->eps = eps;
        stats->marginal_err = err;
        stats->pairs = pairs;
        stats->dense_pairs = dense_pairs;
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                    t_start)
                              .count();
    }
    if (!std::isfinite(S)) return fail(ctx, SKH_ENONFINITE, "non-finite divergence");
    if (P.tol > 0.0 && !converged) return SKH_NOT_CONVERGED;
    return SKH_OK;
}

namespace {

// Shared body of skh_plan_apply and skh_grad_x: up to two plan jobs over the
// same row cloud x, each against its own column cloud, potentials and values.
struct PlanSpec {
    const float *cols;    // caller points (m x d)
    const float *cw;      // column weights
    int64_t m;
    const float *fpot;    // row potential
    const float *gpot;    // column potential
    const float *V;       // values (m x L) or NULL: column coordinates
    int L;
    float *out;           // n x L
    float *mass;          // n or NULL
};

// cost_p != 2: the cost |x - y|^p / p (eps is then blur^p); only the gradient sums
// (V = NULL) exist for it.
int run_plans(skh_ctx *ctx, const float *x, const float *a, int64_t n, int32_t d, double eps,
              int divide_by_a, const PlanSpec *specs, int nspec, float **Xp_out, int *kp_out,
              hipStream_t s, double cost_p = 2.0) {
    const bool pcost = cost_p != 2.0;
    const int kp = skh::packed_width(d);
    int Lmax = 1;
    for (int k = 0; k < nspec; ++k) Lmax = std::max(Lmax, specs[k].L);
    const int lp = skh::plan_value_width(Lmax);
    if (!lp) return fail(ctx, SKH_EINVAL, "L must be <= 64");
    int nb[3] = {skh::bbox_blocks(n), 0, 0};
    for (int k = 0; k < nspec; ++k) nb[1 + k] = skh::bbox_blocks(specs[k].m);
    const int nbt = nb[0] + nb[1] + nb[2];
    skh::PlanBatch batch{};
    batch.n_jobs = nspec;
    batch.d = d;
    batch.kscale = (float)(kLog2e / eps);
    for (int k = 0; k < nspec; ++k) {
        batch.job[k].n_rows = (int)n;
        batch.job[k].n_cols = (int)specs[k].m;
        batch.job[k].L = specs[k].L;
    }
    // many rounds of resident workgroups (four per CU): the last, partly idle one is short
    const int wgs = skh::plan_plan_batch(batch, ctx->num_cus * 96);
    float *Xp, *hnx, *plo, *phi, *lohi, *Cp[2], *hnc[2], *lwc[2], *uc[2], *part[2];
    double *pmass, *mass;
    int *pbad, *bad;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[0] : nullptr);
        Xp = c.take<float>((size_t)n * kp);
        hnx = c.take<float>(n);
        for (int k = 0; k < nspec; ++k) {
            Cp[k] = c.take<float>((size_t)specs[k].m * kp);
            hnc[k] = c.take<float>(specs[k].m);
            lwc[k] = c.take<float>(specs[k].m);
            uc[k] = c.take<float>(specs[k].m);
            part[k] = c.take<float>((size_t)batch.job[k].n_chunks * n * (specs[k].L + 2));
        }
        plo = c.take<float>((size_t)nbt * 64);
        phi = c.take<float>((size_t)nbt * 64);
        pmass = c.take<double>(nbt);
        pbad = c.take<int>(2 * nbt);
        lohi = c.take<float>(192);
        mass = c.take<double>(2);
        bad = c.take<int>(4);
        if (!pass) {
            int rc = ensure_ws(ctx, 0, c.off);
            if (rc) return rc;
        }
    }
    // common centre: bounding box of x and every column cloud
    SKH_HIP(skh::launch_bbox_partial(x, nullptr, n, d, plo, phi, pmass, pbad, s));
    int off = nb[0];
    for (int k = 0; k < nspec; ++k) {
        SKH_HIP(skh::launch_bbox_partial(specs[k].cols, nullptr, specs[k].m, d, plo + (size_t)off * 64,
                                         phi + (size_t)off * 64, pmass + off, pbad + 2 * off, s));
        off += nb[1 + k];
    }
    SKH_HIP(skh::launch_bbox_final(plo, phi, pmass, pbad, nb[0], nbt - nb[0], d, lohi, mass, bad, s));
    SKH_HIP(skh::launch_pack(x, nullptr, n, d, kp, lohi + 128, Xp, hnx, nullptr, s));
    // the p-cost records carry no half-norm expansion terms
    if (pcost) SKH_HIP(hipMemsetAsync(hnx, 0, (size_t)n * sizeof(float), s));
    for (int k = 0; k < nspec; ++k) {
        const PlanSpec &P = specs[k];
        SKH_HIP(skh::launch_pack(P.cols, P.cw, P.m, d, kp, lohi + 128, Cp[k], hnc[k], lwc[k], s));
        if (pcost) SKH_HIP(hipMemsetAsync(hnc[k], 0, (size_t)P.m * sizeof(float), s));
        SKH_HIP(skh::launch_col_offsets(lwc[k], P.gpot, hnc[k], P.m, eps, uc[k], s));
        skh::PlanJob &J = batch.job[k];
        J.rows = Xp;
        J.cols = Cp[k];
        J.u = uc[k];
        J.V = P.V;
        J.part = part[k];
    }
    if (pcost)
        SKH_HIP(skh::launch_plan_pcost(batch, kp, (float)cost_p, wgs, s));
    else
        SKH_HIP(skh::launch_plan_weighted(batch, kp, lp, wgs, s));
    for (int k = 0; k < nspec; ++k) {
        const PlanSpec &P = specs[k];
        SKH_HIP(skh::launch_plan_finish(part[k], batch.job[k].n_chunks, (int)n, P.L, hnx, P.fpot,
                                        divide_by_a ? nullptr : a, eps, P.out, P.mass, s));
    }
    if (Xp_out) *Xp_out = Xp;
    if (kp_out) *kp_out = kp;
    return SKH_OK;
}

}  // namespace

int skh_plan_apply(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                   const float *b, int64_t m, int32_t d, const float *f, const float *g,
                   double eps, const float *V, int32_t L, int32_t divide_by_a, float *out,
                   float *mass) {
    if (!ctx) return SKH_EINVAL;
    if (!x || !a || !y || !b || !f || !g || !V || !out)
        return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || m < 1 || n > kMaxPoints || m > kMaxPoints)
        return fail(ctx, SKH_EINVAL, "n, m out of range");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    if (L < 1 || L > 64) return fail(ctx, SKH_EINVAL, "L must be in [1, 64]");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ctx, SKH_EINVAL, "eps must be > 0");
    DeviceGuard guard(ctx->device);
    PlanSpec sp{y, b, m, f, g, V, L, out, mass};
    return run_plans(ctx, x, a, n, d, eps, divide_by_a, &sp, 1, nullptr, nullptr, ctx->stream);
}

namespace {

// grad_x S from (f, g, p) for the cost |x - y|^cost_p / cost_p at eps = blur^cost_p
int grad_x_impl(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                const float *b, int64_t m, int32_t d, const float *f, const float *g,
                const float *p, double blur, double cost_p, float *grad) {
    hipStream_t s = ctx->stream;
    // value buffers in the loop workspace: P1, m1, P2, m2
    float *buf;
    const size_t words = (size_t)n * d * 2 + (size_t)n * 2;
    {
        int rc = ensure_ws(ctx, 1, words * sizeof(float) + 1024);
        if (rc) return rc;
        buf = static_cast<float *>(ctx->ws[1]);
    }
    float *P1 = buf, *P2 = P1 + (size_t)n * d, *m1 = P2 + (size_t)n * d, *m2 = m1 + n;
    const double eps = std::pow(blur, cost_p);
    PlanSpec sp[2] = {{y, b, m, f, g, nullptr, d, P1, m1}, {x, a, n, p, p, nullptr, d, P2, m2}};
    float *Xp = nullptr;
    int kp = 0;
    int rc = run_plans(ctx, x, a, n, d, eps, 0, sp, 2, &Xp, &kp, s, cost_p);
    if (rc) return rc;
    SKH_HIP(skh::launch_grad_combine(Xp, (int)n, d, kp, P1, m1, P2, m2, grad, s));
    return SKH_OK;
}

}  // namespace

int skh_grad_x(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
               const float *b, int64_t m, int32_t d, const float *f, const float *g,
               const float *p, double blur, float *grad) {
    if (!ctx) return SKH_EINVAL;
    if (!x || !a || !y || !b || !f || !g || !p || !grad)
        return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || m < 1 || n > kMaxPoints || m > kMaxPoints)
        return fail(ctx, SKH_EINVAL, "n, m out of range");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    if (!(blur > 0.0) || !std::isfinite(blur)) return fail(ctx, SKH_EINVAL, "blur must be > 0");
    DeviceGuard guard(ctx->device);
    return grad_x_impl(ctx, x, a, n, y, b, m, d, f, g, p, blur, 2.0, grad);
}

int skh_gradients_p(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                    const float *b, int64_t m, int32_t d, const float *f, const float *g,
                    const float *p, const float *q, double blur, double reach, double cost_p,
                    float *grad_a, float *grad_b, float *grad_x, float *grad_y) {
    if (!ctx) return SKH_EINVAL;
    if (!x || !a || !y || !b || !f || !g || !p || !q) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || m < 1 || n > kMaxPoints || m > kMaxPoints)
        return fail(ctx, SKH_EINVAL, "n, m out of range");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    if (!(blur > 0.0) || !std::isfinite(blur)) return fail(ctx, SKH_EINVAL, "blur must be > 0");
    if (std::isnan(reach)) return fail(ctx, SKH_EINVAL, "reach is NaN");
    if (!(cost_p >= 1.0 && cost_p <= 2.0)) return fail(ctx, SKH_EINVAL, "cost_p must be in [1, 2]");
    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    const double eps = std::pow(blur, cost_p);
    const double rho = (reach > 0.0 && std::isfinite(reach)) ? std::pow(reach, cost_p) : 0.0;
    if (grad_a) SKH_HIP(skh::launch_grad_weights(f, p, n, eps, rho, grad_a, s));
    if (grad_b) SKH_HIP(skh::launch_grad_weights(g, q, m, eps, rho, grad_b, s));
    if (grad_x) {
        const int rc = grad_x_impl(ctx, x, a, n, y, b, m, d, f, g, p, blur, cost_p, grad_x);
        if (rc) return rc;
    }
    if (grad_y) {
        // S is symmetric in (alpha, beta): the x formula with the roles exchanged
        const int rc = grad_x_impl(ctx, y, b, m, x, a, n, d, g, f, q, blur, cost_p, grad_y);
        if (rc) return rc;
    }
    return SKH_OK;
}

int skh_gradients(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                  const float *b, int64_t m, int32_t d, const float *f, const float *g,
                  const float *p, const float *q, double blur, double reach, float *grad_a,
                  float *grad_b, float *grad_x, float *grad_y) {
    return skh_gradients_p(ctx, x, a, n, y, b, m, d, f, g, p, q, blur, reach, 2.0, grad_a, grad_b,
                           grad_x, grad_y);
}

int skh_label_transfer(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                       const float *b, int64_t m, int32_t d, const int32_t *labels, int32_t L,
                       int32_t flip_points, const skh_params *params, float *lab, float *score,
                       skh_stats *stats) {
    if (!ctx) return SKH_EINVAL;
    if (!x || !a || !y || !b || !labels || !params) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (!lab && !score) return fail(ctx, SKH_EINVAL, "lab and score are both NULL");
    if (n < 1 || m < 1 || n > kMaxPoints || m > kMaxPoints)
        return fail(ctx, SKH_EINVAL, "n, m out of range");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    if (L < 1 || L > 64) return fail(ctx, SKH_EINVAL, "L must be in [1, 64]");
    if (flip_points < 0 || (flip_points > 0 && d % flip_points != 0))
        return fail(ctx, SKH_EINVAL, "flip_points must be 0 or divide d");
    const int64_t na = flip_points ? 2 * n : n;
    if (na > kMaxPoints) return fail(ctx, SKH_EINVAL, "2 n exceeds the point limit");
    if (params->cost_p != 0.0 && params->cost_p != 2.0)
        return fail(ctx, SKH_EINVAL, "label transfer uses the cost |x - y|^2 / 2");
    if (params->init != SKH_INIT_COLD || params->fixed || params->labels_x || params->labels_y)
        return fail(ctx, SKH_EINVAL,
                    "label transfer runs its own cold solve (init, fixed, labels_x/y unset)");
    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    float *xa = nullptr, *aa = nullptr, *f, *g, *p, *q, *V, *aug;
    int *bad;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[3] : nullptr);
        if (flip_points) {
            xa = c.take<float>((size_t)na * d);
            aa = c.take<float>(na);
        }
        f = c.take<float>(na);
        p = c.take<float>(na);
        g = c.take<float>(m);
        q = c.take<float>(m);
        V = c.take<float>((size_t)m * L);
        aug = c.take<float>((size_t)na * L);
        bad = c.take<int>(1);
        if (!pass) {
            int rc = ensure_ws(ctx, 3, c.off);
            if (rc) return rc;
        }
    }
    char *hb = static_cast<char *>(ctx->host);
    SKH_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    SKH_HIP(skh::launch_check_labels(labels, (int)m, L, bad, s));
    SKH_HIP(hipMemcpyAsync(hb + 3072, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipStreamSynchronize(s));
    if (*reinterpret_cast<const int *>(hb + 3072))
        return fail(ctx, SKH_EINVAL, "atlas label out of range [0, L)");
    if (flip_points) SKH_HIP(skh::launch_flip_augment(x, a, n, d, flip_points, xa, aa, s));
    const float *X = flip_points ? xa : x, *A = flip_points ? aa : a;
    // only the cross loop is needed (eq. (7) uses f and g alone): the self loops stay
    // fixed at zero
    skh_params P = *params;
    P.fixed = SKH_FIX_P | SKH_FIX_Q;
    SKH_HIP(hipMemsetAsync(p, 0, sizeof(float) * na, s));
    SKH_HIP(hipMemsetAsync(q, 0, sizeof(float) * m, s));
    if (!P.multiscale) {  // dense: the cross loop starts from given zeros
        P.init = SKH_INIT_GIVEN;
        SKH_HIP(hipMemsetAsync(f, 0, sizeof(float) * na, s));
        SKH_HIP(hipMemsetAsync(g, 0, sizeof(float) * m, s));
    }
    double S = 0.0;
    SKH_HIP(skh::launch_one_hot(labels, m, L, V, s));
    if (P.multiscale) {
        // the plan runs inside the solve, over the cluster blocks kept at the final potentials
        const PostPlan pp{V, L, aug};
        const int rc = solve(ctx, X, A, na, y, b, m, d, &P, &S, f, g, p, q, stats, nullptr, &pp);
        if (rc < 0) return rc;
        SKH_HIP(skh::launch_label_fold(aug, n, L, flip_points ? 1 : 0, lab, score, s));
        return rc;
    }
    const int rc = skh_sinkhorn_divergence(ctx, X, A, na, y, b, m, d, &P, &S, f, g, p, q, stats);
    if (rc < 0) return rc;
    const int rc2 = skh_plan_apply(ctx, X, A, na, y, b, m, d, f, g, P.blur * P.blur, V, L, 1, aug,
                                   nullptr);
    if (rc2) return rc2;
    SKH_HIP(skh::launch_label_fold(aug, n, L, flip_points ? 1 : 0, lab, score, s));
    return rc;
}

int skh_diameter(skh_ctx *ctx, const float *x, int64_t n, const float *y, int64_t m, int32_t d,
                 double *out) {
    if (!ctx) return SKH_EINVAL;
    if (!x || !y || !out) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || m < 1 || n > kMaxPoints || m > kMaxPoints)
        return fail(ctx, SKH_EINVAL, "n, m out of range");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    const int nbx = skh::bbox_blocks(n), nby = skh::bbox_blocks(m);
    float *plo, *phi, *lohi;
    double *pmass, *mass;
    int *pbad, *bad;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[0] : nullptr);
        plo = c.take<float>((size_t)(nbx + nby) * 64);
        phi = c.take<float>((size_t)(nbx + nby) * 64);
        pmass = c.take<double>(nbx + nby);
        pbad = c.take<int>(2 * (nbx + nby));
        lohi = c.take<float>(192);
        mass = c.take<double>(2);
        bad = c.take<int>(4);
        if (!pass) {
            int rc = ensure_ws(ctx, 0, c.off);
            if (rc) return rc;
        }
    }
    SKH_HIP(skh::launch_bbox_partial(x, nullptr, n, d, plo, phi, pmass, pbad, s));
    SKH_HIP(skh::launch_bbox_partial(y, nullptr, m, d, plo + (size_t)nbx * 64, phi + (size_t)nbx * 64,
                                     pmass + nbx, pbad + 2 * nbx, s));
    SKH_HIP(skh::launch_bbox_final(plo, phi, pmass, pbad, nbx, nby, d, lohi, mass, bad, s));
    char *hb = static_cast<char *>(ctx->host);
    SKH_HIP(hipMemcpyAsync(hb, lohi, 128 * sizeof(float), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipMemcpyAsync(hb + 528, bad, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipStreamSynchronize(s));
    const float *hlo = reinterpret_cast<const float *>(hb);
    const int *hbad = reinterpret_cast<const int *>(hb + 528);
    if (hbad[0] || hbad[2]) return fail(ctx, SKH_ENONFINITE, "non-finite coordinate");
    double s2 = 0.0;
    for (int k = 0; k < d; ++k) {
        const double t = (double)hlo[64 + k] - (double)hlo[k];
        s2 += t * t;
    }
    *out = std::sqrt(s2);
    return SKH_OK;
}

int skh_self_potential(skh_ctx *ctx, const float *x, const float *a, int64_t n, int32_t d,
                       const skh_params *params, float *p, skh_stats *stats) {
    if (!ctx) return SKH_EINVAL;
    if (!x || !a || !params || !p) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || n > kMaxPoints) return fail(ctx, SKH_EINVAL, "n out of range");
    if (params->fixed) return fail(ctx, SKH_EINVAL, "fixed must be 0");
    if (params->multiscale) return fail(ctx, SKH_EINVAL, "the self loop runs dense");
    // the alpha<->alpha loop of the pair (alpha, alpha); the other three vectors
    // are zero placeholders, fixed, in the network workspace
    float *dummy;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[2] : nullptr);
        dummy = c.take<float>((size_t)3 * n);
        if (!pass) {
            int rc = ensure_ws(ctx, 2, c.off);
            if (rc) return rc;
        }
    }
    {
        DeviceGuard guard(ctx->device);
        SKH_HIP(hipMemsetAsync(dummy, 0, (size_t)3 * n * sizeof(float), ctx->stream));
    }
    skh_params P2 = *params;
    P2.fixed = SKH_FIX_Q | SKH_FIX_CROSS;
    int rc = skh_sinkhorn_divergence(ctx, x, a, n, x, a, n, d, &P2, nullptr, dummy, dummy + n, p,
                                     dummy + 2 * n, stats);
    return rc;
}

int skh_kmeans(skh_ctx *ctx, const float *x, const float *w, int64_t n, int32_t d, int32_t k,
               int32_t iters, float *centres, float *masses, int32_t *labels, int32_t *perm,
               int32_t *offsets) {
    if (!ctx) return SKH_EINVAL;
    if (!x) return fail(ctx, SKH_EINVAL, "NULL x");
    if (n < 1 || n > kMaxPoints) return fail(ctx, SKH_EINVAL, "n out of range");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    if (k < 1 || k > 4096 || k > n) return fail(ctx, SKH_EINVAL, "k must be in [1, min(n, 4096)]");
    if (iters < 0) return fail(ctx, SKH_EINVAL, "iters must be >= 0");
    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    const int kp = skh::packed_width(d);
    const int nb = skh::bbox_blocks(n);
    float *Xp, *hn, *plo, *phi, *lohi, *C, *cm;
    double *pmass, *mass;
    int *pbad, *bad, *kws;
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws[0] : nullptr);
        Xp = c.take<float>((size_t)n * kp);
        hn = c.take<float>(n);
        plo = c.take<float>((size_t)nb * 64);
        phi = c.take<float>((size_t)nb * 64);
        pmass = c.take<double>(nb);
        pbad = c.take<int>(2 * nb);
        lohi = c.take<float>(192);
        mass = c.take<double>(2);
        bad = c.take<int>(4);
        C = c.take<float>((size_t)k * kp);
        cm = c.take<float>(k);
        kws = c.take<int>(skh::kmeans_workspace_ints((int)n, k));
        if (!pass) {
            int rc = ensure_ws(ctx, 0, c.off);
            if (rc) return rc;
        }
    }
    SKH_HIP(skh::launch_bbox_partial(x, w, n, d, plo, phi, pmass, pbad, s));
    SKH_HIP(skh::launch_bbox_final(plo, phi, pmass, pbad, nb, 0, d, lohi, mass, bad, s));
    SKH_HIP(skh::launch_pack(x, w, n, d, kp, lohi + 128, Xp, hn, nullptr, s));
    int *dperm = nullptr, *doff = nullptr;
    SKH_HIP(skh::run_kmeans(Xp, w, (int)n, kp, k, iters, C, cm, nullptr, kws, &dperm, &doff, s));
    if (centres) SKH_HIP(skh::launch_unpack_centres(C, k, d, kp, lohi + 128, centres, s));
    if (masses) SKH_HIP(hipMemcpyAsync(masses, cm, k * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (labels) SKH_HIP(hipMemcpyAsync(labels, kws, n * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (perm) SKH_HIP(hipMemcpyAsync(perm, dperm, n * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (offsets)
        SKH_HIP(hipMemcpyAsync(offsets, doff, (k + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
    return SKH_OK;
}

}  // extern "C"
