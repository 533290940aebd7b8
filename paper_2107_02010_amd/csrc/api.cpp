// Host driver and C ABI of libskh (declared in include/skh.h).
//
// The driver runs the symmetric, averaged Sinkhorn loop with eps-scaling
// (Algorithm) on one device stream: per iteration one softmin launch covering
// the four problems (alpha<->alpha, beta<->beta, alpha->beta, beta->alpha)
// and one O(n + m) launch that merges, averages and prepares the next column
// offsets.  The host synchronises only for the bounding box (scale list and
// validation), for the periodic marginal-error check in converged mode, and
// for the final FP64 value of eq. (6).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "skh.h"
#include "skh_internal.h"

struct skh_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *host = nullptr;  // pinned, kHostBytes
    int num_cus = 256;
    std::vector<hipEvent_t> events;  // pairs bracketing timed softmin launches
    std::string err;
};

namespace {

constexpr size_t kHostBytes = 4096;
thread_local std::string g_create_err;

int fail(skh_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define SKH_HIP(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(ctx, SKH_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Sub-allocates one workspace; a first pass with base == nullptr measures.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

int ensure_ws(skh_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return SKH_OK;
    SKH_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->ws) {
        SKH_HIP(hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    size_t want = bytes + bytes / 8;
    if (hipMalloc(&ctx->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        ctx->ws = nullptr;
        return fail(ctx, SKH_ENOMEM,
                    "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    ctx->ws_bytes = want;
    return SKH_OK;
}

bool is_balanced(double reach) { return !(reach > 0.0) || std::isinf(reach); }

// lambda of the Algorithm, 1 / (1 + (sigma / reach)^2).
double damping(double sigma, double reach) {
    if (is_balanced(reach)) return 1.0;
    const double t = sigma / reach;
    return 1.0 / (1.0 + t * t);
}

// The scale list [d, d q, ..., blur] of the Algorithm's loop header:
// d q^k for k < K = ceil(log(d / blur) / log(1 / q)), then blur; [blur] when d <= blur.
std::vector<double> scale_list(double diameter, double blur, double scaling) {
    std::vector<double> s;
    if (!(diameter > blur)) {
        s.push_back(blur);
        return s;
    }
    const int K = (int)std::ceil(std::log(diameter / blur) / std::log(1.0 / scaling));
    for (int k = 0; k < K; ++k) s.push_back(diameter * std::pow(scaling, (double)k));
    s.push_back(blur);
    return s;
}

int target_wgs(const skh_ctx *ctx) { return ctx->num_cus * 8; }

int ensure_events(skh_ctx *ctx, size_t count) {
    while (ctx->events.size() < count) {
        hipEvent_t e;
        SKH_HIP(hipEventCreate(&e));
        ctx->events.push_back(e);
    }
    return SKH_OK;
}

// Bounding box, centre, masses and validation of one or two clouds; results
// land in ctx->host: floats [lo 64 | hi 64 | centre 64], then masses, then bad counts.
struct BBoxOut {
    float lo[64], hi[64];
    double mass[2];
    int bad[4];
};

}  // namespace

extern "C" {

void skh_params_default(skh_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->blur = 0.05;
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
    *out = ctx;
    return SKH_OK;
}

void skh_destroy(skh_ctx *ctx) {
    if (!ctx) return;
    {
        DeviceGuard guard(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        if (ctx->ws) (void)hipFree(ctx->ws);
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

int skh_softmin(skh_ctx *ctx, const float *x, int64_t n, const float *y, int64_t m, int32_t d,
                const float *w, const float *h, double eps, double lam, int32_t precision,
                float *out) {
    if (!ctx) return SKH_EINVAL;
    if (!x || !y || !w || !h || !out) return fail(ctx, SKH_EINVAL, "NULL array argument");
    if (n < 1 || m < 1) return fail(ctx, SKH_EINVAL, "n and m must be >= 1");
    if (n > INT32_MAX / 2 || m > INT32_MAX / 2) return fail(ctx, SKH_EINVAL, "n or m too large");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ctx, SKH_EINVAL, "eps must be > 0");
    if (!(lam > 0.0) || lam > 1.0) return fail(ctx, SKH_EINVAL, "lam must be in (0, 1]");
    if (precision != SKH_FP32 && precision != SKH_BF16_SPLIT)
        return fail(ctx, SKH_EINVAL, "unknown precision");
    DeviceGuard guard(ctx->device);
    const int kp = skh::packed_width(d);
    skh::SoftminBatch batch{};
    batch.n_jobs = 1;
    batch.d = d;
    batch.kscale = (float)(1.4426950408889634074 / eps);
    batch.job[0].n_rows = (int)n;
    batch.job[0].n_cols = (int)m;
    const int wgs = skh::plan_softmin_batch(batch, target_wgs(ctx));
    const int nbx = skh::bbox_blocks(n), nby = skh::bbox_blocks(m);

    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws : nullptr);
        float *Xp = c.take<float>((size_t)n * kp);
        float *Yp = c.take<float>((size_t)m * kp);
        float *hnx = c.take<float>(n);
        float *hny = c.take<float>(m);
        float *lwy = c.take<float>(m);
        float *u = c.take<float>(m);
        float2 *part = c.take<float2>((size_t)batch.job[0].n_chunks * n);
        float *plo = c.take<float>((size_t)(nbx + nby) * 64);
        float *phi = c.take<float>((size_t)(nbx + nby) * 64);
        double *pmass = c.take<double>(nbx + nby);
        int *pbad = c.take<int>(2 * (nbx + nby));
        float *lohi = c.take<float>(192);
        double *mass = c.take<double>(2);
        int *bad = c.take<int>(4);
        if (!pass) {
            int rc = ensure_ws(ctx, c.off);
            if (rc) return rc;
            continue;
        }
        hipStream_t s = ctx->stream;
        SKH_HIP(skh::launch_bbox_partial(x, nullptr, n, d, plo, phi, pmass, pbad, s));
        SKH_HIP(skh::launch_bbox_partial(y, w, m, d, plo + (size_t)nbx * 64, phi + (size_t)nbx * 64,
                                         pmass + nbx, pbad + 2 * nbx, s));
        SKH_HIP(skh::launch_bbox_final(plo, phi, pmass, pbad, nbx, nby, d, lohi, mass, bad, s));
        SKH_HIP(skh::launch_pack(x, nullptr, n, d, kp, lohi + 128, Xp, hnx, nullptr, s));
        SKH_HIP(skh::launch_pack(y, w, m, d, kp, lohi + 128, Yp, hny, lwy, s));
        SKH_HIP(skh::launch_col_offsets(lwy, h, hny, m, eps, u, s));
        batch.job[0].rows = Xp;
        batch.job[0].cols = Yp;
        batch.job[0].u = u;
        batch.job[0].part = part;
        SKH_HIP(skh::launch_softmin(batch, kp, precision, wgs, s));
        SKH_HIP(skh::launch_softmin_finish(part, batch.job[0].n_chunks, n, hnx, eps, lam, out, s));
    }
    return SKH_OK;
}

int skh_sinkhorn_divergence(skh_ctx *ctx, const float *x, const float *a, int64_t n,
                            const float *y, const float *b, int64_t m, int32_t d,
                            const skh_params *params, double *S_out, float *f, float *g, float *p,
                            float *q, skh_stats *stats) {
    if (!ctx) return SKH_EINVAL;
    const auto t_start = std::chrono::steady_clock::now();
    if (!x || !a || !y || !b || !params) return fail(ctx, SKH_EINVAL, "NULL argument");
    if (n < 1 || m < 1) return fail(ctx, SKH_EINVAL, "n and m must be >= 1");
    if (n > INT32_MAX / 2 || m > INT32_MAX / 2) return fail(ctx, SKH_EINVAL, "n or m too large");
    if (d < 1 || d > SKH_MAX_DIM) return fail(ctx, SKH_EINVAL, "d must be in [1, 63]");
    const skh_params P = *params;
    if (!(P.blur > 0.0) || !std::isfinite(P.blur)) return fail(ctx, SKH_EINVAL, "blur must be > 0");
    if (!(P.scaling > 0.0 && P.scaling < 1.0))
        return fail(ctx, SKH_EINVAL, "scaling must be in (0, 1)");
    if (std::isnan(P.reach) || std::isnan(P.diameter) || std::isnan(P.tol))
        return fail(ctx, SKH_EINVAL, "NaN parameter");
    if (P.extra_iters < 0 || P.max_iters < 0) return fail(ctx, SKH_EINVAL, "negative iteration count");
    if (P.precision != SKH_FP32 && P.precision != SKH_BF16_SPLIT)
        return fail(ctx, SKH_EINVAL, "unknown precision");
    for (int k = 0; k < 6; ++k)
        if (P.reserved[k]) return fail(ctx, SKH_EINVAL, "reserved params must be zero");
    if (P.init && (!f || !g || !p || !q))
        return fail(ctx, SKH_EINVAL, "init requires f, g, p and q");
    const int check_every = P.check_every < 1 ? 1 : P.check_every;
    const bool balanced = is_balanced(P.reach);
    const double rho = balanced ? 0.0 : P.reach * P.reach;

    DeviceGuard guard(ctx->device);
    hipStream_t s = ctx->stream;
    const int kp = skh::packed_width(d);
    skh::SoftminBatch batch{};
    batch.n_jobs = 4;
    batch.d = d;
    // job 0: a~^{aa} (rows x, cols x); job 1: b~^{bb} (rows y, cols y);
    // job 2: a~^{a->b} (rows y, cols x); job 3: b~^{b->a} (rows x, cols y).
    const int64_t nr[4] = {n, m, m, n}, nc[4] = {n, m, n, m};
    for (int k = 0; k < 4; ++k) {
        batch.job[k].n_rows = (int)nr[k];
        batch.job[k].n_cols = (int)nc[k];
    }
    const int wgs = skh::plan_softmin_batch(batch, target_wgs(ctx));
    const int nbx = skh::bbox_blocks(n), nby = skh::bbox_blocks(m);
    const int fbx = skh::finish_blocks(n), fby = skh::finish_blocks(m);

    float *Xp = nullptr, *Yp = nullptr, *hnx = nullptr, *hny = nullptr, *lwx = nullptr,
          *lwy = nullptr, *u[4] = {nullptr, nullptr, nullptr, nullptr};
    float2 *part[4] = {nullptr, nullptr, nullptr, nullptr};
    float *plo = nullptr, *phi = nullptr, *lohi = nullptr;
    double *pmass = nullptr, *mass = nullptr, *acc = nullptr, *sums = nullptr;
    int *pbad = nullptr, *bad = nullptr;
    float *pot[4] = {f, g, p, q};
    for (int pass = 0; pass < 2; ++pass) {
        Carver c(pass ? ctx->ws : nullptr);
        Xp = c.take<float>((size_t)n * kp);
        Yp = c.take<float>((size_t)m * kp);
        hnx = c.take<float>(n);
        hny = c.take<float>(m);
        lwx = c.take<float>(n);
        lwy = c.take<float>(m);
        for (int k = 0; k < 4; ++k) u[k] = c.take<float>(nc[k]);
        for (int k = 0; k < 4; ++k) part[k] = c.take<float2>((size_t)batch.job[k].n_chunks * nr[k]);
        plo = c.take<float>((size_t)(nbx + nby) * 64);
        phi = c.take<float>((size_t)(nbx + nby) * 64);
        pmass = c.take<double>(nbx + nby);
        pbad = c.take<int>(2 * (nbx + nby));
        lohi = c.take<float>(192);
        mass = c.take<double>(2);
        bad = c.take<int>(4);
        acc = c.take<double>((size_t)(fbx + fby) * 4);
        sums = c.take<double>(8);
        // potentials the caller did not ask for live in the workspace
        const int64_t plen[4] = {n, m, n, m};
        for (int k = 0; k < 4; ++k) {
            float *t = c.take<float>(plen[k]);
            if (pass && !pot[k]) pot[k] = t;
        }
        if (!pass) {
            int rc = ensure_ws(ctx, c.off);
            if (rc) return rc;
        }
    }
    float *F = pot[0], *G = pot[1], *Pp = pot[2], *Q = pot[3];

    // Bounding box, centre, masses, validation (one sync).
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
    const float *hhi = hlo + 64;
    const double *hmass = reinterpret_cast<const double *>(hb + 512);
    const int *hbad = reinterpret_cast<const int *>(hb + 528);
    if (hbad[1] || hbad[3]) return fail(ctx, SKH_EINVAL, "negative, NaN or infinite weight");
    if (hbad[0] || hbad[2]) return fail(ctx, SKH_ENONFINITE, "non-finite coordinate");
    if (!(hmass[0] > 0.0) || !(hmass[1] > 0.0))
        return fail(ctx, SKH_EINVAL, "total weight must be positive");

    double diam = P.diameter;
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
    if (!P.init) {
        SKH_HIP(hipMemsetAsync(F, 0, n * sizeof(float), s));
        SKH_HIP(hipMemsetAsync(Pp, 0, n * sizeof(float), s));
        SKH_HIP(hipMemsetAsync(G, 0, m * sizeof(float), s));
        SKH_HIP(hipMemsetAsync(Q, 0, m * sizeof(float), s));
    }
    {
        const double e0 = sigma_at(0) * sigma_at(0);
        SKH_HIP(skh::launch_col_offsets(lwx, Pp, hnx, n, e0, u[0], s));
        SKH_HIP(skh::launch_col_offsets(lwy, Q, hny, m, e0, u[1], s));
        SKH_HIP(skh::launch_col_offsets(lwx, F, hnx, n, e0, u[2], s));
        SKH_HIP(skh::launch_col_offsets(lwy, G, hny, m, e0, u[3], s));
    }
    const float *rowp[4] = {Xp, Yp, Yp, Xp}, *colp[4] = {Xp, Yp, Xp, Yp};
    for (int k = 0; k < 4; ++k) {
        batch.job[k].rows = rowp[k];
        batch.job[k].cols = colp[k];
        batch.job[k].u = u[k];
        batch.job[k].part = part[k];
    }
    skh::FinishSide sx{}, sy{};
    sx.part_self = part[0];
    sx.part_cross = part[3];
    sx.chunks_self = batch.job[0].n_chunks;
    sx.chunks_cross = batch.job[3].n_chunks;
    sx.n = n;
    sx.hn = hnx;
    sx.lw = lwx;
    sx.w = a;
    sx.pot_self = Pp;
    sx.pot_cross = F;
    sx.u_self = u[0];
    sx.u_cross = u[2];
    sy.part_self = part[1];
    sy.part_cross = part[2];
    sy.chunks_self = batch.job[1].n_chunks;
    sy.chunks_cross = batch.job[2].n_chunks;
    sy.n = m;
    sy.hn = hny;
    sy.lw = lwy;
    sy.w = b;
    sy.pot_self = Q;
    sy.pot_cross = G;
    sy.u_self = u[1];
    sy.u_cross = u[3];

    if (P.timing) {
        int rc = ensure_events(ctx, 2 * (size_t)cap);
        if (rc) return rc;
    }
    double err = -1.0, eps = P.blur * P.blur, pairs = 0.0;
    int it = 0, checks = 0;
    bool converged = false;
    const double pairs_per_iter = (double)n * n + (double)m * m + 2.0 * (double)n * m;
    for (; it < cap; ++it) {
        const double sigma = sigma_at(it);
        eps = sigma * sigma;
        const double lam = damping(sigma, P.reach);
        const double sn = sigma_at(it + 1);
        batch.kscale = (float)(1.4426950408889634074 / eps);
        if (P.timing) SKH_HIP(hipEventRecord(ctx->events[2 * it], s));
        SKH_HIP(skh::launch_softmin(batch, kp, P.precision, wgs, s));
        if (P.timing) SKH_HIP(hipEventRecord(ctx->events[2 * it + 1], s));
        pairs += pairs_per_iter;
        bool check = (it == cap - 1);
        if (P.tol > 0.0 && it >= total && ((it - total + 1) % check_every == 0)) check = true;
        SKH_HIP(skh::launch_iteration_finish(sx, sy, eps, lam, rho, balanced ? 1 : 0, sn * sn,
                                             check ? 1 : 0, acc, s));
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

    // eq. (6) at eps = blur^2, FP64 on the device.
    int nbd = 0;
    SKH_HIP(skh::launch_divergence_terms(a, F, Pp, n, b, G, Q, m, rho, balanced ? 1 : 0, acc, &nbd,
                                         s));
    SKH_HIP(skh::launch_sum_partials(acc, nbd, 4, sums, s));
    SKH_HIP(hipMemcpyAsync(hb + 1024, sums, sizeof(double), hipMemcpyDeviceToHost, s));
    SKH_HIP(hipStreamSynchronize(s));
    double S = *reinterpret_cast<const double *>(hb + 1024);
    const double eps_blur = P.blur * P.blur;
    if (!balanced) S = -(rho + 0.5 * eps_blur) * S;
    if (S_out) *S_out = S;
    double ms_softmin = 0.0;
    if (P.timing) {
        for (int k = 0; k < it; ++k) {
            float ms = 0.0f;
            SKH_HIP(hipEventElapsedTime(&ms, ctx->events[2 * k], ctx->events[2 * k + 1]));
            ms_softmin += ms;
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->softmin_launches = it;
        stats->ms_softmin = ms_softmin;
        stats->iters = it;
        stats->n_scales = L;
        stats->converged = converged ? 1 : 0;
        stats->checks = checks;
        stats->diameter = diam;
        stats->eps = eps;
        stats->marginal_err = err;
        stats->pairs = pairs;
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                    t_start)
                              .count();
    }
    if (!std::isfinite(S)) return fail(ctx, SKH_ENONFINITE, "non-finite divergence");
    if (P.tol > 0.0 && !converged) return SKH_NOT_CONVERGED;
    return SKH_OK;
}

}  // extern "C"
