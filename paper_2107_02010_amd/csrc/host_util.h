// Host-side context and helpers shared by the C-ABI translation units of libskh.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "skh.h"
#include "skh_internal.h"

struct skh_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // setup, loop, warm-start network, label-transfer buffers
    void *ws[4] = {nullptr, nullptr, nullptr, nullptr};
    size_t ws_bytes[4] = {0, 0, 0, 0};
    size_t ws_limit = 0;   // cap on the sum of ws_bytes (0: none)
    void *host = nullptr;  // pinned, kHostBytes
    void *scratch = nullptr;  // this device's address of the fixed scratch array (api.cpp)
    int num_cus = 256;
    std::vector<hipEvent_t> events;  // pairs bracketing timed softmin launches
    std::string err;
};

namespace skh_host {

constexpr size_t kHostBytes = 4096;

inline int fail(skh_ctx *c, int code, const std::string &msg) {
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

inline size_t ws_total(const skh_ctx *ctx) {
    size_t t = 0;
    for (size_t b : ctx->ws_bytes) t += b;
    return t;
}

inline int ensure_ws(skh_ctx *ctx, int slot, size_t bytes) {
    if (bytes <= ctx->ws_bytes[slot]) return SKH_OK;
    size_t want = bytes + bytes / 8;  // headroom against regrowth
    if (ctx->ws_limit) {  // checked before anything is freed: the context stays usable
        const size_t others = ws_total(ctx) - ctx->ws_bytes[slot];
        if (others + bytes > ctx->ws_limit)
            return fail(ctx, SKH_ENOMEM,
                        "workspace limit of " + std::to_string(ctx->ws_limit) + " bytes: " +
                            std::to_string(others + bytes) + " needed");
        want = std::min(want, ctx->ws_limit - others);
    }
    SKH_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->ws[slot]) {
        SKH_HIP(hipFree(ctx->ws[slot]));
        ctx->ws[slot] = nullptr;
        ctx->ws_bytes[slot] = 0;
    }
    if (hipMalloc(&ctx->ws[slot], want) != hipSuccess) {
        (void)hipGetLastError();
        ctx->ws[slot] = nullptr;
        return fail(ctx, SKH_ENOMEM,
                    "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    ctx->ws_bytes[slot] = want;
    return SKH_OK;
}

inline bool is_balanced(double reach) { return !(reach > 0.0) || std::isinf(reach); }

// lambda of the Algorithm, 1 / (1 + (sigma / reach)^2).
// lambda = 1 / (1 + eps / rho) = 1 / (1 + (sigma / reach)^p)
inline double damping(double sigma, double reach, double p = 2.0) {
    if (is_balanced(reach)) return 1.0;
    const double t = sigma / reach;
    return 1.0 / (1.0 + (p == 2.0 ? t * t : std::pow(t, p)));
}

// The scale list [d, d q, ..., blur] of the Algorithm's loop header:
// d q^k for k < K = ceil(log(d / blur) / log(1 / q)), then blur; [blur] when d <= blur.
inline std::vector<double> scale_list(double diameter, double blur, double scaling) {
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

inline int target_wgs(const skh_ctx *ctx) { return ctx->num_cus * 8; }
// Workgroup target of the fine-loop softmin launches.  A workgroup sweeps a whole column
// chunk for milliseconds; splitting the columns into more chunks (at the 200k-point
// shape: three for the BF16 split kernel, three resident workgroups per CU; four for
// the FP32 kernel) gives many rounds of resident workgroups, so the last, partly idle
// round costs little.
inline int target_wgs_softmin(const skh_ctx *ctx, bool split) {
    return ctx->num_cus * (split ? 64 : 96);
}

inline int ensure_events(skh_ctx *ctx, size_t count) {
    while (ctx->events.size() < count) {
        hipEvent_t e;
        SKH_HIP(hipEventCreate(&e));
        ctx->events.push_back(e);
    }
    return SKH_OK;
}

constexpr double kLog2e = 1.4426950408889634074;
constexpr int64_t kMaxPoints = 1 << 28;
constexpr int kKmeansIters = 10;
constexpr int kRowTile = skh::kRowsPerBlock;

// Number of K-means clusters for n points: ceil(sqrt(n)), at most 4096.
inline int kmeans_k(int64_t n) {
    int k = (int)std::ceil(std::sqrt((double)n));
    if (k < 1) k = 1;
    if (k > 4096) k = 4096;
    return k;
}

// Device buffers of one cloud in the cluster-sorted, 32-padded layout.

}  // namespace skh_host
