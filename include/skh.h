/*
 * skh — symmetric, debiased, multiscale Sinkhorn divergence on MI355X (gfx950).
 *
 * C ABI of libskh.so.  The operations follow the problem statement of Feydy,
 * Roussillon, Trouve, Gori, "Fast and Scalable Optimal Transport for Brain
 * Tractograms" (MICCAI 2019, arXiv 2107.02010), Section 2:
 *
 *   alpha = sum_i a_i delta_{x_i},  beta = sum_j b_j delta_{y_j},  x, y in R^D,
 *   cost C(x, y) = |x - y|^2 / 2  (p = 2; skh_params.cost_p selects |x - y|^p / p),
 *   eps = sigma^2, rho = reach^2, lambda = 1 / (1 + eps / rho)  (sigma^p, reach^p).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Point arrays are row-major FP32, n x d (point i at x[i*d .. i*d+d-1]);
 *    weights and potentials are FP32 vectors.  Every array pointer is a DEVICE
 *    pointer on the context's device, owned by the caller.  Inputs are never
 *    written; outputs are written in the caller's point order.
 *  - 1 <= d <= SKH_MAX_DIM.  n >= 1, m >= 1.
 *  - All work is enqueued on the context's stream (skh_set_stream).  Calls
 *    that return host values (S, statistics) synchronise that stream before
 *    returning; the others return without synchronising.
 *  - The context owns a workspace that grows on demand and is freed by
 *    skh_destroy.  One context must not be used by two host threads at once.
 *  - Return codes: SKH_OK (0); SKH_NOT_CONVERGED (1): outputs are valid but
 *    the tolerance was not met; negative values are errors, with a message
 *    from skh_last_error.  On an error no output is guaranteed.
 *  - balanced problem: reach <= 0 or reach = +inf.
 */
#ifndef SKH_H
#define SKH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SKH_MAX_DIM 63

enum {
    SKH_OK = 0,
    SKH_NOT_CONVERGED = 1,
    SKH_EINVAL = -1,     /* bad argument: NULL, sizes, d, blur, scaling, negative or NaN weight */
    SKH_EHIP = -2,       /* HIP runtime error */
    SKH_ENOMEM = -3,     /* device allocation failed */
    SKH_ENONFINITE = -4, /* non-finite coordinate, or non-finite result */
};

/* precision of the x.y contraction inside the softmin; the log-sum-exp is FP32
 * in both modes. */
enum { SKH_FP32 = 0, SKH_BF16_SPLIT = 1 };

/* skh_params.fixed: the Algorithm's four updates form three independent loops
 * (alpha<->alpha reads only p, beta<->beta only q, the cross pair only f and g;
 * they meet in eq. (6) and the marginal check), so a loop whose fixed point is
 * already known can be left out: its vectors are read from the caller's
 * buffers (whatever init says), never updated, and its problems drop out of
 * the launches and of the marginal check.  With the same scale list the other
 * vectors come out exactly as in the full solve.  SKH_FIX_CROSS needs a dense
 * solve; SKH_FIX_P and SKH_FIX_Q also apply to multiscale solves (the coarse
 * loop, the jump and the block masks then skip the fixed self problems too). */
enum { SKH_FIX_P = 1, SKH_FIX_Q = 2, SKH_FIX_CROSS = 4 };

/* skh_params.init: where the dual vectors start. */
enum {
    SKH_INIT_COLD = 0,  /* zero, at the largest scale (the Algorithm's start) */
    SKH_INIT_GIVEN = 1, /* f, g, p, q hold starting values */
    SKH_INIT_WARM = 2   /* as GIVEN, but checked first: if any value is NaN or
                           infinite they are discarded and the call runs cold
                           (stats.warm_fallback = 1) */
};

typedef struct skh_ctx skh_ctx;

/* Solver parameters (the Algorithm's parameter lines and the two run modes). */
typedef struct skh_params {
    double blur;         /* finest scale sigma; eps = blur^2.  > 0 */
    double reach;        /* rho = reach^2; <= 0 or +inf: balanced */
    double scaling;      /* ratio q of consecutive scales, in (0, 1); the paper's default is 0.9 */
    double diameter;     /* largest scale; <= 0: diagonal of the joint bounding box of x and y */
    double tol;          /* > 0: converged mode, iterate at blur until the marginal error <= tol */
    double jump_scale;   /* multiscale: the fine phase starts at the first sigma <= jump_scale;
                            0: the mass-weighted RMS cluster radius; < 0: no coarse phase */
    double trunc_theta;  /* multiscale: keep cluster blocks whose weight bound is >= e^{-theta};
                            <= 0: keep every block */
    double start_scale;  /* init != COLD: largest scale of the schedule (start_scale q^k, then
                            blur); <= 0: the diameter rule.  A cold run ignores it */
    double cost_p;       /* exponent p of the cost C(x, y) = |x - y|^p / p (Section 2), in [1, 2];
                            eps = sigma^p, rho = reach^p, lambda = 1 / (1 + eps / rho).  0 is
                            read as 2.  p != 2: dense FP32 solves only (no multiscale, no BF16
                            split); the plan, gradient and label-transfer entries use p = 2 */
    const int32_t *labels_x; /* clustered paths (BF16 split, multiscale): optional cluster label
                            of every point of x in [0, k) (device, n values), k = n_clusters or
                            ceil(sqrt(n)); replaces the K-means (points are grouped, centres
                            are their weighted means).  Both or neither.  SKH_EINVAL when a
                            label is out of range */
    const int32_t *labels_y; /* the same for y (m values) */
    int32_t extra_iters; /* iterations at sigma = blur after the scale list (>= 0) */
    int32_t max_iters;   /* converged mode: at most this many iterations after the list */
    int32_t check_every; /* converged mode: marginal-error check period (>= 1) */
    int32_t precision;   /* SKH_FP32 or SKH_BF16_SPLIT */
    int32_t init;        /* SKH_INIT_COLD, SKH_INIT_GIVEN or SKH_INIT_WARM; a given start
                            skips the multiscale coarse phase */
    int32_t timing;      /* nonzero: time every softmin launch with HIP events (skh_stats) */
    int32_t multiscale;  /* nonzero: K-means coarse phase + cluster-block truncation */
    int32_t n_clusters;  /* multiscale / split path: clusters per cloud; 0: ceil(sqrt(n)) */
    int32_t kmeans_iters;/* Lloyd iterations (>= 0) */
    int32_t fixed;       /* SKH_FIX_* bits: dual vectors that are inputs, kept as given */
    int32_t reserved[4]; /* must be zero */
} skh_params;

/* Run statistics. */
typedef struct skh_stats {
    int32_t iters;       /* iterations run (each = four softmins + averaging) */
    int32_t n_scales;    /* length of the scale list */
    int32_t converged;   /* converged mode: tolerance met */
    int32_t checks;      /* number of marginal-error checks (each one host sync) */
    int32_t softmin_launches; /* softmin kernel launches (one per iteration) */
    int32_t coarse_iters;/* multiscale: iterations on the coarse (K-means) clouds */
    int32_t warm_fallback;/* SKH_INIT_WARM: the starting values were not finite, ran cold */
    int32_t reserved_i[1];
    double diameter;     /* largest scale used */
    double eps;          /* eps of the last iteration */
    double marginal_err; /* last measured relative L1 marginal error (max of the four problems) */
    double pairs;        /* point pairs evaluated by the softmin kernels (kept blocks only) */
    double ms_total;     /* wall time of the call, ms (host clock, inputs resident) */
    double ms_softmin;   /* params.timing: summed device time of the softmin launches, ms */
    double dense_pairs;  /* pairs a dense solve with the same iterations would evaluate */
    double reserved[1];
} skh_stats;

/* Fills *p with blur = 0.05, reach = +inf (balanced), scaling = 0.9,
 * diameter = 0 (auto), tol = 0 (schedule mode), extra_iters = 0,
 * max_iters = 1000, check_every = 5, precision = SKH_FP32, init = 0, timing = 0,
 * multiscale = 0, jump_scale = 0, trunc_theta = 20, start_scale = 0,
 * n_clusters = 0, kmeans_iters = 10, fixed = 0, cost_p = 2. */
void skh_params_default(skh_params *p);

/* Creates a context on HIP device `device` bound to stream `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Returns SKH_OK or SKH_EHIP. */
int skh_create(skh_ctx **out, int device, void *hip_stream);
void skh_destroy(skh_ctx *ctx);
/* Rebinds the context to another stream of the same device. */
int skh_set_stream(skh_ctx *ctx, void *hip_stream);
/* Message of the last error on this context (ctx may be NULL: last create error). */
const char *skh_last_error(const skh_ctx *ctx);
/* Caps the device workspace this context may hold at `bytes` (0: no cap, the
 * default).  A call whose workspace would exceed the cap fails with SKH_ENOMEM
 * before the workspace grows (earlier launches of that call may have run; its
 * outputs are then undefined) and leaves the context usable.  Setting a cap
 * below the current holding synchronizes the stream and frees the workspace.
 * Returns SKH_OK, SKH_EINVAL (NULL ctx) or SKH_EHIP. */
int skh_set_workspace_limit(skh_ctx *ctx, size_t bytes);
/* Device workspace bytes the context holds now (*out). */
int skh_workspace_bytes(const skh_ctx *ctx, size_t *out);

/*
 * One softmin, the reduction behind each of the four updates of the
 * Algorithm (the tilde lines), on arbitrary inputs:
 *
 *   out_i = -lam * eps * log sum_j w_j exp((h_j - C(x_i, y_j)) / eps),  i < n.
 *
 * x: n x d rows, y: m x d columns, w: m weights (>= 0; zero weights drop
 * out), h: m potential values.  eps > 0, 0 < lam <= 1.  A row with no
 * positive weight gets +inf.  precision: SKH_FP32 or SKH_BF16_SPLIT.
 * Errors: SKH_EINVAL for bad sizes/arguments, SKH_EHIP.
 */
int skh_softmin(skh_ctx *ctx, const float *x, int64_t n, const float *y, int64_t m, int32_t d,
                const float *w, const float *h, double eps, double lam, int32_t precision,
                float *out);

/*
 * skh_softmin for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments, same kernels and the same result as skh_softmin, but the call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * Its workspace is a fixed device array of 64 MiB compiled into the library,
 * one copy per device, held from the first context on that device until the
 * process ends.  Roughly (n + m) * 4 * (kp + 4) bytes plus the per-chunk
 * softmin partials must fit (kp = packed width, 64 for d = 60), e.g. a few
 * 10^4 points at d = 60; larger problems get SKH_EINVAL with the byte count
 * before any work is enqueued.  Every call on a device shares that device's
 * array and leaves its contents behind (nothing in it needs to start at
 * zero): calls that overlap on one device (two streams, two host threads,
 * two contexts) race and must be serialised by the caller.  The BF16 split
 * path synchronises the stream once (the padded column count), as
 * skh_softmin does.  Errors: as skh_softmin.
 */
int skh_softmin_noalloc(skh_ctx *ctx, const float *x, int64_t n, const float *y, int64_t m,
                        int32_t d, const float *w, const float *h, double eps, double lam,
                        int32_t precision, float *out);

/*
 * Symmetric, debiased Sinkhorn divergence S_{eps,rho}(alpha, beta), eq. (5),
 * evaluated through its dual form eq. (6) after the averaged symmetric loop
 * with eps-scaling (Algorithm).  Outputs (all nullable):
 *   S_out (host): the divergence, summed in FP64 on the device;
 *   f (n): b^{beta->alpha}, g (m): a^{alpha->beta},
 *   p (n): a^{alpha<->alpha}, q (m): b^{beta<->beta}  (device, FP32).
 * When params->init is nonzero, f, g, p, q must be given and hold the
 * starting values (caller order); the schedule then starts at
 * params->start_scale.  Returns SKH_OK, SKH_NOT_CONVERGED (converged mode only),
 * or an error.  Weights must be >= 0 and not all zero; coordinates finite.
 */
int skh_sinkhorn_divergence(skh_ctx *ctx, const float *x, const float *a, int64_t n,
                            const float *y, const float *b, int64_t m, int32_t d,
                            const skh_params *params, double *S_out, float *f, float *g, float *p,
                            float *q, skh_stats *stats);

/*
 * K independent problems solved together (a batched multi-pair call; the
 * barycenter of Section 3 runs its maps' cross loops this way): pair k is
 * (alpha_k, beta_k) with the points [x_off[k], x_off[k+1]) of x, a and
 * [y_off[k], y_off[k+1]) of y, b.  Every iteration runs the four softmins of
 * all pairs in one launch, each row tile against its own pair's columns only,
 * so the result of pair k is that of skh_sinkhorn_divergence on (alpha_k,
 * beta_k) with the same scale list.  The scale list is shared: its largest
 * scale is params.diameter, or the diagonal of the joint bounding box of all
 * points (an upper bound of every pair's distances); converged mode tests the
 * marginal error summed over all pairs.  The packing centres all points on one
 * midpoint (C is translation invariant; pairs far apart lose FP32 digits).
 * x_off, y_off: host arrays of K + 1 nondecreasing offsets from 0, every pair
 * at least one point on each side.  S_out: host array of K values of eq. (6).
 * f, g, p, q: as for skh_sinkhorn_divergence over the concatenated points
 * (fixed, init allowed).  Dense FP32 with p = 2 only (SKH_EINVAL otherwise).
 */
int skh_sinkhorn_divergence_batched(skh_ctx *ctx, const float *x, const float *a,
                                    const int64_t *x_off, const float *y, const float *b,
                                    const int64_t *y_off, int32_t K, int32_t d,
                                    const skh_params *params, double *S_out, float *f, float *g,
                                    float *p, float *q, skh_stats *stats);

/*
 * The largest scale of the Algorithm's list for the pair (x, y): the diagonal
 * of their joint bounding box (an upper bound of max |x_i - y_j|, the
 * diameter of the parameter lines).  *out is a host double.  Synchronises.
 */
int skh_diameter(skh_ctx *ctx, const float *x, int64_t n, const float *y, int64_t m, int32_t d,
                 double *out);

/*
 * Self dual vector p = a^{alpha<->alpha} alone: the Algorithm's alpha<->alpha
 * loop (one softmin per iteration) with the scale list, damping and stopping
 * rule of params (params->diameter should be the diameter of the full
 * problem, so that p matches the p of that solve; <= 0: the diagonal of x's
 * own bounding box).  init/start_scale apply to p; fixed must be 0.  p (n,
 * device) is written; stats as for skh_sinkhorn_divergence (nullable).
 */
int skh_self_potential(skh_ctx *ctx, const float *x, const float *a, int64_t n, int32_t d,
                       const skh_params *params, float *p, skh_stats *stats);

/*
 * Transport plan of eq. (4) applied to column values:
 *   out_il = a_i sum_j b_j exp((f_i + g_j - C(x_i, y_j)) / eps) V_jl,
 * i < n, l < L, V: m x L row-major (device), 1 <= L <= 64.  With
 * divide_by_a != 0 the a_i factor is left out: for one-hot label vectors V
 * this is the soft segmentation Lab_i of eq. (7).  f (n) and g (m) are the
 * dual vectors b^{beta->alpha}, a^{alpha->beta} of a previous solve (FP32,
 * caller order).  mass (n, nullable) receives the plan's row sums
 * sum_j pi_ij (a_i left out as for out).  Rows use FP32 arithmetic
 * throughout (MFMA contraction, online maximum).
 */
int skh_plan_apply(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                   const float *b, int64_t m, int32_t d, const float *f, const float *g,
                   double eps, const float *V, int32_t L, int32_t divide_by_a, float *out,
                   float *mass);

/*
 * Gradient of S_{eps,rho}(alpha, beta) with respect to the positions x_i, from
 * the dual vectors of a converged solve (envelope theorem on eq. (3); the
 * paper notes the gradients are expressions of the four dual vectors):
 *   grad_i = sum_j pi_ij (x_i - y_j) - sum_k pi^{aa}_ik (x_i - x_k),
 * pi from (f, g) and pi^{aa} from (p, p) by eq. (4) at eps = blur^2.
 * grad: n x d (device, caller order).  Valid for balanced and unbalanced S
 * (the marginal penalties do not depend on x).
 */
int skh_grad_x(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
               const float *b, int64_t m, int32_t d, const float *f, const float *g,
               const float *p, double blur, float *grad);

/*
 * All four gradients of S_{eps,rho}(alpha, beta) from the dual vectors of a
 * converged solve (Section 2: the gradients with respect to alpha_i, x_i,
 * beta_j, y_j are expressions of the four dual vectors f, p on alpha and g, q
 * on beta):
 *   grad_a_i = (rho + eps)(e^{-p_i/rho} - e^{-f_i/rho}), f_i - p_i when balanced
 *              (envelope theorem on the dual of eq. (3) for the three OT terms
 *              of eq. (5); the mass terms cancel); grad_b from (g, q);
 *   grad_x   as skh_grad_x;  grad_y the same with the roles of the measures
 *              exchanged: sum_i pi_ij (y_j - x_i) - sum_l pi^{bb}_jl (y_j - y_l).
 * eps = blur^2, rho = reach^2; reach <= 0 or infinite: balanced (grad_a and
 * grad_b are then defined up to one shared additive constant, the free constant
 * of (f, g)).  Inputs: all required (device, caller order, as returned by
 * skh_sinkhorn_divergence).  Outputs (device, FP32): grad_a (n), grad_b (m),
 * grad_x (n x d), grad_y (m x d); each may be NULL and is then not computed.
 * Errors: SKH_EINVAL for NULL inputs, sizes out of range, blur <= 0, NaN reach.
 */
int skh_gradients(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                  const float *b, int64_t m, int32_t d, const float *f, const float *g,
                  const float *p, const float *q, double blur, double reach, float *grad_a,
                  float *grad_b, float *grad_x, float *grad_y);

/*
 * skh_gradients for the cost C(x, y) = |x - y|^P / P with P = cost_p in [1, 2]
 * (Section 2, the cost and the parameter lines of the Algorithm: eps = blur^P,
 * rho = reach^P), from the dual vectors of a solve with that cost
 * (skh_params.cost_p = P).  Same arguments, layouts and ownership as
 * skh_gradients; cost_p = 2 is skh_gradients itself.  dS/d alpha, dS/d beta
 * take the same expression at that eps and rho;
 *   grad_x S_i = sum_j pi_ij |x_i - y_j|^{P-2} (x_i - y_j)
 *              - sum_k pi^aa_ik |x_i - x_k|^{P-2} (x_i - x_k)
 * (envelope theorem on eq. (3), pi from eq. (4) with that cost; pairs at
 * distance 0 contribute 0, the zero subgradient when P = 1), on a dense FP32
 * path for P != 2.  Errors: those of skh_gradients, and SKH_EINVAL for cost_p
 * outside [1, 2].
 */
int skh_gradients_p(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                    const float *b, int64_t m, int32_t d, const float *f, const float *g,
                    const float *p, const float *q, double blur, double reach, double cost_p,
                    float *grad_a, float *grad_b, float *grad_x, float *grad_y);

/*
 * Label transfer from a segmented atlas beta to a subject alpha (Section 3,
 * label transfer; eq. (7)): the cross dual vectors (f, g) of OT_{eps,rho}(alpha,
 * beta) from the symmetric loop, then soft labels
 *   Lab_i = sum_j beta_j onehot(labels_j) exp((f_i + g_j - C_ij) / eps)  (eq. (7))
 * and score_i = sum_l Lab_il, the fraction of alpha_i the plan transports: near 1
 * for a matched fibre, near 0 for an outlier (unbalanced problems, reach > 0).
 * flip_points = P > 0: the points are fibres of P points (d / P coordinates each,
 * point-major); the subject is augmented with the mirror flip of every fibre at
 * the same weight (Section 2, unoriented fibres), and the two versions of fibre
 * i add up in Lab_i (the plan keeps the better-oriented one).  0: no flips.
 * params: blur, reach, scaling, tolerance, multiscale settings as for
 * skh_sinkhorn_divergence; init must be SKH_INIT_COLD, fixed 0 and labels_x/y
 * NULL (the entry runs its own solve and holds the self loops, unused by eq. (7),
 * fixed at zero).  labels: m ints in [0, L) (device), 1 <= L <= 64.  Outputs (device,
 * caller order, each nullable but not both): lab (n x L), score (n).  stats as
 * for skh_sinkhorn_divergence (of the augmented problem).
 * Returns SKH_OK, SKH_NOT_CONVERGED (outputs valid), or an error: SKH_EINVAL for
 * NULL inputs, labels out of range, flip_points not dividing d, 2 n beyond the
 * point limit, or the parameter restrictions above.
 */
int skh_label_transfer(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                       const float *b, int64_t m, int32_t d, const int32_t *labels, int32_t L,
                       int32_t flip_points, const skh_params *params, float *lab, float *score,
                       skh_stats *stats);

/*
 * K-means coarse scale of one cloud (coarse-to-fine strategy, Section 2: a
 * K-means subsampling of the points for the first, coarse iterations).
 * Lloyd iterations from k evenly strided points (point floor(c n / k) for
 * centre c); a point joins the nearest centre, ties to the lowest index; a
 * centre becomes the w-weighted mean of its members (FP64 sums), an empty or
 * massless cluster keeps its centre.  After `iters` updates the points are
 * assigned once more and the centres set to the weighted means of those final
 * clusters.  w may be NULL (unit weights); 1 <= k <= min(n, 4096); iters >= 0.
 * Outputs (device, each nullable):
 *   centres (k x d, caller's coordinates), masses (k, sum of member weights),
 *   labels (n), perm (n: cluster-sorted position -> point index, stable in
 *   point order within a cluster), offsets (k + 1: cluster c occupies
 *   perm[offsets[c] .. offsets[c+1])).
 */
int skh_kmeans(skh_ctx *ctx, const float *x, const float *w, int64_t n, int32_t d, int32_t k,
               int32_t iters, float *centres, float *masses, int32_t *labels, int32_t *perm,
               int32_t *offsets);

/* ---------------------------------------------------------------------------
 * Learned warm start.  Not part of the paper's method: a set encoder that
 * predicts, for every K-means cluster of the two clouds (the coarse scale of
 * Section 2's coarse-to-fine strategy), the cluster's mean cross dual and
 * self dual divided by blur^2.  Broadcast to the points, the predictions are
 * starting values for skh_sinkhorn_divergence (init = SKH_INIT_WARM), whose
 * Algorithm then runs from start_scale to blur and decides the fixed point.
 *
 * Tokens (SKH_WS_IN = 64 features per cluster c of one cloud):
 *   [ (centre_c - mu) / diam  (d values, zeros up to index 59),
 *     log(k m_c / M), r_c / diam, [alpha side], [beta side] ]
 * with mu the centre and diam the diagonal of the joint bounding box of x and
 * y, m_c the cluster's mass, M the cloud's mass, k its cluster count and r_c
 * the largest distance of a member to the centre.  Token weight m_c.
 * d <= 60.
 *
 * Network: parameters theta = one FP32 vector of SKH_WS_N_PARAMS values,
 * in order W1 (256 x 64), b1, W2 (256 x 256), b2, W3 (256 x 256), b3,
 * W4 (256 x 768), b4, W5 (2 x 256), b5 (weights row-major, out x in).
 *   h = relu(relu(relu(X W1^T + b1) W2^T + b2) W3^T + b3)
 *   P_alpha, P_beta: token-weighted means of h over each cloud of a pair
 *   y_t = relu([h_t, P_alpha, P_beta] W4^T + b4) W5^T + b5    (2 values)
 * Batches: n_pairs cloud pairs, tokens in order pair 0 alpha, pair 0 beta,
 * pair 1 alpha, ...; seg (HOST array, 2 n_pairs + 1 offsets, seg[0] = 0,
 * non-decreasing, every segment non-empty) delimits them; T = seg[2 n_pairs].
 * Loss (training): mean over pairs of sum_t (w_t / W_pair) |y_t - target_t|^2.
 * ------------------------------------------------------------------------- */
#define SKH_WS_IN 64
#define SKH_WS_WIDTH 256
#define SKH_WS_OUT 2
#define SKH_WS_N_PARAMS 345602
#define SKH_WS_MAX_PAIRS 256

/* Tokens of the pair (alpha, beta): K-means of each cloud exactly as the
 * multiscale solver clusters it (k = n_clusters, or ceil(sqrt(n)) when 0, at
 * most 4096; kmeans_iters Lloyd iterations).  Writes tokens (kx + ky rows of
 * 64, alpha clusters first), tok_w (kx + ky), labels_x (n), labels_y (m) and
 * k_out[0] = kx, k_out[1] = ky (host).  cap_tokens: rows available in tokens
 * (SKH_EINVAL when kx + ky exceeds it).  Synchronises the stream. */
int skh_ws_tokens(skh_ctx *ctx, const float *x, const float *a, int64_t n, const float *y,
                  const float *b, int64_t m, int32_t d, int32_t n_clusters, int32_t kmeans_iters,
                  int32_t cap_tokens, float *tokens, float *tok_w, int32_t *labels_x,
                  int32_t *labels_y, int32_t *k_out);

/* Network forward on a batch: out (T x 2).  precision SKH_FP32 or
 * SKH_BF16_SPLIT (dense layers on bfloat16 operands, FP32 accumulation). */
int skh_ws_forward(skh_ctx *ctx, const float *theta, int32_t n_pairs, const int32_t *seg,
                   const float *tokens, const float *tok_w, int32_t precision, float *out);

/* Loss (host, FP64 sum) and its gradient grad (SKH_WS_N_PARAMS, device) for
 * targets (T x 2); FP32 forward and backward.  Synchronises the stream. */
int skh_ws_loss_grad(skh_ctx *ctx, const float *theta, int32_t n_pairs, const int32_t *seg,
                     const float *tokens, const float *tok_w, const float *target, double *loss,
                     float *grad);

/* One Adam update (Kingma & Ba, bias-corrected; step >= 1) of theta with
 * moments m and v (n values each, device). */
int skh_ws_adam(skh_ctx *ctx, int64_t n, float *theta, const float *grad, float *m, float *v,
                int32_t step, double lr, double beta1, double beta2, double eps);

/* Training targets of one cloud: out[c] = (scale * mean of pot_cross,
 * scale * mean of pot_self) over the points with label c, weighted by w
 * (FP64 sums in point order; 0 for a massless cluster).  labels in [0, k). */
int skh_ws_targets(skh_ctx *ctx, const int32_t *labels, int64_t n, int32_t k, const float *w,
                   const float *pot_cross, const float *pot_self, double scale, float *out);

/* Starting values of one cloud from the predictions pred (k x 2):
 * pot_cross[i] = scale pred[labels[i]][0], pot_self[i] = scale pred[labels[i]][1]. */
int skh_ws_expand(skh_ctx *ctx, const int32_t *labels, int64_t n, int32_t k, const float *pred,
                  double scale, float *pot_cross, float *pot_self);

#ifdef __cplusplus
}
#endif
#endif /* SKH_H */
