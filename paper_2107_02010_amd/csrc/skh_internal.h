// Internal declarations shared by the HIP kernels and the host driver of libskh.
// Not part of the public C ABI (include/skh.h).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace skh {

// Packed point layout in HBM: one row of KP floats per point (KP = 4, 8, 16,
// 32 or 64, the smallest with d + 1 <= KP).  Slots [0, d) hold the coordinates
// minus a common centre (the cost is translation invariant), slot d is
// reserved for the augmented term of the softmin contraction, the rest is 0.
int packed_width(int d);
// Width of the packed rows for the BF16 split path: slots d, d+1, d+2 carry the
// three bf16 terms of the column offset and slot KP-1 the row reference, so
// d + 4 <= KP; KP is 16, 32 or 64 (0: d too large).
int packed_width_bf16(int d);

constexpr int kRowsPerBlock = 128;  // 4 waves x 32 rows
constexpr int kColsPerTile = 128;   // columns staged to LDS per step
constexpr int kMaxJobs = 4;

// One softmin reduction over a row set and a column set (one "instance").
//   L2_i = log2 sum_j 2^{ k * <x_i, y_j> + u_j }    (k = log2(e) / eps)
// written as (max, sum) partials per column chunk: part[chunk * n_rows + i].
struct SoftminJob {
    const float *rows;  // n_rows x KP packed FP32 (centred coordinates)
    const float *cols;  // FP32 path: n_cols x KP packed
    const __hip_bfloat16 *cols_hi;  // split path: n_cols x KP, hi part of y_j - c_J, with this
                                    // problem's column offsets in slots d..d+2 and 1.0 in KP-1
    const __hip_bfloat16 *cols_lo;  // split path: lo part (slots d.. are zero)
    const int *col_blk_cluster;     // split path: cluster of each 32-column block
    const float *col_centroids;     // split path: centre of each 32-column block's cluster (KP)
    const float *u;     // n_cols log2-domain column offsets; -inf = no mass
    float2 *part;       // n_chunks x n_rows
    int n_rows, n_cols;
    int row_tiles;      // ceil(n_rows / kRowsPerBlock)
    int n_chunks;       // column chunks
    int chunk_cols;     // columns per chunk (multiple of kColsPerTile)
    int wg_begin;       // first workgroup of this job in the launch
    // Block-sparse mode (tiles != NULL): workgroup w handles tiles[w % n_tiles] =
    // {row_begin, row_end, row_cluster, 0} (rows of one cluster, at most
    // kRowsPerBlock) against the column ranges ranges[cluster * range_cap ..
    // + range_count[cluster]), each [begin, end) in padded column order; chunk
    // c = w / n_tiles takes ranges c, c + n_chunks, ... of that list.
    const int4 *tiles;
    const int2 *ranges;
    const int *range_count;
    int range_cap;
    int n_tiles;
};

struct SoftminBatch {
    SoftminJob job[kMaxJobs];
    int n_jobs;
    int d;         // coordinates per point; slot d carries the augmented term
    float kscale;  // log2(e) / eps
    float cost_p;  // exponent p of the cost |x - y|^p / p; 0 or 2: the p = 2 kernels
    // log2 of the largest term (relative to a row's level) that a skipped block may
    // hold, set by plan_softmin_batch from the longest column set of the launch: with a
    // row sum >= 2^-4 of the level, m such terms add less than 2^-28 m 2^skip_log2,
    // below FP32 rounding when skip_log2 <= -28 - log2(m)
    float skip_log2;
};

// Builds chunking for a batch of jobs so that the launch holds enough
// workgroups to fill the device; returns the total workgroup count.
int plan_softmin_batch(SoftminBatch &b, int target_wgs);

hipError_t launch_softmin(const SoftminBatch &b, int kp, int precision, int total_wgs,
                          hipStream_t s);
hipError_t launch_softmin_bf16(const SoftminBatch &b, int kp, int total_wgs, hipStream_t s);
// cost |x - y|^p / p with p != 2 (dense FP32 path, one row per thread)
hipError_t launch_softmin_pcost(const SoftminBatch &b, int kp, int total_wgs, hipStream_t s);
// u -> three bf16 terms in slots d..d+2 of a packed hi plane (split path)
hipError_t launch_u_slots(const float *u, int n, int kp, int d, __hip_bfloat16 *hi,
                          hipStream_t s);

// ---- Plan applied to column values (plan.hip) ----
struct PlanJob {
    const float *rows;  // n_rows x KP packed FP32
    const float *cols;  // n_cols x KP packed FP32
    const float *u;     // n_cols column offsets (as in SoftminJob)
    const float *V;     // n_cols x L values, or NULL: the centred column coordinates (L = d)
    float *part;        // n_chunks x n_rows records [M, W, P_0 .. P_{L-1}]
    int n_rows, n_cols, L;
    int row_tiles, n_chunks, chunk_cols, wg_begin;
    // Block-sparse mode (tiles != NULL), as in SoftminJob: workgroup w takes the rows
    // tiles[w] = {begin, end, row cluster, 0} against that cluster's column ranges.
    const int4 *tiles;
    const int2 *ranges;
    const int *range_count;
    int range_cap;
    int n_tiles;
};
struct PlanBatch {
    PlanJob job[kMaxJobs];
    int n_jobs;
    int d;
    float kscale;
    int pad;
};
int plan_plan_batch(PlanBatch &b, int target_wgs);
int plan_value_width(int L);  // 4..64, 0 if L > 64
// Block-sparse plan launches split a row tile's range list over at most this many
// workgroups (records per row: that many times L + 2 floats).
constexpr int kMaxPlanTileChunks = 4;
hipError_t launch_plan_weighted(const PlanBatch &b, int kp, int lp, int total_wgs, hipStream_t s);
// gradient records for the cost |x - y|^p / p, p != 2 (dense jobs, V = NULL, L = d < kp;
// packed half-norms zero): [M, sum 2^{s-M} w, sum 2^{s-M} w y], w = |x - y|^{p-2}
hipError_t launch_plan_pcost(const PlanBatch &b, int kp, float pexp, int total_wgs, hipStream_t s);
hipError_t launch_plan_finish(const float *part, int chunks, int n, int L, const float *hn,
                              const float *pot, const float *w, double eps, float *out,
                              float *mass, hipStream_t s);
hipError_t launch_grad_combine(const float *X, int n, int d, int kp, const float *P1,
                               const float *m1, const float *P2, const float *m2, float *grad,
                               hipStream_t s);
hipError_t launch_grad_weights(const float *f, const float *p, int64_t n, double eps, double rho,
                               float *out, hipStream_t s);
hipError_t launch_flip_augment(const float *x, const float *a, int64_t n, int d, int P, float *xa,
                               float *aa, hipStream_t s);
hipError_t launch_one_hot(const int *labels, int64_t m, int L, float *V, hipStream_t s);
hipError_t launch_label_fold(const float *aug, int64_t n, int L, int flips, float *lab, float *score,
                             hipStream_t s);

// ---- K-means and the cluster-sorted, 32-padded layout (kmeans.hip) ----
size_t kmeans_workspace_ints(int n, int k);
// Lloyd iterations on X (n x kp, centred FP32) with weights w; C: k x kp centres
// (output), cmass/radius: k (nullable).  *perm_out / *off_out point into ws:
// perm (sorted position -> point) and off (k + 1 cluster offsets).
hipError_t run_kmeans(const float *X, const float *w, int n, int kp, int k, int iters, float *C,
                      float *cmass, float *radius, int *ws, int **perm_out, int **off_out,
                      hipStream_t s);
int scan_sums_len(int64_t len);
hipError_t launch_exclusive_scan(const int *in, int64_t len, int *sums, int *out, hipStream_t s);
// poff (k + 1): exclusive scan of the cluster sizes rounded up to 32 (psize: k + 1 ints).
hipError_t build_padded_layout(const int *perm, const int *off, int k, int *psize, int *poff,
                               int *scan_sums, hipStream_t s);
hipError_t fill_padded_layout(const int *perm, const int *off, const int *poff, int k,
                              int *perm_pad, int *blk_cluster, hipStream_t s);
// Xf: centred FP32 rows; Yhi0/Yhi1: two copies of the hi plane of x - c (one per
// problem that reads the cloud as columns), slot KP-1 = 1.0; Ylo: the lo plane.
hipError_t launch_pack_padded(const float *X, const float *w, const int *perm_pad,
                              const int *blk_cluster, const float *C, int n_pad, int kp, float *Xf,
                              __hip_bfloat16 *Yhi0, __hip_bfloat16 *Yhi1, __hip_bfloat16 *Ylo,
                              float *hn, float *lw, float *wp, hipStream_t s);
// blk_cent[b * kp + t] = C[blk_cluster[b] * kp + t] for the n_pad / 32 blocks
hipError_t launch_blk_centroids(const int *blk_cluster, const float *C, int nblk, int kp,
                                float *blk_cent, hipStream_t s);
hipError_t launch_unpack_centres(const float *C, int k, int d, int kp, const float *centre,
                                 float *out, hipStream_t s);
hipError_t launch_permute_rows(const float *src, const int *perm_pad, int n_pad, int L, float *out,
                               hipStream_t s);
hipError_t launch_unpermute_rows(const float *in, const int *perm_pad, int n_pad, int L,
                                 float *out, hipStream_t s);
hipError_t launch_unpermute(const float *in, const int *perm_pad, int n_pad, float *out,
                            hipStream_t s);
hipError_t launch_permute(const float *src, const int *perm_pad, int n_pad, float *out,
                          hipStream_t s);

// ---- Coarse-to-fine support (multiscale.hip) ----
hipError_t launch_cluster_max(const float *pot, const float *w, const int *poff, int k, float *out,
                              hipStream_t s);
hipError_t launch_centroid_dist(const float *CI, int ki, const float *CJ, int kj, int kp,
                                float *dist, hipStream_t s);
hipError_t launch_block_ranges(int ki, int kj, const float *rmax, const float *cmax,
                               const float *dist, const float *rrad, const float *crad,
                               const int *cpoff, const int *coff, const int *roff, double lam,
                               double theta_eps, int keep_all, int cap, int2 *ranges, int *count,
                               unsigned long long *pairs, hipStream_t s);
hipError_t launch_coarse_prep(const float *C, const float *cmass, int k, int kp, float *hn,
                              float *lw, hipStream_t s);
// tiles: ceil(size_c / kRowsPerBlock) entries per cluster (cnt, toff: k + 1 ints)
hipError_t build_row_tiles(const int *poff, int k, int *cnt, int *toff, int *scan_sums,
                           int4 *tiles, hipStream_t s);

// Bounding box and validation of one cloud.
//   plo/phi: nb x 64 partial min/max, pmass: nb FP64 partial weight sums,
//   pbad: nb counts of (non-finite coordinate) + 2^20 * (negative/NaN weight).
int bbox_blocks(int64_t n);
hipError_t launch_bbox_partial(const float *x, const float *w, int64_t n, int d, float *plo,
                               float *phi, double *pmass, int *pbad, hipStream_t s);
// Reduces the partials of up to two clouds into out: [lo[64], hi[64]] floats,
// mass[2] doubles, bad[2] ints.
hipError_t launch_bbox_final(const float *plo, const float *phi, const double *pmass,
                             const int *pbad, int nb0, int nb1, int d, float *lohi, double *mass,
                             int *bad, hipStream_t s);

// Packs a cloud: P[i] = x_i - centre (computed in FP64, rounded once), zero
// padded to KP; hn[i] = |P_i|^2 / 2; lw[i] = log w_i (-inf for w_i = 0).
hipError_t launch_pack(const float *x, const float *w, int64_t n, int d, int kp,
                       const float *centre, float *P, float *hn, float *lw, hipStream_t s);

// u_j = log2(e) * (lw_j + (h_j - hn_j) / eps)  (h may be NULL: zero potential).
hipError_t launch_col_offsets(const float *lw, const float *h, const float *hn, int64_t n,
                              double eps, float *u, hipStream_t s);

// Merges the chunk partials of one softmin into
//   out_i = lam * (hn_i - eps * ln2 * L2_i)      (+inf when the row has no mass).
hipError_t launch_softmin_finish(const float2 *part, int n_chunks, int64_t n, const float *hn,
                                 double eps, double lam, float *out, hipStream_t s);

// One cloud's side of an iteration: merges the partials of its two softmins
// (self problem -> s, cross problem -> c), optionally accumulates the
// marginal-error sums, averages, and writes the next column offsets.
struct FinishSide {
    const float2 *part_self;  // partials of the self problem (p~ or q~)
    const float2 *part_cross; // partials of the cross problem (f~ or g~)
    int chunks_self, chunks_cross;
    int64_t n;
    const float *hn, *lw, *w;
    float *pot_self, *pot_cross;  // p, f (cloud x) or q, g (cloud y): read, then averaged
    float *u_self, *u_cross;      // next column offsets for the problems that read this cloud
};
// acc: per-block FP64 partials, 4 doubles per block per side:
// [|r-t| cross, t cross, |r-t| self, t self].
int finish_blocks(int64_t n);
hipError_t launch_iteration_finish(const FinishSide &sx, const FinishSide &sy, double eps,
                                   double lam, double rho, int balanced, double eps_next,
                                   int check, double *acc, hipStream_t s);

// Sums W doubles over nb blocks of partials (row-major nb x W) in a fixed
// order into out[W].
hipError_t launch_sum_partials(const double *part, int nb, int W, double *out, hipStream_t s);

// Per-block FP64 partials of eq. (6): the a-side and b-side terms.
hipError_t launch_divergence_terms(const float *a, const float *f, const float *p, int64_t n,
                                   const float *b, const float *g, const float *q, int64_t m,
                                   double rho, int balanced, double *part, int *nb_out,
                                   hipStream_t s);
hipError_t launch_divergence_segments(const float *a, const float *f, const float *p,
                                      const int64_t *xo, const float *b, const float *g,
                                      const float *q, const int64_t *yo, int K, double rho,
                                      int balanced, double *out, hipStream_t s);

// ---- Learned warm start (set encoder over K-means cluster tokens) ----
constexpr int kWsIn = 64;      // token features
constexpr int kWsWidth = 256;  // hidden width
constexpr int kWsOut = 2;      // (cross dual, self dual) / blur^2 per cluster

// Strided GEMM with a fused epilogue, see warmstart.hip.
struct GemmArgs {
    const float *A;
    int64_t a_m, a_k;
    const float *B;
    int64_t b_k, b_n;
    float *C;
    int64_t ldc;
    int M, N, K;
    const float *bias;   // [N] or NULL
    const float *G;      // group term rows (stride ldg) or NULL
    int64_t ldg;
    const int *grp;      // group of each output row (divided by grp_div)
    int grp_div;
    const float *rs;     // per-row scale of the group term or NULL
    const float *mask;   // zero the output where mask <= 0 (stride ldm) or NULL
    int64_t ldm;
    int relu;
};
hipError_t launch_gemm(const GemmArgs &g, bool bf16, hipStream_t s);
size_t colsum_part_len(int N);
hipError_t launch_colsum(const float *A, int M, int N, int64_t ld, float *part, float *out,
                         hipStream_t s);
hipError_t launch_segsum(const float *X, const int *off, int stride, int n_seg, const float *w,
                         int normalise, float *out, double *wsum, hipStream_t s);
hipError_t launch_token_index(const int *off, int n_seg, const float *w, const double *wsum, int T,
                              int *seg, float *share, float *lw, hipStream_t s);
hipError_t launch_head(const float *a4, const float *W5, const float *b5, int T, const float *target,
                       const float *lw, float *y, float *dy, double *tl, hipStream_t s);
hipError_t launch_head_bwd(const float *dy, const float *W5, const float *a4, int T, float *da4,
                           hipStream_t s);
hipError_t launch_sum_f64(const double *v, int n, double *out, hipStream_t s);
hipError_t launch_adam(int64_t n, float *theta, const float *grad, float *m, float *v, double lr,
                       double b1, double b2, int step, double eps, hipStream_t s);
hipError_t launch_tokens(const float *C, const float *cm, const float *rad, int k, int kp, int d,
                         double total, double scale, int side, float *tok, float *tw, hipStream_t s);
hipError_t launch_cluster_means(const int *perm, const int *off, const float *w, const float *p0,
                                const float *p1, int k, double scale, float *out, hipStream_t s);
hipError_t launch_expand(const int *lab, int64_t n, const float *pred, int k, double scale, float *p0,
                         float *p1, int *bad, hipStream_t s);
hipError_t launch_labels_from_perm(const int *perm, const int *off, int k, int *lab, hipStream_t s);
hipError_t launch_nonfinite(const float *v, int64_t n, int *bad, hipStream_t s);
hipError_t launch_check_labels(const int *lab, int n, int k, int *bad, hipStream_t s);
// The clustering of run_kmeans from given labels in [0, k): sort, means, radii.
hipError_t clusters_from_labels(const float *X, const float *w, int n, int kp, int k,
                                const int *labels, float *C, float *cmass, float *radius, int *ws,
                                int **perm_out, int **off_out, hipStream_t s);
// Stable counting sort of the labels in ws[0, n) (K-means workspace layout).
hipError_t sort_labels(int n, int k, int *ws, int **perm_out, int **off_out, hipStream_t s);

}  // namespace skh
