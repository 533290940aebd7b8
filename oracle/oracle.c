/*
 * FP64 CPU oracle for the symmetric, debiased Sinkhorn divergence of
 * Feydy, Roussillon, Trouve, Gori, "Fast and Scalable Optimal Transport for
 * Brain Tractograms" (MICCAI 2019, arXiv 2107.02010).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library; the two meet only through the seeded input generators.
 *
 * Everything is plain double precision, dense, O(N*M) per reduction, written
 * for a reader to check against the paper by eye.  Rows are spread over
 * OpenMP threads; each row is computed the same way whatever the thread
 * count, so results do not depend on it.
 *
 * Notation (Section 2 of the paper):
 *   alpha = sum_i a_i delta_{x_i}, beta = sum_j b_j delta_{y_j}, x, y in R^D.
 *   Cost C(x, y) = |x - y|^p / p, p = 2 unless stated (the entries with a
 *   suffix _p take p in [1, 2]); eps = sigma^p, rho = reach^p.
 *   Dual vectors returned by the symmetric loop (Algorithm, "Return"):
 *     f = b^{beta->alpha} (length N),  g = a^{alpha->beta} (length M),
 *     p = a^{alpha<->alpha} (length N), q = b^{beta<->beta} (length M).
 *   eps = sigma^p, rho = reach^p, lambda = 1 / (1 + eps / rho)  (Algorithm).
 *   reach <= 0 or reach = +inf means the balanced problem: lambda = 1 and the
 *   rho -> inf limits of eqs. (2), (3) and (6).
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - the diameter d = max |x_i - y_j| of the Algorithm is replaced by the
 *     diagonal of the joint axis-aligned bounding box, an upper bound that
 *     costs O(N + M);
 *   - the scale list [d, d q, d q^2, ..., blur] holds d q^k for
 *     k = 0 .. K-1 with K = ceil(log(d / blur) / log(1 / q)), then blur
 *     itself; if d <= blur the list is [blur];
 *   - the four softmins of one iteration all read the values from before the
 *     iteration (Jacobi order, as printed), then all four are averaged;
 *   - after the list, optional extra iterations at sigma = blur ("schedule
 *     mode"), or iterations at blur until the marginal error falls below a
 *     tolerance ("converged mode");
 *   - eq. (6) differences are evaluated as e^{-p/rho} expm1(-(f - p)/rho),
 *     an exact rewrite that keeps precision for large rho.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_INF (1.0 / 0.0)

/* Number of threads the OpenMP loops below use (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of threads of the OpenMP loops (k >= 1; no effect without
 * OpenMP).  Used to time the oracle on one core and on all cores. */
void oracle_set_num_threads(int k) {
#ifdef _OPENMP
    if (k >= 1) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

static int is_balanced(double reach) { return !(reach > 0.0) || isinf(reach); }

/* Cost C(x, y) = |x - y|^p / p (Section 2, the cost function), evaluated from
 * coordinate differences, never from norms; p = 2 is the default everywhere. */
static double cost_p(const double *x, const double *y, int d, double pexp) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = x[k] - y[k];
        s += t * t;
    }
    return pexp == 2.0 ? 0.5 * s : pow(s, 0.5 * pexp) / pexp;
}

static double cost(const double *x, const double *y, int d) { return cost_p(x, y, d, 2.0); }

/* sigma^p: eps from a scale, rho from the reach (the Algorithm's parameter lines) */
static double power_p(double v, double pexp) { return pexp == 2.0 ? v * v : pow(v, pexp); }

/* One softmin, the operation behind each of the four "tilde" updates of the
 * Algorithm:
 *     out_i = -lam * eps * log sum_j w_j exp((h_j - C(r_i, c_j)) / eps)
 * for rows r (n x d) against columns c (m x d) with weights w and potential h.
 * The log-sum-exp is taken with its maximum factored out.  Columns with zero
 * weight contribute nothing (log 0 = -inf); a row with no positive weight
 * gets +inf.  buf: scratch of m doubles per thread, allocated here. */
void oracle_softmin_p(int64_t n, int64_t m, int d, const double *r, const double *c,
                      const double *w, const double *h, double eps, double lam, double pexp,
                      double *out) {
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double mx = -OR_INF;
            for (int64_t j = 0; j < m; ++j) {
                if (w[j] > 0.0) {
                    s[j] = log(w[j]) + (h[j] - cost_p(r + i * d, c + j * d, d, pexp)) / eps;
                    if (s[j] > mx) mx = s[j];
                } else {
                    s[j] = -OR_INF;
                }
            }
            if (mx == -OR_INF) {
                out[i] = OR_INF;
                continue;
            }
            double sum = 0.0;
            for (int64_t j = 0; j < m; ++j)
                if (w[j] > 0.0) sum += exp(s[j] - mx);
            out[i] = -lam * eps * (mx + log(sum));
        }
        free(s);
    }
}

void oracle_softmin(int64_t n, int64_t m, int d, const double *r, const double *c,
                    const double *w, const double *h, double eps, double lam, double *out) {
    oracle_softmin_p(n, m, d, r, c, w, h, eps, lam, 2.0, out);
}

/* Diameter heuristic of the Algorithm's parameter line, read as the diagonal
 * of the joint bounding box of both clouds. */
double oracle_diameter(int64_t n, int64_t m, int d, const double *x, const double *y) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double lo = OR_INF, hi = -OR_INF;
        for (int64_t i = 0; i < n; ++i) {
            if (x[i * d + k] < lo) lo = x[i * d + k];
            if (x[i * d + k] > hi) hi = x[i * d + k];
        }
        for (int64_t j = 0; j < m; ++j) {
            if (y[j * d + k] < lo) lo = y[j * d + k];
            if (y[j * d + k] > hi) hi = y[j * d + k];
        }
        if (n + m > 0) s += (hi - lo) * (hi - lo);
    }
    return sqrt(s);
}

/* epsilon-scaling list of the Algorithm's loop header: d, d q, d q^2, ...,
 * blur.  Writes at most cap values; returns the length of the full list. */
int oracle_schedule(double diameter, double blur, double scaling, double *sigmas, int cap) {
    if (!(diameter > blur)) {
        if (cap > 0) sigmas[0] = blur;
        return 1;
    }
    int K = (int)ceil(log(diameter / blur) / log(1.0 / scaling));
    for (int k = 0; k < K; ++k)
        if (k < cap) sigmas[k] = diameter * pow(scaling, (double)k);
    if (K < cap) sigmas[K] = blur;
    return K + 1;
}

/* lambda of the Algorithm: 1 / (1 + eps / rho) = 1 / (1 + (sigma / reach)^p). */
static double damping(double sigma, double reach, double pexp) {
    if (is_balanced(reach)) return 1.0;
    double t = sigma / reach;
    return 1.0 / (1.0 + power_p(t, pexp));
}

/* Relative L1 error between a transport plan's row sums and their target.
 * Plan row sums follow from eq. (4) and the softmin just computed from the
 * same potentials:  (pi 1)_i = a_i exp((f_i - ft_i / lam) / eps).
 * Target: a_i exp(-f_i / rho), or a_i when balanced (first-order condition of
 * eq. (3)). */
static double marginal_error(int64_t n, const double *a, const double *f, const double *ft,
                             double eps, double lam, double reach, double pexp) {
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(a[i] > 0.0)) continue;
        double r = a[i] * exp((f[i] - ft[i] / lam) / eps);
        double t = is_balanced(reach) ? a[i] : a[i] * exp(-f[i] / power_p(reach, pexp));
        num += fabs(r - t);
        den += t;
    }
    return den > 0.0 ? num / den : 0.0;
}

/*
 * The symmetric, averaged Sinkhorn loop with epsilon-scaling (Algorithm).
 *   extra_iters: iterations at sigma = blur after the scale list.
 *   tol > 0: converged mode; after the list (and the extra iterations) keep
 *     iterating at sigma = blur until the marginal error (max over the four
 *     problems, checked every check_every iterations) is <= tol, at most
 *     max_iters further iterations.
 *   diameter <= 0: use oracle_diameter.
 *   f, g, p, q: in/out.  If init != 0 they hold the starting values,
 *     otherwise they are zeroed (Algorithm, first line).
 *   info (6 doubles, nullable): [iterations, scale-list length, last marginal
 *     error, diameter used, final eps, converged flag].
 * Returns the number of iterations run.
 */
int oracle_sinkhorn_p(int64_t n, int64_t m, int d, const double *x, const double *a,
                      const double *y, const double *b, double blur, double reach, double scaling,
                      double diameter, int extra_iters, double tol, int max_iters,
                      int check_every, int init, double pexp, double *f, double *g, double *p,
                      double *q, double *info) {
    if (!(diameter > 0.0)) diameter = oracle_diameter(n, m, d, x, y);
    int L = oracle_schedule(diameter, blur, scaling, NULL, 0);
    double *sig = (double *)malloc(sizeof(double) * (size_t)L);
    oracle_schedule(diameter, blur, scaling, sig, L);

    if (!init) {
        memset(f, 0, sizeof(double) * (size_t)n);
        memset(p, 0, sizeof(double) * (size_t)n);
        memset(g, 0, sizeof(double) * (size_t)m);
        memset(q, 0, sizeof(double) * (size_t)m);
    }
    double *ft = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double *pt = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double *gt = (double *)malloc(sizeof(double) * (size_t)(m ? m : 1));
    double *qt = (double *)malloc(sizeof(double) * (size_t)(m ? m : 1));

    int total = L + (extra_iters > 0 ? extra_iters : 0);
    int cap = total + (tol > 0.0 ? (max_iters > 0 ? max_iters : 0) : 0);
    if (check_every < 1) check_every = 1;
    double err = -1.0, eps = power_p(blur, pexp);
    int it = 0, converged = 0;
    for (; it < cap; ++it) {
        double sigma = it < L ? sig[it] : blur;
        eps = power_p(sigma, pexp);
        double lam = damping(sigma, reach, pexp);
        /* the four tilde updates, all from the values before this iteration */
        oracle_softmin_p(n, n, d, x, x, a, p, eps, lam, pexp, pt); /* a~^{alpha<->alpha}_i */
        oracle_softmin_p(m, m, d, y, y, b, q, eps, lam, pexp, qt); /* b~^{beta<->beta}_j  */
        oracle_softmin_p(m, n, d, y, x, a, f, eps, lam, pexp, gt); /* a~^{alpha->beta}_j  */
        oracle_softmin_p(n, m, d, x, y, b, g, eps, lam, pexp, ft); /* b~^{beta->alpha}_i  */
        int check = (it == cap - 1);
        if (tol > 0.0 && it >= total && ((it - total + 1) % check_every == 0)) check = 1;
        if (check) {
            double e1 = marginal_error(n, a, f, ft, eps, lam, reach, pexp);
            double e2 = marginal_error(m, b, g, gt, eps, lam, reach, pexp);
            double e3 = marginal_error(n, a, p, pt, eps, lam, reach, pexp);
            double e4 = marginal_error(m, b, q, qt, eps, lam, reach, pexp);
            err = fmax(fmax(e1, e2), fmax(e3, e4));
        }
        /* averaging step of the Algorithm */
        for (int64_t i = 0; i < n; ++i) {
            f[i] = 0.5 * (f[i] + ft[i]);
            p[i] = 0.5 * (p[i] + pt[i]);
        }
        for (int64_t j = 0; j < m; ++j) {
            g[j] = 0.5 * (g[j] + gt[j]);
            q[j] = 0.5 * (q[j] + qt[j]);
        }
        if (tol > 0.0 && check && err <= tol) {
            converged = 1;
            ++it;
            break;
        }
    }
    if (info) {
        info[0] = it;
        info[1] = L;
        info[2] = err;
        info[3] = diameter;
        info[4] = eps;
        info[5] = converged;
    }
    free(sig);
    free(ft);
    free(pt);
    free(gt);
    free(qt);
    return it;
}

int oracle_sinkhorn(int64_t n, int64_t m, int d, const double *x, const double *a, const double *y,
                    const double *b, double blur, double reach, double scaling, double diameter,
                    int extra_iters, double tol, int max_iters, int check_every, int init,
                    double *f, double *g, double *p, double *q, double *info) {
    return oracle_sinkhorn_p(n, m, d, x, a, y, b, blur, reach, scaling, diameter, extra_iters, tol,
                             max_iters, check_every, init, 2.0, f, g, p, q, info);
}

/* Sinkhorn divergence in dual form, eq. (6), at eps = blur^2:
 *   S = -(rho + eps/2) <a, e^{-f/rho} - e^{-p/rho}> - (rho + eps/2) <b, e^{-g/rho} - e^{-q/rho}>.
 * Balanced (rho -> inf): S = <a, f - p> + <b, g - q>. */
double oracle_divergence_p(int64_t n, int64_t m, const double *a, const double *b, const double *f,
                           const double *g, const double *p, const double *q, double blur,
                           double reach, double pexp) {
    double eps = power_p(blur, pexp);
    double s = 0.0;
    if (is_balanced(reach)) {
        for (int64_t i = 0; i < n; ++i) s += a[i] * (f[i] - p[i]);
        for (int64_t j = 0; j < m; ++j) s += b[j] * (g[j] - q[j]);
        return s;
    }
    double rho = power_p(reach, pexp);
    for (int64_t i = 0; i < n; ++i) s += a[i] * exp(-p[i] / rho) * expm1(-(f[i] - p[i]) / rho);
    for (int64_t j = 0; j < m; ++j) s += b[j] * exp(-q[j] / rho) * expm1(-(g[j] - q[j]) / rho);
    return -(rho + 0.5 * eps) * s;
}

double oracle_divergence(int64_t n, int64_t m, const double *a, const double *b, const double *f,
                         const double *g, const double *p, const double *q, double blur,
                         double reach) {
    return oracle_divergence_p(n, m, a, b, f, g, p, q, blur, reach, 2.0);
}

/* Dual objective of eq. (3) for OT_{eps,rho}(alpha, beta) at (f, g):
 *   rho <a, 1 - e^{-f/rho}> + rho <b, 1 - e^{-g/rho}>
 *   + eps <a (x) b, 1 - exp((f_i + g_j - C_ij) / eps)>.
 * Balanced: <a, f> + <b, g> + eps <a (x) b, 1 - exp(...)>. */
double oracle_ot_dual_p(int64_t n, int64_t m, int d, const double *x, const double *a,
                        const double *y, const double *b, const double *f, const double *g,
                        double eps, double reach, double pexp) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int bal = is_balanced(reach);
    double rho = bal ? 0.0 : power_p(reach, pexp);
    for (int64_t i = 0; i < n; ++i) s1 += bal ? a[i] * f[i] : rho * a[i] * (-expm1(-f[i] / rho));
    for (int64_t j = 0; j < m; ++j) s2 += bal ? b[j] * g[j] : rho * b[j] * (-expm1(-g[j] / rho));
#pragma omp parallel for reduction(+ : s3) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double r = 0.0;
        for (int64_t j = 0; j < m; ++j)
            r += a[i] * b[j] * (-expm1((f[i] + g[j] - cost_p(x + i * d, y + j * d, d, pexp)) / eps));
        s3 += r;
    }
    return s1 + s2 + eps * s3;
}

double oracle_ot_dual(int64_t n, int64_t m, int d, const double *x, const double *a, const double *y,
                      const double *b, const double *f, const double *g, double eps, double reach) {
    return oracle_ot_dual_p(n, m, d, x, a, y, b, f, g, eps, reach, 2.0);
}

/* KL(u, v) = sum u log(u / v) - u + v, with 0 log 0 = 0 (Section 2). */
static double kl_term(double u, double v) {
    if (u > 0.0) return u * log(u / v) - u + v;
    return v;
}

/* Primal objective of eq. (2) at the plan of eq. (4),
 *   pi_ij = a_i b_j exp((f_i + g_j - C_ij) / eps):
 *   <pi, C> + eps KL(pi, a (x) b) + rho KL(pi 1, a) + rho KL(pi^T 1, b).
 * Balanced: the two marginal terms are constraints and are left out. */
double oracle_ot_primal_p(int64_t n, int64_t m, int d, const double *x, const double *a,
                          const double *y, const double *b, const double *f, const double *g,
                          double eps, double reach, double pexp) {
    double *row = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    double *col = (double *)calloc((size_t)(m ? m : 1), sizeof(double));
    double lin = 0.0, ent = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double ab = a[i] * b[j];
            if (!(ab > 0.0)) continue;
            double c = cost_p(x + i * d, y + j * d, d, pexp);
            double pij = ab * exp((f[i] + g[j] - c) / eps);
            lin += pij * c;
            ent += kl_term(pij, ab);
            row[i] += pij;
            col[j] += pij;
        }
    }
    double s = lin + eps * ent;
    if (!is_balanced(reach)) {
        double rho = power_p(reach, pexp), k1 = 0.0, k2 = 0.0;
        for (int64_t i = 0; i < n; ++i) k1 += kl_term(row[i], a[i]);
        for (int64_t j = 0; j < m; ++j) k2 += kl_term(col[j], b[j]);
        s += rho * (k1 + k2);
    }
    free(row);
    free(col);
    return s;
}

double oracle_ot_primal(int64_t n, int64_t m, int d, const double *x, const double *a,
                        const double *y, const double *b, const double *f, const double *g,
                        double eps, double reach) {
    return oracle_ot_primal_p(n, m, d, x, a, y, b, f, g, eps, reach, 2.0);
}

/* Row and column sums of the plan of eq. (4). */
void oracle_marginals(int64_t n, int64_t m, int d, const double *x, const double *a, const double *y,
                      const double *b, const double *f, const double *g, double eps, double *row,
                      double *col) {
    for (int64_t j = 0; j < m; ++j) col[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        row[i] = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double pij = a[i] * b[j] * exp((f[i] + g[j] - cost(x + i * d, y + j * d, d)) / eps);
            row[i] += pij;
            col[j] += pij;
        }
    }
}

/* Plan applied to a value matrix V (m x L), from eq. (4):
 *   out_i = a_i sum_j b_j exp((f_i + g_j - C_ij) / eps) V_j.
 * With divide_by_a != 0 the a_i factor is left out, which is the soft label
 * of eq. (7). */
void oracle_plan_apply(int64_t n, int64_t m, int d, const double *x, const double *a,
                       const double *y, const double *b, const double *f, const double *g,
                       double eps, const double *V, int L, int divide_by_a, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int l = 0; l < L; ++l) out[i * L + l] = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double k = b[j] * exp((f[i] + g[j] - cost(x + i * d, y + j * d, d)) / eps);
            if (!divide_by_a) k *= a[i];
            for (int l = 0; l < L; ++l) out[i * L + l] += k * V[j * L + l];
        }
    }
}

/* Derivative of S with respect to the weight alpha_i, from the dual vectors.
 * The envelope theorem on the dual of eq. (3) gives, for OT(alpha, beta) at its
 * optimal (f, g), d/d alpha_i = rho (1 - e^{-f_i/rho}) + eps sum_j beta_j (1 -
 * exp((f_i + g_j - C_ij)/eps)); the optimality condition in f_i turns the sum
 * into eps (m_beta - e^{-f_i/rho}).  OT(alpha, alpha) carries alpha in both
 * slots (twice the same expression with p and m_alpha), and the mass term of
 * eq. (5) adds eps (m_alpha - m_beta); in S the mass terms cancel:
 *   dS/d alpha_i = (rho + eps) (e^{-p_i/rho} - e^{-f_i/rho}),
 * evaluated as -(rho + eps) e^{-p_i/rho} expm1(-(f_i - p_i)/rho).  Balanced
 * (rho -> infinity): f_i - p_i.  The same with (g, q) gives dS/d beta_j. */
void oracle_grad_weights(int64_t n, const double *f, const double *p, double blur, double reach,
                         double *out) {
    double eps = blur * blur;
    if (is_balanced(reach)) {
        for (int64_t i = 0; i < n; ++i) out[i] = f[i] - p[i];
        return;
    }
    double rho = reach * reach;
    for (int64_t i = 0; i < n; ++i) out[i] = -(rho + eps) * exp(-p[i] / rho) * expm1(-(f[i] - p[i]) / rho);
}

/* Gradient of S with respect to the positions x_i, by the envelope theorem
 * applied to eq. (3) at the optimal dual vectors (the paper states that the
 * gradients are expressions of the four dual vectors):
 *   grad_i = sum_j pi_ij (x_i - y_j) - sum_k pi^{aa}_ik (x_i - x_k),
 * with pi from (f, g) and pi^{aa} from (p, p), both by eq. (4), at eps. */
void oracle_grad_x(int64_t n, int64_t m, int d, const double *x, const double *a, const double *y,
                   const double *b, const double *f, const double *g, const double *p, double eps,
                   double *grad) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < d; ++k) grad[i * d + k] = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double pij = a[i] * b[j] * exp((f[i] + g[j] - cost(x + i * d, y + j * d, d)) / eps);
            for (int k = 0; k < d; ++k) grad[i * d + k] += pij * (x[i * d + k] - y[j * d + k]);
        }
        for (int64_t l = 0; l < n; ++l) {
            double pil = a[i] * a[l] * exp((p[i] + p[l] - cost(x + i * d, x + l * d, d)) / eps);
            for (int k = 0; k < d; ++k) grad[i * d + k] -= pil * (x[i * d + k] - x[l * d + k]);
        }
    }
}
