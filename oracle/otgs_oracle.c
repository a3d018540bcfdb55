/*
 * FP64 CPU oracle for smooth-dual optimal transport with the squared-L2 plus
 * group-lasso regulariser (Ida et al., "Fast Regularized Discrete Optimal
 * Transport with Group-Sparse Regularizers", AAAI 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or constant with the
 * HIP library.
 *
 * Conventions: n_src labelled source rows (the paper's m), n_tgt target
 * columns (the paper's n); C is row-major [n_src x n_tgt]; labels in
 * [0, L); groups are the sets of rows sharing a label, in ascending row
 * order.  Everything is double precision.
 *
 * Functions and the passages they follow:
 *   orc_cost_sqeuclid  - c_ij = ||x_i - y_j||^2            (Sec. 2.1)
 *   orc_dual_grad      - D(alpha, beta) of the smooth relaxed dual (Eq. 4)
 *   orc_dual_grad_par  - the same values, bit for bit, computed by OpenMP
 *                        threads over target columns (used to time the
 *                        definition on every host core)
 *                        and its gradient; per column j and group l the
 *                        block of grad psi is the group soft-threshold of
 *                        [f]_+ / gamma (Eq. 5, rewritten with z_lj as in
 *                        Sec. 3.2); psi itself uses its closed form
 *                        sum_l [z_l - mu gamma]_+^2 / (2 gamma).
 *   orc_plan           - t_j = grad psi(alpha + beta_j 1 - c_j)   (Sec. 2.3)
 *   orc_primal         - <T, C> + sum_j Psi(t_j)               (Eqs. 2-3)
 *   orc_group_norms    - z_lj, o_lj = ||[f]_-||, k_lj = ||f|| (Defs. 1-2)
 *   orc_upper_bound    - Eq. 6 (Def. 1)
 *   orc_lower_bound    - Eq. 7 (Def. 2)
 *   orc_gradpsi        - Algorithm 2 (skip / extract gradient evaluation)
 *   orc_extract        - Algorithm 1, construction of the set N (Eq. 8)
 *   orc_solve          - Algorithm 1 driving limited-memory BFGS (Liu and
 *                        Nocedal) with a strong-Wolfe line search; with
 *                        screening off it is the original dense method.
 *   orc_agd_solve      - Algorithm 1 driving another first-order solver
 *                        (the screening's solver-independence, Theorem 1
 *                        and its remark in Sec. 3.4): accelerated gradient
 *                        ascent (Nesterov's momentum in the FISTA form of
 *                        Beck and Teboulle) with backtracking on the
 *                        step and the function-value restart of
 *                        O'Donoghue and Candes, in variables scaled by the
 *                        marginals.  The paper fixes no such solver; its
 *                        steps are stated with the function.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ns, nt, L;
    const double *C;     /* [ns*nt] */
    const int *labels;   /* [ns] */
    const double *a;     /* [ns] */
    const double *b;     /* [nt] */
    double gamma, mu;
} orc_problem;

/* group membership in ascending row order */
typedef struct {
    int L;
    int *off;   /* [L+1] */
    int *rows;  /* [ns] */
} groups_t;

static int groups_build(const orc_problem *P, groups_t *G) {
    G->L = P->L;
    G->off = (int *)calloc((size_t)P->L + 1, sizeof(int));
    G->rows = (int *)malloc(sizeof(int) * (size_t)(P->ns > 0 ? P->ns : 1));
    if (!G->off || !G->rows) return -1;
    for (int i = 0; i < P->ns; ++i) {
        int l = P->labels[i];
        if (l < 0 || l >= P->L) return -2;
        G->off[l + 1]++;
    }
    for (int l = 0; l < P->L; ++l) G->off[l + 1] += G->off[l];
    int *fill = (int *)calloc((size_t)P->L, sizeof(int));
    if (!fill) return -1;
    for (int i = 0; i < P->ns; ++i) {
        int l = P->labels[i];
        G->rows[G->off[l] + fill[l]++] = i;
    }
    free(fill);
    return 0;
}

static void groups_free(groups_t *G) {
    free(G->off);
    free(G->rows);
}

/* Neumaier-compensated running sum */
typedef struct { double s, c; } ksum_t;
static inline void kadd(ksum_t *k, double x) {
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}
static inline double kval(const ksum_t *k) { return k->s + k->c; }

/* ------------------------------------------------------------------ cost */

void orc_cost_sqeuclid(int ns, int nt, int d, const double *xs, const double *xt,
                       double *C) {
    for (int i = 0; i < ns; ++i)
        for (int j = 0; j < nt; ++j) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) {
                double t = xs[(size_t)i * d + k] - xt[(size_t)j * d + k];
                s += t * t;
            }
            C[(size_t)i * nt + j] = s;
        }
}

/* ------------------------------------------------ dense gradient (Eq. 4-5) */

/* One column j, one group: soft-threshold block.  Writes the column block
 * of T into rowacc (added) and returns the column sum, adds psi to *psi. */
static double group_block(const orc_problem *P, const groups_t *G, int l, int j,
                          const double *alpha, const double *beta,
                          double *rowacc, double *psi, double *Tcol /* or NULL */) {
    const double thr = P->mu * P->gamma;
    double z2 = 0.0;
    for (int q = G->off[l]; q < G->off[l + 1]; ++q) {
        int i = G->rows[q];
        double f = alpha[i] + beta[j] - P->C[(size_t)i * P->nt + j];
        double p = f > 0.0 ? f : 0.0;
        z2 += p * p;
    }
    double z = sqrt(z2);
    if (!(z > thr)) return 0.0;           /* zero block when z <= mu*gamma */
    double kappa = (z - thr) / (P->gamma * z);
    double col = 0.0;
    for (int q = G->off[l]; q < G->off[l + 1]; ++q) {
        int i = G->rows[q];
        double f = alpha[i] + beta[j] - P->C[(size_t)i * P->nt + j];
        double t = f > 0.0 ? kappa * f : 0.0;
        rowacc[i] += t;
        col += t;
        if (Tcol) Tcol[(size_t)i * P->nt + j] = t;
    }
    *psi += (z - thr) * (z - thr) / (2.0 * P->gamma);
    return col;
}

static double dual_linear(const orc_problem *P, const double *alpha, const double *beta) {
    ksum_t k = {0, 0};
    for (int i = 0; i < P->ns; ++i) kadd(&k, alpha[i] * P->a[i]);
    for (int j = 0; j < P->nt; ++j) kadd(&k, beta[j] * P->b[j]);
    return kval(&k);
}

int orc_dual_grad(const orc_problem *P, const double *alpha, const double *beta,
                  double *grad_a, double *grad_b, double *obj, double *T) {
    groups_t G;
    int rc = groups_build(P, &G);
    if (rc) { groups_free(&G); return rc; }
    double *rowacc = (double *)calloc((size_t)P->ns + 1, sizeof(double));
    if (T) memset(T, 0, sizeof(double) * (size_t)P->ns * P->nt);
    ksum_t psi_tot = {0, 0};
    for (int j = 0; j < P->nt; ++j) {
        double col = 0.0, psi = 0.0;
        for (int l = 0; l < P->L; ++l)
            col += group_block(P, &G, l, j, alpha, beta, rowacc, &psi, T);
        if (grad_b) grad_b[j] = P->b[j] - col;
        kadd(&psi_tot, psi);
    }
    if (grad_a)
        for (int i = 0; i < P->ns; ++i) grad_a[i] = P->a[i] - rowacc[i];
    if (obj) *obj = dual_linear(P, alpha, beta) - kval(&psi_tot);
    free(rowacc);
    groups_free(&G);
    return 0;
}

/* orc_dual_grad with the columns shared among `nthreads` OpenMP threads (0:
 * the runtime's default).  Pass 1 takes the columns: every block's norm,
 * soft-threshold factor kappa, column sum and psi (the same arithmetic as
 * group_block); pass 2 takes the rows: each row adds its entries of T over
 * the columns in ascending order, the order orc_dual_grad adds them in, so
 * the results are identical. */
int orc_dual_grad_par(const orc_problem *P, const double *alpha, const double *beta,
                      double *grad_a, double *grad_b, double *obj, int nthreads) {
    groups_t G;
    int rc = groups_build(P, &G);
    if (rc) { groups_free(&G); return rc; }
    const double thr = P->mu * P->gamma;
    const int nt = P->nt, L = P->L;
    double *kap = (double *)calloc((size_t)L * nt + 1, sizeof(double));
    double *col = (double *)calloc((size_t)nt + 1, sizeof(double));
    double *psi = (double *)calloc((size_t)nt + 1, sizeof(double));
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nt; ++j) {
        double cj = 0.0, pj = 0.0;
        for (int l = 0; l < L; ++l) {
            double z2 = 0.0;
            for (int q = G.off[l]; q < G.off[l + 1]; ++q) {
                int i = G.rows[q];
                double f = alpha[i] + beta[j] - P->C[(size_t)i * nt + j];
                double p = f > 0.0 ? f : 0.0;
                z2 += p * p;
            }
            double z = sqrt(z2);
            if (!(z > thr)) continue;
            double kappa = (z - thr) / (P->gamma * z);
            double cl = 0.0;
            for (int q = G.off[l]; q < G.off[l + 1]; ++q) {
                int i = G.rows[q];
                double f = alpha[i] + beta[j] - P->C[(size_t)i * nt + j];
                cl += f > 0.0 ? kappa * f : 0.0;
            }
            cj += cl;
            pj += (z - thr) * (z - thr) / (2.0 * P->gamma);
            kap[(size_t)l * nt + j] = kappa;
        }
        col[j] = cj;
        psi[j] = pj;
    }
    if (grad_a) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < P->ns; ++i) {
            const double *kl = kap + (size_t)P->labels[i] * nt;
            double r = 0.0;
            for (int j = 0; j < nt; ++j) {
                if (!(kl[j] > 0.0)) continue;
                double f = alpha[i] + beta[j] - P->C[(size_t)i * nt + j];
                r += f > 0.0 ? kl[j] * f : 0.0;
            }
            grad_a[i] = P->a[i] - r;
        }
    }
    ksum_t psi_tot = {0, 0};
    for (int j = 0; j < nt; ++j) {
        if (grad_b) grad_b[j] = P->b[j] - col[j];
        kadd(&psi_tot, psi[j]);
    }
    if (obj) *obj = dual_linear(P, alpha, beta) - kval(&psi_tot);
    free(kap); free(col); free(psi);
    groups_free(&G);
    return 0;
}

int orc_plan(const orc_problem *P, const double *alpha, const double *beta, double *T) {
    return orc_dual_grad(P, alpha, beta, NULL, NULL, NULL, T);
}

double orc_primal(const orc_problem *P, const double *T) {
    groups_t G;
    if (groups_build(P, &G)) { groups_free(&G); return NAN; }
    ksum_t tot = {0, 0};
    for (int j = 0; j < P->nt; ++j) {
        double sq = 0.0, grp = 0.0;
        for (int l = 0; l < P->L; ++l) {
            double g2 = 0.0;
            for (int q = G.off[l]; q < G.off[l + 1]; ++q) {
                int i = G.rows[q];
                double t = T[(size_t)i * P->nt + j];
                kadd(&tot, t * P->C[(size_t)i * P->nt + j]);
                g2 += t * t;
            }
            sq += g2;
            grp += sqrt(g2);
        }
        kadd(&tot, P->gamma * (0.5 * sq + P->mu * grp));
    }
    groups_free(&G);
    return kval(&tot);
}

/* ------------------------------------------------ group norms and bounds */

/* z_lj = ||[f_[l]]_+||, o_lj = ||[f_[l]]_-||, k_lj = ||f_[l]||, each [L x nt] */
int orc_group_norms(const orc_problem *P, const double *alpha, const double *beta,
                    double *Z, double *O, double *K) {
    groups_t G;
    int rc = groups_build(P, &G);
    if (rc) { groups_free(&G); return rc; }
    for (int l = 0; l < P->L; ++l)
        for (int j = 0; j < P->nt; ++j) {
            double zp = 0.0, zn = 0.0;
            for (int q = G.off[l]; q < G.off[l + 1]; ++q) {
                int i = G.rows[q];
                double f = alpha[i] + beta[j] - P->C[(size_t)i * P->nt + j];
                if (f > 0.0) zp += f * f; else zn += f * f;
            }
            size_t o = (size_t)l * P->nt + j;
            if (Z) Z[o] = sqrt(zp);
            if (O) O[o] = sqrt(zn);
            if (K) K[o] = sqrt(zp + zn);
        }
    groups_free(&G);
    return 0;
}

/* per-group norms of the change in alpha since the snapshot:
 * up = ||[d_[l]]_+||, dn = ||[d_[l]]_-||, all = ||d_[l]|| */
static void alpha_change_norms(const orc_problem *P, const groups_t *G,
                               const double *alpha, const double *alpha_s,
                               double *up, double *dn, double *all) {
    for (int l = 0; l < P->L; ++l) {
        double u = 0, n = 0;
        for (int q = G->off[l]; q < G->off[l + 1]; ++q) {
            int i = G->rows[q];
            double d = alpha[i] - alpha_s[i];
            if (d > 0) u += d * d; else n += d * d;
        }
        if (up) up[l] = sqrt(u);
        if (dn) dn[l] = sqrt(n);
        if (all) all[l] = sqrt(u + n);
    }
}

/* Eq. 6: zbar = z~ + ||[da_[l]]_+|| + sqrt(g_l) [db_j]_+ */
int orc_upper_bound(const orc_problem *P, const double *alpha, const double *beta,
                    const double *alpha_s, const double *beta_s, const double *Zs,
                    double *Zbar) {
    groups_t G;
    int rc = groups_build(P, &G);
    if (rc) { groups_free(&G); return rc; }
    double *up = (double *)malloc(sizeof(double) * (size_t)P->L);
    alpha_change_norms(P, &G, alpha, alpha_s, up, NULL, NULL);
    for (int l = 0; l < P->L; ++l) {
        double sg = sqrt((double)(G.off[l + 1] - G.off[l]));
        for (int j = 0; j < P->nt; ++j) {
            double db = beta[j] - beta_s[j];
            size_t o = (size_t)l * P->nt + j;
            Zbar[o] = Zs[o] + up[l] + sg * (db > 0 ? db : 0.0);
        }
    }
    free(up);
    groups_free(&G);
    return 0;
}

/* Eq. 7: zlow = k~ - ||da_[l]|| - sqrt(g_l)|db_j| - o~ - ||[da_[l]]_-|| - sqrt(g_l)|[db_j]_-| */
int orc_lower_bound(const orc_problem *P, const double *alpha, const double *beta,
                    const double *alpha_s, const double *beta_s, const double *Ks,
                    const double *Os, double *Zlow) {
    groups_t G;
    int rc = groups_build(P, &G);
    if (rc) { groups_free(&G); return rc; }
    double *dn = (double *)malloc(sizeof(double) * (size_t)P->L);
    double *all = (double *)malloc(sizeof(double) * (size_t)P->L);
    alpha_change_norms(P, &G, alpha, alpha_s, NULL, dn, all);
    for (int l = 0; l < P->L; ++l) {
        double sg = sqrt((double)(G.off[l + 1] - G.off[l]));
        for (int j = 0; j < P->nt; ++j) {
            double db = beta[j] - beta_s[j];
            double dbn = db < 0 ? -db : 0.0;
            size_t o = (size_t)l * P->nt + j;
            Zlow[o] = Ks[o] - all[l] - sg * fabs(db) - Os[o] - dn[l] - sg * dbn;
        }
    }
    free(dn);
    free(all);
    groups_free(&G);
    return 0;
}

/* ------------------------------------------------ Algorithms 1 and 2 */

typedef struct {
    double *alpha_s, *beta_s;   /* snapshot point */
    double *Zs, *Os, *Ks;       /* snapshot norms [L x nt] */
    unsigned char *inN;         /* set N as a mask [L x nt] */
    /* Theorem 1 counters */
    long long s_i;   /* pairs evaluated because they are in N */
    long long s_n;   /* pairs outside N whose upper bound was checked */
    long long s_u;   /* checked pairs that could not be skipped */
    long long s_r;   /* snapshot refreshes */
} orc_screen_state;

/* Algorithm 2: gradient of the dual with gradient blocks in N computed
 * directly, the others skipped when the upper bound shows they are zero. */
int orc_gradpsi(const orc_problem *P, orc_screen_state *S, const double *alpha,
                const double *beta, double *grad_a, double *grad_b, double *obj) {
    groups_t G;
    int rc = groups_build(P, &G);
    if (rc) { groups_free(&G); return rc; }
    const double thr = P->mu * P->gamma;
    double *rowacc = (double *)calloc((size_t)P->ns + 1, sizeof(double));
    double *up = (double *)malloc(sizeof(double) * (size_t)P->L);
    double *colacc = (double *)calloc((size_t)P->nt + 1, sizeof(double));
    double *psicol = (double *)calloc((size_t)P->nt + 1, sizeof(double));
    /* blocks in N: exact evaluation without a check */
    for (int j = 0; j < P->nt; ++j)
        for (int l = 0; l < P->L; ++l) {
            size_t o = (size_t)l * P->nt + j;
            if (!S->inN[o]) continue;
            S->s_i++;
            colacc[j] += group_block(P, &G, l, j, alpha, beta, rowacc, &psicol[j], NULL);
        }
    /* the rest: upper bound first */
    alpha_change_norms(P, &G, alpha, S->alpha_s, up, NULL, NULL);
    for (int j = 0; j < P->nt; ++j) {
        double db = beta[j] - S->beta_s[j];
        double dbp = db > 0 ? db : 0.0;
        for (int l = 0; l < P->L; ++l) {
            size_t o = (size_t)l * P->nt + j;
            if (S->inN[o]) continue;
            S->s_n++;
            double sg = sqrt((double)(G.off[l + 1] - G.off[l]));
            double zbar = S->Zs[o] + up[l] + sg * dbp;
            if (zbar <= thr) continue;                    /* block is zero */
            S->s_u++;
            colacc[j] += group_block(P, &G, l, j, alpha, beta, rowacc, &psicol[j], NULL);
        }
    }
    ksum_t psi_tot = {0, 0};
    for (int j = 0; j < P->nt; ++j) {
        if (grad_b) grad_b[j] = P->b[j] - colacc[j];
        kadd(&psi_tot, psicol[j]);
    }
    if (grad_a)
        for (int i = 0; i < P->ns; ++i) grad_a[i] = P->a[i] - rowacc[i];
    if (obj) *obj = dual_linear(P, alpha, beta) - kval(&psi_tot);
    free(rowacc); free(up); free(colacc); free(psicol);
    groups_free(&G);
    return 0;
}

/* Algorithm 1: rebuild N from lower bounds against the current snapshot */
int orc_extract(const orc_problem *P, orc_screen_state *S, const double *alpha,
                const double *beta) {
    size_t LN = (size_t)P->L * P->nt;
    double *Zl = (double *)malloc(sizeof(double) * LN);
    int rc = orc_lower_bound(P, alpha, beta, S->alpha_s, S->beta_s, S->Ks, S->Os, Zl);
    const double thr = P->mu * P->gamma;
    for (size_t o = 0; o < LN; ++o) S->inN[o] = (unsigned char)(Zl[o] > thr);
    free(Zl);
    return rc;
}

/* Algorithm 1, "update the snapshots": snapshot point and its group norms */
int orc_snapshot(const orc_problem *P, orc_screen_state *S, const double *alpha,
                 const double *beta) {
    memcpy(S->alpha_s, alpha, sizeof(double) * (size_t)P->ns);
    memcpy(S->beta_s, beta, sizeof(double) * (size_t)P->nt);
    S->s_r++;
    return orc_group_norms(P, alpha, beta, S->Zs, S->Os, S->Ks);
}

/* ------------------------------------------------ L-BFGS (minimises -D) */

typedef struct {
    int max_iter;       /* iterations (accepted steps) */
    int hist;           /* history size */
    int r;              /* snapshot / N refresh period (Algorithm 1) */
    int use_screen;     /* 0: original dense method, 1: Algorithms 1-2 */
    int use_lower;      /* 0: never build N (upper bounds only) */
    int max_ls;         /* evaluations per line search */
    double c1, c2;      /* strong-Wolfe constants */
    double gtol;        /* stop when ||grad||_inf <= gtol */
    int nthreads;       /* dense evaluations by orc_dual_grad_par with this many
                           threads (same values); 0: orc_dual_grad */
} orc_solve_opts;

typedef struct {
    int iters, evals, status;   /* status 0 max_iter, 1 converged, 2 line search failed */
    double obj, gnorm_inf;
    long long s_i, s_n, s_u, s_r;
} orc_solve_info;

typedef struct {
    const orc_problem *P;
    orc_screen_state *S;
    int use_screen;
    int evals;
    double *ga, *gb;
    int nthreads;
} evaluator_t;

/* F = -D, G = -grad D, x = [alpha; beta] */
static double eval_fg(evaluator_t *E, const double *x, double *g) {
    const orc_problem *P = E->P;
    double D;
    E->evals++;
    if (E->use_screen)
        orc_gradpsi(P, E->S, x, x + P->ns, E->ga, E->gb, &D);
    else if (E->nthreads > 0)
        orc_dual_grad_par(P, x, x + P->ns, E->ga, E->gb, &D, E->nthreads);
    else
        orc_dual_grad(P, x, x + P->ns, E->ga, E->gb, &D, NULL);
    for (int i = 0; i < P->ns; ++i) g[i] = -E->ga[i];
    for (int j = 0; j < P->nt; ++j) g[P->ns + j] = -E->gb[j];
    return -D;
}

static double vdot(const double *x, const double *y, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* Minimiser of the cubic interpolating (t0,f0,d0) and (t1,f1,d1), safeguarded
 * into the middle 80% of the interval; bisection when the cubic has no
 * usable minimiser (Nocedal and Wright, Sec. 3.5). */
static double cubic_step(double t0, double f0, double d0, double t1, double f1, double d1) {
    double lo = t0 < t1 ? t0 : t1, hi = t0 < t1 ? t1 : t0;
    double w = hi - lo;
    double d1c = d0 + d1 - 3.0 * (f0 - f1) / (t0 - t1);
    double disc = d1c * d1c - d0 * d1;
    double t = 0.5 * (lo + hi);
    if (disc >= 0.0) {
        double d2 = copysign(sqrt(disc), t1 - t0);
        double den = d1 - d0 + 2.0 * d2;
        if (den != 0.0) {
            double c = t1 - (t1 - t0) * (d1 + d2 - d1c) / den;
            if (isfinite(c)) t = c;
        }
    }
    if (t < lo + 0.1 * w || t > hi - 0.1 * w) t = 0.5 * (lo + hi);
    return t;
}

int orc_solve(const orc_problem *P, const orc_solve_opts *o, double *alpha, double *beta,
              orc_solve_info *info, double *obj_trace /* [max_iter+1] or NULL */) {
    const int n = P->ns + P->nt;
    const int h = o->hist;
    size_t LN = (size_t)P->L * P->nt;
    orc_screen_state S;
    memset(&S, 0, sizeof S);
    S.alpha_s = (double *)calloc((size_t)P->ns, sizeof(double));
    S.beta_s = (double *)calloc((size_t)P->nt, sizeof(double));
    S.Zs = (double *)calloc(LN, sizeof(double));
    S.Os = (double *)calloc(LN, sizeof(double));
    S.Ks = (double *)calloc(LN, sizeof(double));
    S.inN = (unsigned char *)calloc(LN, 1);
    evaluator_t E = {P, &S, o->use_screen, 0,
                     (double *)malloc(sizeof(double) * (size_t)P->ns),
                     (double *)malloc(sizeof(double) * (size_t)P->nt), o->nthreads};
    double *x = (double *)malloc(sizeof(double) * n);
    double *g = (double *)malloc(sizeof(double) * n);
    double *d = (double *)malloc(sizeof(double) * n);
    double *xt = (double *)malloc(sizeof(double) * n);
    double *gt = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    double *sk = (double *)malloc(sizeof(double) * (size_t)n * h);
    double *yk = (double *)malloc(sizeof(double) * (size_t)n * h);
    double *rho = (double *)malloc(sizeof(double) * h);
    double *al = (double *)malloc(sizeof(double) * h);
    memcpy(x, alpha, sizeof(double) * P->ns);
    memcpy(x + P->ns, beta, sizeof(double) * P->nt);
    /* Algorithm 1 initialisation: snapshot at the starting point, N empty */
    if (o->use_screen) orc_snapshot(P, &S, x, x + P->ns), S.s_r = 0;
    double f = eval_fg(&E, x, g);
    if (obj_trace) obj_trace[0] = -f;
    int count = 0, head = 0, it = 0, status = 0;
    for (it = 0; it < o->max_iter; ++it) {
        double ginf = 0.0;
        for (int i = 0; i < n; ++i) ginf = fmax(ginf, fabs(g[i]));
        if (ginf <= o->gtol) { status = 1; break; }
        /* two-loop recursion: d = -H g */
        memcpy(q, g, sizeof(double) * n);
        for (int c = 0; c < count; ++c) {
            int k = (head - 1 - c + h) % h;
            al[k] = rho[k] * vdot(sk + (size_t)k * n, q, n);
            for (int i = 0; i < n; ++i) q[i] -= al[k] * yk[(size_t)k * n + i];
        }
        if (count > 0) {
            int k = (head - 1 + h) % h;
            double yy = vdot(yk + (size_t)k * n, yk + (size_t)k * n, n);
            double hs = 1.0 / (rho[k] * yy);
            for (int i = 0; i < n; ++i) q[i] *= hs;
        }
        for (int c = count - 1; c >= 0; --c) {
            int k = (head - 1 - c + h) % h;
            double be = rho[k] * vdot(yk + (size_t)k * n, q, n);
            for (int i = 0; i < n; ++i) q[i] += (al[k] - be) * sk[(size_t)k * n + i];
        }
        for (int i = 0; i < n; ++i) d[i] = -q[i];
        double dphi0 = vdot(g, d, n);
        if (!(dphi0 < 0.0)) {          /* not a descent direction: restart */
            count = 0;
            for (int i = 0; i < n; ++i) d[i] = -g[i];
            dphi0 = vdot(g, d, n);
        }
        double t = 1.0;
        if (count == 0) t = 1.0 / sqrt(vdot(g, g, n));
        /* strong-Wolfe line search (Nocedal and Wright, Algorithms 3.5-3.6) */
        double t_prev = 0.0, f_prev = f, dp_prev = dphi0;
        double t_lo = 0, f_lo = 0, dp_lo = 0, t_hi = 0, f_hi = 0, dp_hi = 0;
        int zoom = 0, ok = 0, nls = 0;
        double f_new = f;
        while (nls < o->max_ls) {
            for (int i = 0; i < n; ++i) xt[i] = x[i] + t * d[i];
            f_new = eval_fg(&E, xt, gt);
            double dp = vdot(gt, d, n);
            ++nls;
            if (!zoom) {
                if (f_new > f + o->c1 * t * dphi0 || (nls > 1 && f_new >= f_prev)) {
                    zoom = 1; t_lo = t_prev; f_lo = f_prev; dp_lo = dp_prev;
                    t_hi = t; f_hi = f_new; dp_hi = dp;
                } else if (fabs(dp) <= -o->c2 * dphi0) {
                    ok = 1; break;
                } else if (dp >= 0.0) {
                    zoom = 1; t_lo = t; f_lo = f_new; dp_lo = dp;
                    t_hi = t_prev; f_hi = f_prev; dp_hi = dp_prev;
                } else {
                    t_prev = t; f_prev = f_new; dp_prev = dp;
                    t = 4.0 * t;  /* extrapolate */
                    continue;
                }
            } else {
                if (f_new > f + o->c1 * t * dphi0 || f_new >= f_lo) {
                    t_hi = t; f_hi = f_new; dp_hi = dp;
                } else {
                    if (fabs(dp) <= -o->c2 * dphi0) { ok = 1; break; }
                    if (dp * (t_hi - t_lo) >= 0.0) { t_hi = t_lo; f_hi = f_lo; dp_hi = dp_lo; }
                    t_lo = t; f_lo = f_new; dp_lo = dp;
                }
            }
            t = cubic_step(t_lo, f_lo, dp_lo, t_hi, f_hi, dp_hi);
        }
        if (!ok) { status = 2; break; }
        /* history update; skip pairs without positive curvature */
        double *sn = sk + (size_t)head * n, *yn = yk + (size_t)head * n;
        for (int i = 0; i < n; ++i) { sn[i] = t * d[i]; yn[i] = gt[i] - g[i]; }
        double sy = vdot(sn, yn, n);
        if (sy > 1e-10 * sqrt(vdot(sn, sn, n) * vdot(yn, yn, n))) {
            rho[head] = 1.0 / sy;
            head = (head + 1) % h;
            if (count < h) count++;
        }
        memcpy(x, xt, sizeof(double) * n);
        memcpy(g, gt, sizeof(double) * n);
        f = f_new;
        if (obj_trace) obj_trace[it + 1] = -f;
        /* Algorithm 1: every r iterations rebuild N, then refresh the snapshot */
        if (o->use_screen && (it + 1) % o->r == 0) {
            if (o->use_lower) orc_extract(P, &S, x, x + P->ns);
            orc_snapshot(P, &S, x, x + P->ns);
        }
    }
    memcpy(alpha, x, sizeof(double) * P->ns);
    memcpy(beta, x + P->ns, sizeof(double) * P->nt);
    if (info) {
        double ginf = 0.0;
        for (int i = 0; i < n; ++i) ginf = fmax(ginf, fabs(g[i]));
        info->iters = it; info->evals = E.evals; info->status = status;
        info->obj = -f; info->gnorm_inf = ginf;
        info->s_i = S.s_i; info->s_n = S.s_n; info->s_u = S.s_u; info->s_r = S.s_r;
    }
    free(S.alpha_s); free(S.beta_s); free(S.Zs); free(S.Os); free(S.Ks); free(S.inN);
    free(E.ga); free(E.gb); free(x); free(g); free(d); free(xt); free(gt); free(q);
    free(sk); free(yk); free(rho); free(al);
    return 0;
}

/* ------------------------------- accelerated gradient ascent (maximises D) */

typedef struct {
    int max_iter;       /* accepted steps */
    int r;              /* snapshot / N refresh period (Algorithm 1) */
    int use_screen, use_lower;
    int max_bt;         /* step halvings per iteration before giving up */
    double gtol;        /* stop when ||grad D||_inf <= gtol at an accepted point */
    double shrink;      /* L <- shrink L after every accepted step, in (0, 1] */
    int momentum;       /* 0: no extrapolation (plain gradient ascent with the
                           same step rule), for comparison */
} orc_agd_opts;

/* The method, in the variables u with x = w * u (x = [alpha; beta]),
 * w_e = 1 / sqrt(M m_e) for the marginal m_e of entry e (1 where it is 0)
 * and M = (n_src + n_tgt) / 2; q(u) = w * grad D(w * u) is the gradient in u.
 *   u_0 = x_0 / w, D_0 = D(x_0), L = ||q(u_0)||_2, v = u_0, t = 1.
 *   each iteration, with q_v = q(v) and D_v = D(w v):
 *     trial u+ = v + q_v / L; while D(w u+) < D_v + ||q_v||^2 / (2 L):
 *       L <- 2 L and a new trial (at most max_bt times, else stop: status 2);
 *     if D(w u+) < D_k and v is not u_k: restart (t = 1, v = u_k) and
 *       take the trial again from there;
 *     else accept: u_{k+1} = u+, t' = (1 + sqrt(1 + 4 t^2)) / 2,
 *       v = u_{k+1} + ((t - 1) / t') (u_{k+1} - u_k), t = t', L <- shrink L.
 * Accepted objectives never decrease: a trial from u_k itself gains at
 * least ||q||^2 / (2 L) >= 0.  With screening, every r accepted steps N is
 * rebuilt and the snapshot refreshed at the accepted point, as Algorithm 1
 * does for any solver. */
int orc_agd_solve(const orc_problem *P, const orc_agd_opts *o, double *alpha, double *beta,
                  orc_solve_info *info, double *obj_trace /* [max_iter+1] or NULL */) {
    const int ns = P->ns, n = P->ns + P->nt;
    size_t LN = (size_t)P->L * P->nt;
    orc_screen_state S;
    memset(&S, 0, sizeof S);
    S.alpha_s = (double *)calloc((size_t)P->ns, sizeof(double));
    S.beta_s = (double *)calloc((size_t)P->nt, sizeof(double));
    S.Zs = (double *)calloc(LN, sizeof(double));
    S.Os = (double *)calloc(LN, sizeof(double));
    S.Ks = (double *)calloc(LN, sizeof(double));
    S.inN = (unsigned char *)calloc(LN, 1);
    evaluator_t E = {P, &S, o->use_screen, 0,
                     (double *)malloc(sizeof(double) * (size_t)P->ns),
                     (double *)malloc(sizeof(double) * (size_t)P->nt), 0};
    double *w = (double *)malloc(sizeof(double) * n);
    double *u = (double *)malloc(sizeof(double) * n);      /* accepted point u_k */
    double *uprev = (double *)malloc(sizeof(double) * n);
    double *v = (double *)malloc(sizeof(double) * n);      /* extrapolated point */
    double *ut = (double *)malloc(sizeof(double) * n);     /* trial point */
    double *x = (double *)malloc(sizeof(double) * n);      /* w * (a point in u) */
    double *g = (double *)malloc(sizeof(double) * n);      /* -grad D at x */
    double *qk = (double *)malloc(sizeof(double) * n);     /* q at u_k */
    double *qv = (double *)malloc(sizeof(double) * n);     /* q at v */
    double *qt = (double *)malloc(sizeof(double) * n);     /* q at the trial */
    const double M = 0.5 * ((double)P->ns + (double)P->nt);
    for (int e = 0; e < n; ++e) {
        double m = e < ns ? P->a[e] : P->b[e - ns];
        w[e] = m > 0.0 ? 1.0 / sqrt(M * m) : 1.0;
    }
    for (int i = 0; i < ns; ++i) u[i] = alpha[i] / w[i];
    for (int j = 0; j < P->nt; ++j) u[ns + j] = beta[j] / w[ns + j];
    if (o->use_screen) orc_snapshot(P, &S, alpha, beta), S.s_r = 0;
    /* value and q at a point given in u */
#define AGD_EVAL(pt, qout, Dout)                                  \
    do {                                                          \
        for (int e = 0; e < n; ++e) x[e] = w[e] * (pt)[e];        \
        (Dout) = -eval_fg(&E, x, g);                              \
        for (int e = 0; e < n; ++e) (qout)[e] = -w[e] * g[e];     \
    } while (0)
    double Dk, Dv, Dt = 0.0;
    AGD_EVAL(u, qk, Dk);
    if (obj_trace) obj_trace[0] = Dk;
    double L = sqrt(vdot(qk, qk, n));
    memcpy(v, u, sizeof(double) * n);
    memcpy(qv, qk, sizeof(double) * n);
    Dv = Dk;
    int at_k = 1;        /* v is u_k */
    double t = 1.0;
    int it = 0, status = 0;
    while (it < o->max_iter) {
        double ginf = 0.0;
        for (int e = 0; e < n; ++e) ginf = fmax(ginf, fabs(qk[e] / w[e]));
        if (ginf <= o->gtol) { status = 1; break; }
        const double qq = vdot(qv, qv, n);
        int bt = 0, ok = 0;
        for (;;) {
            for (int e = 0; e < n; ++e) ut[e] = v[e] + qv[e] / L;
            AGD_EVAL(ut, qt, Dt);
            if (Dt >= Dv + qq / (2.0 * L)) { ok = 1; break; }
            if (++bt > o->max_bt) break;
            L *= 2.0;
        }
        if (!ok) { status = 2; break; }
        if (Dt < Dk && !at_k) {
            /* function-value restart: drop the momentum, step from u_k */
            t = 1.0;
            memcpy(v, u, sizeof(double) * n);
            memcpy(qv, qk, sizeof(double) * n);
            Dv = Dk;
            at_k = 1;
            continue;
        }
        memcpy(uprev, u, sizeof(double) * n);
        memcpy(u, ut, sizeof(double) * n);
        memcpy(qk, qt, sizeof(double) * n);
        Dk = Dt;
        ++it;
        if (obj_trace) obj_trace[it] = Dk;
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        const double mom = o->momentum ? (t - 1.0) / tn : 0.0;
        t = tn;
        L *= o->shrink;
        if (o->use_screen && it % o->r == 0) {
            for (int e = 0; e < n; ++e) x[e] = w[e] * u[e];
            if (o->use_lower) orc_extract(P, &S, x, x + ns);
            orc_snapshot(P, &S, x, x + ns);
        }
        if (mom == 0.0) {
            memcpy(v, u, sizeof(double) * n);
            memcpy(qv, qk, sizeof(double) * n);
            Dv = Dk;
            at_k = 1;
        } else {
            for (int e = 0; e < n; ++e) v[e] = u[e] + mom * (u[e] - uprev[e]);
            AGD_EVAL(v, qv, Dv);
            at_k = 0;
        }
    }
#undef AGD_EVAL
    for (int i = 0; i < ns; ++i) alpha[i] = w[i] * u[i];
    for (int j = 0; j < P->nt; ++j) beta[j] = w[ns + j] * u[ns + j];
    if (info) {
        double ginf = 0.0;
        for (int e = 0; e < n; ++e) ginf = fmax(ginf, fabs(qk[e] / w[e]));
        info->iters = it; info->evals = E.evals; info->status = status;
        info->obj = Dk; info->gnorm_inf = ginf;
        info->s_i = S.s_i; info->s_n = S.s_n; info->s_u = S.s_u; info->s_r = S.s_r;
    }
    free(S.alpha_s); free(S.beta_s); free(S.Zs); free(S.Os); free(S.Ks); free(S.inN);
    free(E.ga); free(E.gb); free(w); free(u); free(uprev); free(v); free(ut); free(x); free(g);
    free(qk); free(qv); free(qt);
    return 0;
}
