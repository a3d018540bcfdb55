/*
 * Test infrastructure: a standalone driver that runs every oracle entry point
 * on small seeded problems, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by the CPU test suite (heap overflows, use of
 * freed memory, leaks and undefined arithmetic in the oracle fail the run).
 * It links otgs_oracle.c directly and checks a few invariants of its own:
 * Algorithm 2 equals the dense gradient, and the gap identity of the
 * duality at the solve's point.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ns, nt, L;
    const double *C;
    const int *labels;
    const double *a;
    const double *b;
    double gamma, mu;
} orc_problem;
typedef struct {
    double *alpha_s, *beta_s;
    double *Zs, *Os, *Ks;
    unsigned char *inN;
    long long s_i, s_n, s_u, s_r;
} orc_screen_state;
typedef struct {
    int max_iter, hist, r, use_screen, use_lower, max_ls;
    double c1, c2, gtol;
    int nthreads;
} orc_solve_opts;
typedef struct {
    int max_iter, r, use_screen, use_lower, max_bt;
    double gtol, shrink;
    int momentum;
} orc_agd_opts;
typedef struct {
    int iters, evals, status;
    double obj, gnorm_inf;
    long long s_i, s_n, s_u, s_r;
} orc_solve_info;

int orc_dual_grad(const orc_problem *, const double *, const double *, double *, double *, double *, double *);
int orc_dual_grad_par(const orc_problem *, const double *, const double *, double *, double *, double *, int);
int orc_plan(const orc_problem *, const double *, const double *, double *);
double orc_primal(const orc_problem *, const double *);
int orc_group_norms(const orc_problem *, const double *, const double *, double *, double *, double *);
int orc_upper_bound(const orc_problem *, const double *, const double *, const double *, const double *,
                    const double *, double *);
int orc_lower_bound(const orc_problem *, const double *, const double *, const double *, const double *,
                    const double *, const double *, double *);
int orc_gradpsi(const orc_problem *, orc_screen_state *, const double *, const double *, double *, double *, double *);
int orc_extract(const orc_problem *, orc_screen_state *, const double *, const double *);
int orc_snapshot(const orc_problem *, orc_screen_state *, const double *, const double *);
int orc_solve(const orc_problem *, const orc_solve_opts *, double *, double *, orc_solve_info *, double *);
int orc_agd_solve(const orc_problem *, const orc_agd_opts *, double *, double *, orc_solve_info *, double *);
void orc_cost_sqeuclid(int, int, int, const double *, const double *, double *);

static unsigned long long rng_state = 88172645463325252ull;
static double urand(void) {   /* xorshift64, uniform in [0, 1) */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int ns, int nt, int L, int d, double gamma, double mu, int empty_label) {
    double *xs = malloc(sizeof(double) * ns * d), *xt = malloc(sizeof(double) * nt * d);
    double *C = malloc(sizeof(double) * ns * nt);
    int *lab = malloc(sizeof(int) * ns);
    double *a = malloc(sizeof(double) * ns), *b = malloc(sizeof(double) * nt);
    for (int i = 0; i < ns * d; ++i) xs[i] = urand();
    for (int i = 0; i < nt * d; ++i) xt[i] = urand() + 0.2;
    for (int i = 0; i < ns; ++i) lab[i] = (int)(urand() * L) % L;
    if (empty_label) for (int i = 0; i < ns; ++i) if (lab[i] == 1) lab[i] = 0;
    for (int i = 0; i < ns; ++i) a[i] = 1.0 / ns;
    for (int j = 0; j < nt; ++j) b[j] = 1.0 / nt;
    orc_cost_sqeuclid(ns, nt, d, xs, xt, C);
    double cmax = 0;
    for (int i = 0; i < ns * nt; ++i) cmax = fmax(cmax, C[i]);
    for (int i = 0; i < ns * nt; ++i) C[i] /= cmax;
    orc_problem P = {ns, nt, L, C, lab, a, b, gamma, mu};
    double *al = calloc(ns, sizeof(double)), *be = calloc(nt, sizeof(double));
    double *ga = malloc(sizeof(double) * ns), *gb = malloc(sizeof(double) * nt);
    double *ga2 = malloc(sizeof(double) * ns), *gb2 = malloc(sizeof(double) * nt);
    double *T = malloc(sizeof(double) * ns * nt);
    size_t LN = (size_t)L * nt;
    double *Z = malloc(sizeof(double) * LN), *O = malloc(sizeof(double) * LN), *K = malloc(sizeof(double) * LN);
    double *ub = malloc(sizeof(double) * LN), *lb = malloc(sizeof(double) * LN);
    orc_solve_opts o = {300, 10, 10, 1, 1, 40, 1e-4, 0.9, 0.0, 0};
    orc_solve_info inf;
    double *trace = malloc(sizeof(double) * (o.max_iter + 1));
    int bad = 0;
    bad |= orc_solve(&P, &o, al, be, &inf, trace) != 0;
    {
        /* accelerated ascent, screened: reaches the L-BFGS value, monotone */
        orc_agd_opts oa = {300, 10, 1, 1, 60, 0.0, 0.8, 1};
        orc_solve_info ia;
        double *a2 = calloc(ns, sizeof(double)), *b2 = calloc(nt, sizeof(double));
        double *tr2 = malloc(sizeof(double) * (oa.max_iter + 1));
        bad |= orc_agd_solve(&P, &oa, a2, b2, &ia, tr2) != 0;
        for (int k = 0; k < ia.iters; ++k) bad |= tr2[k + 1] < tr2[k];
        bad |= ia.obj > inf.obj + 1e-9 * (1 + fabs(inf.obj));
        free(a2); free(b2); free(tr2);
    }
    double D, D2;
    bad |= orc_dual_grad(&P, al, be, ga, gb, &D, T) != 0;
    bad |= orc_dual_grad_par(&P, al, be, ga2, gb2, &D2, 2) != 0;
    bad |= memcmp(ga, ga2, sizeof(double) * ns) != 0 || D != D2;
    double Pv = orc_primal(&P, T), gap = 0;
    for (int i = 0; i < ns; ++i) gap += al[i] * ga[i];
    for (int j = 0; j < nt; ++j) gap += be[j] * gb[j];
    bad |= fabs((Pv - D) + gap) > 1e-9 * (1 + fabs(D));
    bad |= orc_plan(&P, al, be, T) != 0;
    bad |= orc_group_norms(&P, al, be, Z, O, K) != 0;
    orc_screen_state S;
    S.alpha_s = calloc(ns, sizeof(double));
    S.beta_s = calloc(nt, sizeof(double));
    S.Zs = calloc(LN, sizeof(double));
    S.Os = calloc(LN, sizeof(double));
    S.Ks = calloc(LN, sizeof(double));
    S.inN = calloc(LN, 1);
    S.s_i = S.s_n = S.s_u = S.s_r = 0;
    bad |= orc_snapshot(&P, &S, al, be) != 0;
    for (int i = 0; i < ns; ++i) al[i] += 1e-3 * (urand() - 0.5);
    bad |= orc_upper_bound(&P, al, be, S.alpha_s, S.beta_s, S.Zs, ub) != 0;
    bad |= orc_lower_bound(&P, al, be, S.alpha_s, S.beta_s, S.Ks, S.Os, lb) != 0;
    bad |= orc_extract(&P, &S, al, be) != 0;
    bad |= orc_gradpsi(&P, &S, al, be, ga2, gb2, &D2) != 0;
    bad |= orc_dual_grad(&P, al, be, ga, gb, &D, NULL) != 0;
    for (int i = 0; i < ns; ++i) bad |= fabs(ga[i] - ga2[i]) > 1e-13;
    bad |= fabs(D - D2) > 1e-13 * (1 + fabs(D));
    printf("case ns=%d nt=%d L=%d: D=%.12g iters=%d status=%d %s\n", ns, nt, L, inf.obj, inf.iters, inf.status,
           bad ? "FAILED" : "ok");
    free(S.alpha_s); free(S.beta_s); free(S.Zs); free(S.Os); free(S.Ks); free(S.inN);
    free(xs); free(xt); free(C); free(lab); free(a); free(b); free(al); free(be); free(ga); free(gb);
    free(ga2); free(gb2); free(T); free(Z); free(O); free(K); free(ub); free(lb); free(trace);
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= run_case(40, 30, 4, 3, 0.5, 0.3, 0);
    bad |= run_case(23, 57, 5, 2, 0.2, 0.8, 1);
    bad |= run_case(1, 9, 1, 2, 1.0, 0.1, 0);
    bad |= run_case(12, 1, 3, 4, 0.7, 0.0, 0);
    return bad ? 1 : 0;
}
