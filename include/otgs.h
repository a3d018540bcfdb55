/*
 * otgs.h - C ABI of the MI355X (gfx950) library for regularised discrete
 * optimal transport with a group-sparse regulariser (squared L2 plus group
 * lasso, one group per source class label).
 *
 * The problem (paper: Ida et al., AAAI 2023, Sec. 2): labelled source
 * samples x_i (i < n_src, label y_i), unlabelled target samples x_j
 * (j < n_tgt), cost c_ij = ||x_i - x_j||^2 (Sec. 2.1), marginals a, b, and
 *     min_{T in U(a,b)} <T,C> + sum_j Psi(t_j),
 *     Psi(t) = gamma (||t||^2 / 2 + mu sum_l ||t_[l]||)          (Eqs. 2-3).
 * The library works on the smooth relaxed dual (Eq. 4)
 *     D(alpha, beta) = a.alpha + b.beta - sum_j psi(alpha + beta_j 1 - c_j)
 * whose gradient blocks are the group soft threshold of Eq. 5:
 *     grad psi(f)_[l] = [1 - mu gamma / z_lj]_+ [f_[l]]_+ / gamma,
 *     z_lj = ||[f_[l]]_+||.
 * Note on names: the paper calls the source count m and the target count n;
 * this header says n_src and n_tgt.
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller, unless the
 *     comment says "host".  The library never frees caller memory.
 *   - All work is enqueued on the caller's HIP stream `stream` (a
 *     hipStream_t passed as void*; NULL is the default stream) and is
 *     asynchronous unless stated otherwise.
 *   - Arrays indexed by sample are in the caller's order.  For a handle with
 *     several instances ("batch"), per-sample arrays are the concatenation
 *     of the instances in order (instance k starts at the sum of the sizes
 *     of instances 0..k-1); per-instance scalars are arrays of length
 *     `count`.
 *   - Floating point: float32 storage and arithmetic, float64 for the dual
 *     objective accumulation and the L-BFGS dot products.
 *   - Return value: OT_GS_OK (0), a negative error code, or a positive
 *     warning.  On error nothing has been enqueued unless the code is
 *     OT_GS_EDEVICE.  ot_gs_last_error() gives a message (thread-local).
 *     No C++ exception crosses this interface.
 */
#ifndef OTGS_H
#define OTGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define OT_GS_OK              0
#define OT_GS_EINVAL         -1   /* invalid argument (sizes, gamma, mu, labels, NULL) */
#define OT_GS_ESHAPE         -2   /* inconsistent sizes between arguments            */
#define OT_GS_EDEVICE        -3   /* a HIP runtime call failed                        */
#define OT_GS_ENUMERIC       -4   /* NaN or Inf met in an input or the objective      */
#define OT_GS_ENOMEM         -5   /* device allocation failed                         */
#define OT_GS_EVERIFY        -6   /* a verified screened evaluation differed from the
                                     dense one at the same point (Lemma 2 violated)   */
#define OT_GS_NOT_CONVERGED   1   /* solve stopped at max_iter                        */
#define OT_GS_LINESEARCH      2   /* solve stopped: line search found no step         */

/* evaluation modes of ot_gs_dual_grad */
#define OT_GS_DENSE      0  /* every (group, target) block evaluated ("origin")         */
#define OT_GS_SCREENED   1  /* Algorithm 2: blocks in the set N evaluated directly,
                               others skipped when the upper bound of Eq. 6 shows
                               they are zero; needs a snapshot (see SNAPSHOT)          */
#define OT_GS_SNAPSHOT   2  /* dense evaluation that also records the snapshot
                               (alpha~, beta~, z~_lj, o~_lj) of Defs. 1-2 at this
                               point; the set N is first rebuilt from the lower bound
                               of Eq. 7 against the previous snapshot (Algorithm 1)   */
/* flags OR-ed into the mode of ot_gs_dual_grad (both make the call synchronous) */
#define OT_GS_CHECK    0x100  /* report NaN or Inf in this call's alpha, beta or in the
                                 objective as OT_GS_ENUMERIC                          */
#define OT_GS_VERIFY   0x200  /* with SCREENED or SNAPSHOT: evaluate densely at the same
                                 point as well and require bit-identical gradients and
                                 objective (every skipped block is zero, Lemma 2);
                                 OT_GS_EVERIFY otherwise.  Implies OT_GS_CHECK        */

/* cost providers */
#define OT_GS_COST_GIVEN       0  /* caller passes C [n_src x n_tgt] row-major        */
#define OT_GS_COST_MATERIALIZE 1  /* C = ||x_i - x_j||^2 built once from features    */
#define OT_GS_COST_ONTHEFLY    2  /* C tiles recomputed from features in every
                                     evaluation on FP32 matrix cores; never stored.
                                     c_ij = s max(|x_i|^2 + |x_j|^2 - 2 x_i.x_j, 0)
                                     with float32 norms and an FP32 dot product;
                                     1 <= dim <= 256; every instance of a handle
                                     must then use this mode                        */

typedef struct ot_gs_handle ot_gs_handle;

/* One OT instance.  All pointers are device pointers (caller-owned; they
 * need to stay valid only during ot_gs_create, which copies what it keeps). */
typedef struct {
    int n_src;             /* >= 1 labelled source samples (rows)                  */
    int n_tgt;             /* >= 1 target samples (columns)                        */
    int dim;               /* feature dimension (features only)                    */
    int n_groups;          /* labels lie in [0, n_groups); empty labels allowed    */
    const int32_t *labels; /* [n_src]                                              */
    int cost_mode;         /* OT_GS_COST_*                                         */
    const float *cost;     /* [n_src * n_tgt] row-major, C >= 0 (COST_GIVEN)       */
    const float *x_src;    /* [n_src * dim] row-major (COST_MATERIALIZE/ONTHEFLY)  */
    const float *x_tgt;    /* [n_tgt * dim] row-major                              */
    float cost_scale;      /* C is multiplied by this; 0 = 1 / max_ij C_ij (for
                              ONTHEFLY: of the unscaled float32 cost above)        */
    const float *a;        /* [n_src] source marginal, NULL = 1/n_src              */
    const float *b;        /* [n_tgt] target marginal, NULL = 1/n_tgt              */
    double gamma;          /* > 0; the kernels use float32 gamma in the soft
                              threshold and the threshold fl32(mu * gamma) (the
                              product formed in double, rounded once); the
                              objective uses gamma in double                     */
    double mu;             /* >= 0                                                  */
} ot_gs_problem;

/* Screening and timing counters, cumulative since create / last reset.
 * A tile is (group, 32 consecutive targets of the internal layout). */
typedef struct {
    long long evals;            /* gradient evaluations                               */
    long long pairs_total;      /* (group, target) blocks covered, summed over evals  */
    long long pairs_in_N;       /* blocks evaluated because they were in N   (s_i)    */
    long long pairs_checked;    /* blocks outside N whose upper bound was tested (s_n)*/
    long long pairs_unskipped;  /* tested blocks that could not be skipped   (s_u)    */
    long long refreshes;        /* snapshot refreshes                        (s_r)    */
    long long tiles_total;      /* (group, 32-target) tiles covered                   */
    long long tiles_computed;   /* tiles actually streamed through the gradient kernel*/
} ot_gs_stats;

/* ------------------------------------------------------------ handle life */

/* Builds the device layout of `count` instances: groups of rows by label (a
 * stable counting sort), target columns clustered by nearest source class,
 * the cost in that layout (or the features for COST_ONTHEFLY), marginals.
 * Synchronises `stream` before returning.  Errors: OT_GS_EINVAL for
 * n_src/n_tgt < 1, n_groups < 1 or > 16384, gamma <= 0, mu < 0, a label
 * outside [0, n_groups), missing cost or features for the chosen mode, a
 * negative marginal entry, or marginals whose masses differ by more than
 * 1e-6 max(1, sum a, sum b) (no plan with those row and column sums
 * exists; uniform marginals have mass 1); OT_GS_ENUMERIC if the cost, the
 * scale or a marginal is not finite or max C is 0 with cost_scale == 0;
 * OT_GS_ENOMEM, OT_GS_EDEVICE. */
int ot_gs_create(const ot_gs_problem *probs /* host [count] */, int count,
                 ot_gs_handle **out /* host */, void *stream);

void ot_gs_destroy(ot_gs_handle *h);

/* A handle that keeps all its device memory in a caller-owned workspace:
 * ot_gs_workspace_size gives the bytes (it builds the handle once to count
 * them, allocating and freeing device memory, and synchronises `stream`);
 * ot_gs_create_ws builds the same handle in `workspace` (device,
 * caller-owned, kept alive until ot_gs_destroy; any alignment) and reserves
 * everything later calls need: the solver's vectors for histories up to
 * max_hist (1..32), the buffers of checked evaluations, the re-centring copy
 * of a materialised cost and the scratch of ot_gs_plan_csr.  Afterwards
 * ot_gs_dual_grad, ot_gs_solve (hist <= max_hist), ot_gs_plan, ot_gs_plan_csr,
 * ot_gs_transport and ot_gs_screen_state allocate no device memory (the
 * warm-start entry points still do).  Same results, bit for bit, as a handle
 * from ot_gs_create.  Errors: as ot_gs_create; OT_GS_ENOMEM when the
 * workspace is smaller than ot_gs_workspace_size's answer. */
int ot_gs_workspace_size(const ot_gs_problem *probs /* host [count] */, int count, int max_hist,
                         size_t *bytes /* host */, void *stream);
int ot_gs_create_ws(const ot_gs_problem *probs /* host [count] */, int count, int max_hist, void *workspace,
                    size_t ws_bytes, ot_gs_handle **out /* host */, void *stream);

/* ------------------------------------------------------------ hot path */

/* One evaluation of the dual objective (Eq. 4) and its gradient (the ascent
 * direction): grad_alpha = a - T 1, grad_beta = b - T^T 1 with
 * T = [grad psi(alpha + beta_j 1 - c_j)]_j (Eq. 5), for every instance.
 * alpha [sum n_src], beta [sum n_tgt] in; grad_alpha, grad_beta out (same
 * shapes, may be NULL); obj out [count] float64 (device, may be NULL).
 * mode: OT_GS_DENSE, OT_GS_SCREENED or OT_GS_SNAPSHOT, optionally OR-ed with
 * OT_GS_CHECK or OT_GS_VERIFY.  SCREENED results are bit-identical to DENSE
 * at the same point (Theorem 2); SCREENED before any SNAPSHOT uses the zero
 * snapshot (valid for alpha~ = beta~ = 0 since C >= 0).  Without flags the
 * call is asynchronous; a NaN or Inf in alpha or beta then raises a sticky
 * flag that ot_gs_check reports.  With a flag the call synchronises the
 * stream and reports for its own inputs.  Errors: OT_GS_EINVAL (NULL
 * alpha/beta, bad mode or flag), OT_GS_ENUMERIC, OT_GS_EVERIFY (flags
 * only), OT_GS_ENOMEM (the first flagged call allocates two sets of
 * outputs on the handle), OT_GS_EDEVICE. */
int ot_gs_dual_grad(ot_gs_handle *h, const float *alpha, const float *beta,
                    float *grad_alpha, float *grad_beta, double *obj, int mode,
                    void *stream);

/* Solver options (host struct). */
typedef struct {
    int max_iter;         /* accepted L-BFGS iterations (default 200)                */
    int hist;             /* L-BFGS history, 1..32 (default 10)                      */
    int refresh;          /* r of Algorithm 1: snapshot / N refresh period (10)      */
    int use_screen;       /* 1: Algorithms 1-2, 0: dense evaluations ("origin")      */
    int use_lower;        /* 1: build N from the lower bound, 0: never (ablation)    */
    int max_ls;           /* evaluations per line search (default 40)                */
    int init_user;        /* 1: start from alpha_io/beta_io, 0: from zero            */
    double c1, c2;        /* strong-Wolfe constants (1e-4, 0.9)                      */
    double gtol;          /* stop when ||grad||_inf <= gtol (default 0: run max_iter)*/
    double *obj_trace;    /* optional DEVICE [count * (max_iter + 1)] float64: D after
                             each accepted iteration (k = 0 is the starting point)    */
    long long *time_trace;/* optional DEVICE [count * (max_iter + 1)]: device clock
                             (wall_clock64, 100 MHz) at each accepted iteration        */
    int use_graph;        /* 1 (default): record the launches of 16 solver steps
                             into a HIP graph once per call and replay it; same
                             results as 0 (direct launches)                          */
    int verify;           /* 1: every screened evaluation of the solve is repeated
                             densely at the same point (static tile lists, no
                             screen) and the two must agree bit for bit (Lemma 2:
                             skipped blocks are zero); the solve then returns
                             OT_GS_EVERIFY if any evaluation differed.  Direct
                             launches, about twice the evaluation cost; the
                             trajectory is the unverified one.  Default 0.      */
    int recenter;         /* 1 (default; materialised costs only): when a line search
                             finds no step because the float32 iterate cannot move
                             finely enough, the instance is re-centred there: the
                             evaluations go on with the point split as a float64
                             reference plus a small float32 part, on the reduced
                             cost fl32(c_ij - ref_i - ref_j) (a working copy of the
                             cost, allocated by the first such solve) and D plus
                             a.ref_alpha + b.ref_beta; at most 8 times per
                             instance, the second and later ones only after a
                             gain of D above recenter_tol |D| since the previous
                             one (below that the solve has reached the float32
                             floor).  0: stop there (status
                             OT_GS_LINESEARCH).  A re-centred solve leaves the
                             handle with the zero snapshot.                      */
    int solver;           /* OT_GS_SOLVER_LBFGS (default) or OT_GS_SOLVER_AGD: the
                             same evaluations (and screening) driven by another
                             method, see below                                   */
    long long *stats_trace; /* optional DEVICE [count * (max_iter + 1) * 8]: the
                             handle's ot_gs_stats counters (in that struct's order)
                             as instance k's control step saw them at each accepted
                             iteration, including the evaluation that was accepted;
                             differences between iterations give the evaluations,
                             the Theorem 1 counters (s_i, s_n, s_u, s_r) and the
                             skipped tiles of each iteration.  The counters are
                             per handle: exact per instance for a one-instance
                             handle, the whole batch's otherwise                */
    double *gnorm_trace;  /* optional DEVICE [count * (max_iter + 1)]: ||grad D||_inf
                             at each accepted iteration                          */
    int resume;           /* 1: go on from the L-BFGS state on the handle (the last
                             L-BFGS solve on it, or ot_gs_solver_load) instead of
                             starting afresh: instances that stopped at the
                             iteration limit continue up to this call's max_iter
                             (counted from the original start; traces are indexed
                             the same way), with the same iterates, bit for bit,
                             as one uninterrupted solve with the same options.
                             alpha_io / beta_io receive the result; init_user is
                             ignored; hist must equal the state's; a state with a
                             re-centred instance needs recenter = 1.  The first
                             evaluation is a snapshot (dense).  L-BFGS only.     */
    double recenter_tol;  /* relative gain of D since the last re-centring that
                             allows another one (default 1e-9)                 */
} ot_gs_options;

/* Solvers.  The screening changes how an evaluation is computed, never its
 * result (Lemma 2), so any solver built on D and its gradient can use it
 * (Theorem 1 and the remark after it, Sec. 3.4).
 *   OT_GS_SOLVER_LBFGS: the paper's solver (Sec. 2.3), the options above.
 *   OT_GS_SOLVER_AGD:   accelerated gradient ascent (Nesterov momentum in the
 *     FISTA form, backtracking on the step, function-value restart) in the
 *     marginal-scaled variables; max_iter counts accepted steps, max_ls is
 *     the number of step halvings per trial before the solve stops with
 *     OT_GS_LINESEARCH, refresh / use_screen / use_lower / gtol / traces /
 *     use_graph / init_user as for L-BFGS; hist, c1, c2 and recenter are not
 *     used and verify must be 0.  Accepted objectives never decrease. */
#define OT_GS_SOLVER_LBFGS 0
#define OT_GS_SOLVER_AGD   1

/* Solver checkpoint.  The L-BFGS state a solve leaves on the handle - per
 * instance the iterate, gradient, direction, the (s, y) history and its Gram
 * matrices, the line-search state, the iteration count, the re-centring
 * reference and the pending trial point - as one host byte string, and back
 * into a handle built from the same problems (ot_gs_solve with resume then
 * continues it).  The screening snapshot is not part of it: a resumed solve
 * takes a fresh one (Lemma 2: the snapshot changes which blocks are skipped,
 * never the values).
 *   ot_gs_solver_state_size: bytes of the state (host out); OT_GS_EINVAL if
 *     the handle holds no L-BFGS state (no finished L-BFGS solve).
 *   ot_gs_solver_save: writes the state into the caller's HOST buffer of
 *     `bytes` bytes (at least the size above); synchronises `stream`.
 *   ot_gs_solver_load: reads a saved state into a handle with the same
 *     instance shapes (n_src, n_tgt, groups, gamma, mu of every instance;
 *     checked, OT_GS_EINVAL on any mismatch or a truncated buffer); allocates
 *     the solver buffers if the handle has none yet; synchronises `stream`. */
int ot_gs_solver_state_size(ot_gs_handle *h, size_t *bytes);
int ot_gs_solver_save(ot_gs_handle *h, void *host_buf, size_t bytes, void *stream);
int ot_gs_solver_load(ot_gs_handle *h, const void *host_buf, size_t bytes, void *stream);

/* Fills `o` with the defaults listed above. */
void ot_gs_default_options(ot_gs_options *o);

/* Per-instance result (host struct). */
typedef struct {
    int iters, evals, status;   /* status: OT_GS_OK converged, NOT_CONVERGED, LINESEARCH */
    double obj;                 /* final D                                               */
    double gnorm_inf;           /* final ||grad D||_inf                                  */
} ot_gs_info;

/* Maximises D by L-BFGS with every evaluation on the device (Algorithm 1
 * when use_screen = 1).  alpha_io [sum n_src], beta_io [sum n_tgt]: start
 * point if init_user, final point on return.  info: host [count] or NULL.
 * Synchronises the stream before returning.  Returns OT_GS_OK or the worst
 * per-instance status (OT_GS_NOT_CONVERGED, OT_GS_LINESEARCH), or an error:
 * OT_GS_ENUMERIC when the start point holds a NaN or Inf or an instance's
 * objective is not finite there, OT_GS_EVERIFY (opts.verify) when a screened
 * evaluation differed from the dense one. */
int ot_gs_solve(ot_gs_handle *h, const ot_gs_options *opts, float *alpha_io,
                float *beta_io, ot_gs_info *info, void *stream);

/* Plan recovery t_j = grad psi(alpha + beta_j 1 - c_j) (Sec. 2.3) into a
 * dense row-major T, instance k at offset sum_{k'<k} n_src n_tgt, caller
 * order.  Errors as ot_gs_dual_grad. */
int ot_gs_plan(ot_gs_handle *h, const float *alpha, const float *beta, float *T,
               void *stream);

/* The same plan in compressed sparse row form (its entries are exact zeros
 * outside the active (group, target) blocks and where alpha_i + beta_j <
 * c_ij), in two calls at the same (alpha, beta).  Rows are the caller's
 * source rows stacked over the instances (sum n_src); column indices are the
 * caller's target index within the instance.
 * Count (col_idx NULL): row_ptr [sum n_src + 1] (device, int64,
 * caller-allocated) receives the exclusive prefix of the rows' nonzero
 * counts and *nnz (host) their total.  Fill (col_idx, val non-NULL):
 * col_idx [nnz] (device int32) and val [nnz] (device float32,
 * caller-allocated) receive row i's entries at row_ptr[i] .. row_ptr[i+1] - 1,
 * in the library's internal column order (targets grouped by nearest source
 * class; deterministic, not sorted by index); values bit-identical to
 * ot_gs_plan's.  Allocates temporary device memory (4-12 bytes per row and
 * 32-target column block) and synchronises the stream.
 * Errors: as ot_gs_dual_grad; OT_GS_EINVAL for a missing nnz (count) or
 * val (fill); OT_GS_ENOMEM. */
int ot_gs_plan_csr(ot_gs_handle *h, const float *alpha, const float *beta, long long *row_ptr,
                   int *col_idx, float *val, long long *nnz, void *stream);

/* ot_gs_plan_csr for callers that cannot allocate device memory (code
 * that must not call hipMalloc, tight serving loops): the same two calls,
 * arguments, results (bit for bit) and errors, with the call's scratch
 * (segment counts and offsets, 12 bytes per row and 32-target column block
 * for a fill call, 4 per block plus 8 per row for a count) taken from one
 * fixed device array of OT_GS_STATIC_SCRATCH_BYTES that each GPU holds from
 * the first call until the process ends; no device memory is allocated or
 * freed.  Calls on one GPU share that array, so calls that overlap in time
 * on one GPU (other streams, other host threads) race and must not be
 * issued; each call rewrites everything of it that it reads.  Sizes beyond
 * the array are refused with OT_GS_EINVAL before any work is enqueued.
 * Synchronises the stream. */
#define OT_GS_STATIC_SCRATCH_BYTES (64u << 20)
int ot_gs_plan_csr_static(ot_gs_handle *h, const float *alpha, const float *beta, long long *row_ptr,
                          int *col_idx, float *val, long long *nnz, void *stream);

/* Barycentric mapping of the source samples onto the targets with the plan
 * at (alpha, beta) (Sec. 2.1, where the source matrix is transported as
 * n T^T X_S): y_j = (1 / b_j) sum_i T_ij x_i, i.e. n_tgt T^T X_S for uniform
 * b (at a solution every y_j is then a convex combination of source
 * samples).  x_src: device [sum n_src x dim] row-major, caller order (the
 * instances' source rows stacked); y_out: device [sum n_tgt x dim].
 * 1 <= dim <= 256.  Deterministic (fixed summation order).  Materialised or
 * given costs only.  Errors: OT_GS_EINVAL (NULL, dim, on-the-fly handle),
 * OT_GS_EDEVICE. */
int ot_gs_transport(ot_gs_handle *h, const float *alpha, const float *beta, const float *x_src, int dim,
                    float *y_out, void *stream);

/* The scaled cost the evaluations use (Sec. 2.1; for COST_ONTHEFLY the
 * values its matrix-core tiles produce, bit for bit), written to C_out in
 * the layout of ot_gs_plan: instance k at offset sum_{k'<k} n_src n_tgt,
 * row-major, caller order.  C_out: device, caller-owned.  For tests and
 * inspection; the hot path never writes the cost.  Errors: OT_GS_EINVAL
 * (NULL), OT_GS_EDEVICE. */
int ot_gs_cost(ot_gs_handle *h, float *C_out, void *stream);

/* ------------------------------------------------------------ utilities */

/* Synchronises `stream` and reports (OT_GS_ENUMERIC) whether a NaN or Inf
 * dual value reached an evaluation since the last check; clears the flag. */
int ot_gs_check(ot_gs_handle *h, void *stream);

/* The screening state of Algorithm 1 as the last evaluation left it, in the
 * caller's layout: alpha_s [sum n_src], beta_s [sum n_tgt] the snapshot
 * point (caller order); z_snap, o_snap (float32) and in_N (uint8, 1 = in
 * the set N of Eq. 8) per (label, target) pair, instance k as a row-major
 * [n_groups x n_tgt] block (row = label, column = caller's target index)
 * at offset sum_{k'<k} n_groups n_tgt.  z_snap and o_snap are ||[f]_+|| and
 * ||[f]_-|| of Defs. 1-2 at the snapshot point as the gradient kernel
 * computed them; N is the set built at the last SNAPSHOT evaluation (or
 * refresh of a solve) from Eq. 7 against the snapshot before it.  Pairs of
 * empty labels read 0.  Any output may be NULL; all are device arrays owned
 * by the caller.  For tests and inspection.  Errors: OT_GS_EINVAL,
 * OT_GS_EDEVICE. */
int ot_gs_screen_state(ot_gs_handle *h, float *alpha_s, float *beta_s, float *z_snap,
                       float *o_snap, uint8_t *in_N, void *stream);

/* rho parameterisation of the experiments (Sec. 5.2):
 * gamma (1-rho)/2 ||t||^2 + gamma rho sum ||t_[l]||  ==  Eq. 3 with
 * gamma' = gamma (1 - rho), mu' = rho / (1 - rho).  OT_GS_EINVAL unless
 * 0 <= rho < 1 and gamma > 0. */
int ot_gs_rho_to_mu(double gamma, double rho, double *gamma_out, double *mu_out);

/* Copies the cumulative counters (host out) after synchronising `stream`;
 * reset != 0 zeroes them afterwards. */
int ot_gs_get_stats(ot_gs_handle *h, ot_gs_stats *out, int reset, void *stream);

/* Kernel timing with HIP events recorded on the launch stream around every
 * launch of kernel `which` (0: gradient tiles, 1: screen, 2: reduce,
 * 3: L-BFGS); enable != 0 turns it on.  ot_gs_kernel_time synchronises and
 * returns the summed milliseconds and launch count since enabling. */
int ot_gs_kernel_timing(ot_gs_handle *h, int enable);
int ot_gs_kernel_time(ot_gs_handle *h, int which, double *ms, long long *launches);

/* Launch-by-launch cost of the dense gradient tiles (Eq. 5 per (group, 32
 * target) tile): `repeats` back-to-back launches of the tile kernels between
 * two HIP events on `stream`; writes the mean microseconds per launch (host
 * out).  With `alpha` and `beta` (device, caller order, as for
 * ot_gs_dual_grad) the tiles read them as a dense ot_gs_dual_grad call does;
 * with NULL they read the handle's current evaluation point.  Leaves the row
 * and column partials of a dense evaluation; synchronises `stream`. */
int ot_gs_profile_tiles(ot_gs_handle *h, const float *alpha, const float *beta, int repeats,
                        double *us_per_launch, void *stream);

/* Tile configuration.  The gradient tiles are launched per bucket of the
 * work lists (groups of similar size; buckets 0..12, bucket 13 holds the
 * chunks of split groups: over 2048 rows with the materialized cost, over
 * 1024 on the fly).  A bucket has a variant and a grid multiplier
 * (workgroups launched per resident workgroup slot, 1-16, default 2).
 * Materialized cost, bucket b of groups up to 64 (b = 0), 128 b rows
 * (b = 1..8) or 1024 + 256 (b - 8) rows (b = 9..12): variant 0 = teams (8,
 * 4, 2 tiles per workgroup for groups up to 64, 128, 256 rows, else one),
 * 1 = the next tile's loads in flight during the current tile (b <= 8),
 * 2 = the next tile copied into LDS meanwhile (groups up to 512 rows);
 * buckets 0 and 9..12 have variant 0 only.  On-the-fly cost,
 * buckets 1-4: 0 = one 32-row block per wavefront, 1 = two blocks per
 * wavefront and half the wavefronts; other buckets variant 0 only.  Every
 * configuration gives bit-identical results.
 *
 * ot_gs_autotune times every variant with multipliers 1, 2 and 4 on the
 * handle's buckets (`repeats` dense launches each, at the handle's current
 * point), keeps the fastest, and, when the environment variable
 * OTGS_AUTOTUNE_CACHE names a file, records them there ("key variant
 * multiplier" lines; the key names the device, the cost path, the bucket,
 * the feature padding and the tile count's power of two).  ot_gs_create
 * applies matching entries of that file.  Synchronises `stream`. */
int ot_gs_autotune(ot_gs_handle *h, int repeats, void *stream);
int ot_gs_tile_config(ot_gs_handle *h, int bucket, int variant, int grid_mult);
int ot_gs_get_tile_config(ot_gs_handle *h, int bucket, int *variant, int *grid_mult, int *n_tiles);

/* Size facts of instance k (host out, any may be NULL): groups that are
 * nonempty, padded target count of the internal layout, tiles. */
int ot_gs_layout_info(ot_gs_handle *h, int k, int *n_groups_nonempty,
                      int *n_tgt_padded, int *n_tiles);

/* ------------------------------------------------------------ warm start
 *
 * Not part of the paper's method (Algorithm 1 starts from zero duals): a
 * network that predicts a starting point (alpha, beta) from per-sample
 * features, trained on converged duals of the plain solver.  Any starting
 * point leads the solver to the same optimum (Eq. 4 is concave); a good one
 * saves iterations.  ot_gs_solve with init_user = 1 takes the prediction and
 * makes its first evaluation a snapshot (Algorithm 1's snapshot must be
 * exact at the start).
 *
 * Features (dim + 8 per sample, float32): the feature vector times
 * sqrt(cost_scale); the squared distance (times cost_scale) to the sample's
 * own centroid (a source's class centroid; a target's pseudo-class centroid,
 * the pseudo-class being the class of its nearest source centroid); the
 * least squared distance (times cost_scale) to the other side's centroids;
 * the fraction of its side in its (pseudo-)class; side (0 source, 1
 * target); log gamma; log max(mu, 1e-8); log n_src; log n_tgt.
 *
 * Network: Linear(d_in, w) - GELU - Linear(w, w) - GELU - Linear(w, 1),
 * GELU(z) = z Phi(z) (exact normal CDF).  The three products run on bf16
 * matrix cores: their operands are rounded to bfloat16 (nearest even),
 * accumulation and all other arithmetic is float32.  Parameters form one
 * float32 vector: W1 [d_in x w] row-major (row = input), b1 [w],
 * W2 [w x w], b2 [w], w3 [w], b3 [1].  Training minimises the mean squared
 * error with Adam (beta1 0.9, beta2 0.999, eps 1e-8). */
typedef struct ot_gs_mlp ot_gs_mlp;

/* Network for d_in inputs and width w; buffers for up to max_rows rows per
 * product (inference and training batches).  Parameters start at zero; set
 * them with ot_gs_mlp_set_params.  Errors: OT_GS_EINVAL, OT_GS_ENOMEM. */
int ot_gs_mlp_create(int d_in, int width, int max_rows, ot_gs_mlp **out /* host */);
void ot_gs_mlp_destroy(ot_gs_mlp *m);
int ot_gs_mlp_n_params(const ot_gs_mlp *m);

/* Copies the parameter vector in (and resets the Adam moments) or out;
 * params: device [n_params]. */
int ot_gs_mlp_set_params(ot_gs_mlp *m, const float *params, void *stream);
int ot_gs_mlp_get_params(ot_gs_mlp *m, float *params, void *stream);

/* out[i] = network(F[i, :]) for n_rows rows of F (device, row-major
 * [n_rows x d_in]); out: device [n_rows]. */
int ot_gs_mlp_forward(ot_gs_mlp *m, const float *F, long long n_rows, float *out, void *stream);

/* Mean squared error of the network on rows F, targets y (device
 * [n_rows], 1 <= n_rows <= max_rows): loss (device float64, may be NULL)
 * and its gradient (device [n_params], same layout as the parameters, may
 * be NULL). */
int ot_gs_mlp_loss_grad(ot_gs_mlp *m, const float *F, const float *y, int n_rows, double *loss,
                        float *grad, void *stream);

/* `epochs` passes over consecutive batches of `batch` rows of (F, y), one
 * Adam step (learning rate lr) per batch; the caller shuffles the rows.
 * loss_trace: optional device float64 [epochs * ceil(n_rows / batch)], the
 * loss of every batch before its step. */
int ot_gs_mlp_train(ot_gs_mlp *m, const float *F, const float *y, long long n_rows, int batch,
                    int epochs, float lr, double *loss_trace, void *stream);

/* Features of `count` instances (probs as for ot_gs_create, with x_src,
 * x_tgt and one common dim) into F (device, [sum n_src + sum n_tgt] x
 * (dim + 8)): the sources of every instance in order, then the targets.
 * scales: host [count], the cost scale of each instance (see
 * ot_gs_cost_scale).  Synchronises `stream`. */
int ot_gs_features(const ot_gs_problem *probs, int count, const float *scales, float *F, void *stream);

/* The cost scale each instance of a handle uses (host out [count]). */
int ot_gs_cost_scale(ot_gs_handle *h, float *scales);

/* Predicted starting point of every instance of h: features of probs (the
 * problems h was created from; they need x_src and x_tgt) through the
 * network; alpha_out [sum n_src], beta_out [sum n_tgt] (device).  Errors:
 * OT_GS_EINVAL (NULL, network input size), OT_GS_ESHAPE (probs do not match
 * h), OT_GS_ENOMEM, OT_GS_EDEVICE.  Synchronises `stream`. */
int ot_gs_warm_start(ot_gs_handle *h, ot_gs_mlp *m, const ot_gs_problem *probs, float *alpha_out,
                     float *beta_out, void *stream);

const char *ot_gs_last_error(void);
const char *ot_gs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OTGS_H */
