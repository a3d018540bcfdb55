// Device L-BFGS for the smooth relaxed dual (it minimises F = -D), one state
// machine per instance, no host round trip per iteration.
//
// The two-loop recursion of Liu and Nocedal is run on coefficients: with the
// history pairs (s_i, y_i) and the current gradient G, every vector the
// recursion forms is G scaled plus a combination of the s_i and y_i, so the
// recursion needs only the float64 dot products s_i.G, y_i.G, s_i.y_j, y_i.y_j
// (kept as Gram matrices and updated from the dots of each new gradient) and
// yields coefficients (cg, cs_i, cy_i) of the direction d = cg G + sum cs_i
// s_i + cy_i y_i.  Per function evaluation the solver runs three kernels:
//   dots   - every dot product it needs, in float64, fixed-order partials;
//   ctrl   - one wavefront per instance: strong-Wolfe line search (bracketing
//            then cubic zoom, Nocedal and Wright Algs. 3.5-3.6), history and
//            Gram update on acceptance, the coefficient recursion, the
//            convergence test and the mode of the next evaluation (screened,
//            or dense with a snapshot refresh every r accepted iterations as
//            in Algorithm 1);
//   update - the vector work: accept the trial point, push (s, y), form the
//            new direction and the next trial point.
// The iteration runs on scaled variables x = (alpha_i / w_i, beta_j / w_j)
// with w_i = 1 / sqrt(M a_i), w_j = 1 / sqrt(M b_j), M = (n_src + n_tgt) / 2
// (a diagonal preconditioner: the dual's curvature along alpha_i and beta_j
// scales with the marginals a_i and b_j, so with n_src != n_tgt the two
// blocks differ by the size ratio; for n_src = n_tgt and uniform marginals
// every w is 1).  Evaluations see the actual point w x; the gradient with
// respect to x is w times the gradient of D.
#include "otgs_internal.h"

namespace otgs {

constexpr int HMAX = 32;
constexpr int LB_BLOCK = 64;
constexpr int LB_PER_THREAD = 8;
constexpr int LB_VB = LB_BLOCK * LB_PER_THREAD;   // vector elements per dots block
// batched handles with at least this many vector elements in all form their
// dots with k_lbfgs_dots_seq
constexpr long long LB_SEQ_MIN_VTOT = 32768;
constexpr int LB_SEQ_SPLIT = 2;   // wavefronts sharing the history slots of a vector block

enum LbStatus { LB_RUNNING = 0, LB_CONVERGED = 1, LB_LSFAIL = 2, LB_MAXITER = 3, LB_RECENTER = 4 };
constexpr int RECENTER_MAX = 8;   // re-centrings per instance and solve

struct LbParams {
  int hist, max_iter, max_ls, refresh, use_screen, use_lower;
  int recenter;           // re-centre instead of stopping on a failed search
  double c1, c2, gtol;
  double recenter_tol;    // gain of D (relative) since the last re-centring that allows another
  double* obj_trace;      // [count * (max_iter + 1)] or NULL
  long long* time_trace;  // [count * (max_iter + 1)] or NULL
  long long* stats_trace; // [count * (max_iter + 1)][CNT_NUM] or NULL
  double* gnorm_trace;    // [count * (max_iter + 1)] or NULL
};


struct LbState {
  int status, phase, iter, evals, nls, zoom;
  int count, head;            // history ring
  int accept, push, slot, newdir;
  int since_refresh, mode_eval;   // mode_eval: mode of the evaluation just done
  int force, n_rec;               // force: accept the next evaluation (best step of a failed search);
                                  // n_rec: re-centrings so far
  double f, gtd0, gmax;
  double t, t_prev, f_prev, dp_prev;
  double t_lo, f_lo, dp_lo, t_hi, f_hi, dp_hi;
  double t_acc, t_next;
  double GG, cg;
  double SG[HMAX], YG[HMAX], rho[HMAX];
  double cs[HMAX], cy[HMAX];
  double f_restart;   // objective when the memory was last dropped after a failed search
  double f_rec;       // objective at the last re-centring
  double h0;          // s.y / y.y of the newest pair accepted into the memory (0: none yet)
};
// The Gram matrices s_i.y_j and y_i.y_j of an instance live next to the state
// as [2][hist][hist] float64 (row-major, stride hist); the control kernel
// keeps them in LDS during a step.
struct LbGram {
  double* SY;   // SY[i * hist + j] = s_i . y_j
  double* YY;   // YY[i * hist + j] = y_i . y_j
  int h;
  __device__ __forceinline__ double& sy(int i, int j) { return SY[i * h + j]; }
  __device__ __forceinline__ double& yy(int i, int j) { return YY[i * h + j]; }
};
static_assert(sizeof(LbState) % 16 == 0, "LbState is copied as int4");

struct LbArgs {
  const InstDev* inst;
  LbParams P;
  LbState* st;
  int* inst_mode;
  int* n_active;
  // vectors, instance k at voff[k], length ns + nt_pad (alpha rows, then beta columns)
  const long long* voff;
  float* X;
  float* G;
  float* Dv;
  float* S;      // [hist][total]
  float* Y;
  long long vtot;
  float* alpha;  // trial point (internal order), read by the evaluation
  float* beta;
  const float* ga;  // gradient of D at the trial point
  const float* gb;
  const double* obj;
  double* part;  // [count][ndot][maxb] dot partials per vector block
  int maxb;
  int ndot;
  const double* obj_part;   // assembly partials of D, [count][obj_stride]
  long long obj_stride;
  double* obj_out;          // D of every instance (also written by ctrl)
  double* gram;             // [count][2][hist][hist]
  float* alpha_s;           // snapshot point, written at snapshot evaluations
  float* beta_s;
  long long* counters;      // unscreened solves: evaluation counters, advanced here
  // group statistics formed by the update (k_lbfgs_update_gs)
  GroupStats* gstats;
  const int* g_start;
  const int* g_size;
  int* counts;              // work-list counts of the next screen pass
  int max_le;               // most groups of an instance
  int batched;              // more than one instance: finished ones skip their update
  const float* W;           // [vtot] variable scales w (actual = w * scaled)
  const int* w_unit;        // [count] 1: every scale of the instance is 1 (W is not read)
  // re-centred solves (see k_recenter_vec): the evaluations see the point
  // relative to a reference xref (actual variables, float64) through the
  // reduced cost c_ij - xref_i - xref_j; D adds obj_const = a.xref_a + b.xref_b
  double* xref;             // [vtot] or NULL
  double* obj_const;        // [count]
  int* n_recenter;          // instances waiting for a re-centring
  // the screen pass's per-workgroup counters (added to `counters` by
  // ot_gs_get_stats; the statistics trace adds them the same way)
  const long long* block_counters;
  int n_screen_blocks;
};

// Per-iteration traces besides D and the clock.  The handle's counters as
// ot_gs_get_stats forms them (the global array plus the screen pass's
// per-workgroup counters), summed by the 64 lanes and read before this
// control step adds anything; in unscreened solves its own additions for
// the evaluation just done are added here.  Every lane gets the sums.
__device__ __forceinline__ void lb_counter_sums(const LbArgs& A, const InstDev& I, long long (&cs)[CNT_NUM]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < CNT_NUM; ++c) cs[c] = lane == 0 ? A.counters[c] : 0;
  for (int b = lane; b < A.n_screen_blocks; b += 64)
#pragma unroll
    for (int c = 0; c < CNT_NUM; ++c) cs[c] += A.block_counters[(size_t)b * CNT_NUM + c];
#pragma unroll
  for (int c = 0; c < CNT_NUM; ++c)
    for (int o = 32; o > 0; o >>= 1) cs[c] += __shfl_xor(cs[c], o);
  if (!A.P.use_screen) {
    const long long tiles = (long long)I.Le * I.njb;
    cs[CNT_EVALS] += 1;
    cs[CNT_PAIRS_TOTAL] += (long long)I.Le * I.nt;
    cs[CNT_TILES_TOTAL] += tiles;
    cs[CNT_TILES_COMPUTED] += tiles;
  }
}

// the statistics and gradient-norm traces at entry idx (one lane writes)
__device__ __forceinline__ void lb_write_traces(const LbParams& P, const long long (&cs)[CNT_NUM], size_t idx,
                                                double gmax) {
  if (P.stats_trace)
    for (int c = 0; c < CNT_NUM; ++c) P.stats_trace[idx * CNT_NUM + c] = cs[c];
  if (P.gnorm_trace) P.gnorm_trace[idx] = gmax;
}

// An instance whose solve has ended and whose last control step accepted no
// point has a zero step and no new direction: its update would rewrite the
// same values (and form group statistics no screen reads).  Batches skip it,
// unless the evaluation just done was a snapshot: its z~ and o~ were written
// at the trial point, so that point must still become alpha~, beta~ (a later
// screened evaluation on the handle pairs them).  A single instance does not
// wait for its state before its first loads.
__device__ __forceinline__ bool lb_update_idle(const LbArgs& A, const LbState& S) {
  return A.batched && S.status != LB_RUNNING && !S.accept && S.mode_eval != EM_SNAPSHOT;
}

__device__ __forceinline__ int lb_ndot(int hist) { return 5 + 3 * hist; }

// dot slots: 0 Gt.d, 1 Gt.Gt, 2 Gt.G, 3 d.d, 4 max|Gt| (as a double),
// 5 + 3i: Gt.s_i, 6 + 3i: Gt.y_i, 7 + 3i: d.y_i

// element e of instance k: trial gradient of F (= -grad D) in the actual
// variables (lb_gt) and in the scaled ones (times w)
__device__ __forceinline__ float lb_gt(const LbArgs& A, const InstDev& I, int e) {
  return e < I.ns ? -A.ga[I.row_off + e] : -A.gb[I.col_off + (e - I.ns)];
}

// Per-lane partials, then fixed-order wavefront reductions (the totals in
// every lane).  Base dots of a vector block: g~.d, g~.g~, g~.G, d.d (scaled
// variables) and the lane's max |grad D| gm in the actual ones (lane j
// holds dot j, lanes >= 4 the maximum).
__device__ __forceinline__ double lb_base_dots(const float* gt, const float* G, const float* d, int lane, float gm) {
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
  for (int q = 0; q < LB_PER_THREAD; ++q) {
    a0 += (double)gt[q] * d[q];
    a1 += (double)gt[q] * gt[q];
    a2 += (double)gt[q] * G[q];
    a3 += (double)d[q] * d[q];
  }
  a0 = wave_sum_dd(a0);
  a1 = wave_sum_dd(a1);
  a2 = wave_sum_dd(a2);
  a3 = wave_sum_dd(a3);
  const double g4 = wave_max_d((double)gm);
  return lane == 0 ? a0 : lane == 1 ? a1 : lane == 2 ? a2 : lane == 3 ? a3 : g4;
}

// Dots of history slot i over a vector block: g~.s_i, g~.y_i, d.y_i (lane j
// holds dot j, lanes >= 2 the last).
__device__ __forceinline__ double lb_slot_dots(const float* gt, const float* s_, const float* y_,
                                               const float* d, int lane) {
  double s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
  for (int q = 0; q < LB_PER_THREAD; ++q) {
    s0 += (double)gt[q] * s_[q];
    s1 += (double)gt[q] * y_[q];
    s2 += (double)d[q] * y_[q];
  }
  s0 = wave_sum_dd(s0);
  s1 = wave_sum_dd(s1);
  s2 = wave_sum_dd(s2);
  return lane == 0 ? s0 : lane == 1 ? s1 : s2;
}

// One wavefront per (vector block b, slot z) of instance k, LB_PER_THREAD
// elements per lane: z = 0 forms the five base dots, z = 1 + i the three
// dots of history slot i, so every wavefront issues all its loads at once.
// Each lane adds its elements' products, fixed-order wavefront reductions
// (maximum for dot 4) give one float64 partial per block and dot.  Run by
// k_lbfgs_dots (grid (maxb, count, 1 + hist)).
__device__ __forceinline__ void lb_dots_wave(const LbArgs& A, const InstDev& I, int k, int b, int z, int lane) {
  const long long v0 = A.voff[k];
  const LbState& S = A.st[k];
  const int st_status = S.status, st_phase = S.phase, st_count = S.count;
  const int n = I.ns + I.nt_pad;
  if (b * LB_VB >= n) return;           // beyond this instance: ctrl reads no such partial
  const bool wu = A.w_unit[k] != 0;
  const bool run = st_status == LB_RUNNING;
  const int cnt = (run && st_phase != 0) ? st_count : 0;
  const int slot = z - 1;
  // partial table [count][ndot][maxb]: dot d of block b at out[d * maxb]
  double* out = A.part + (size_t)k * A.ndot * A.maxb + b;
  if (z > 0 && slot >= cnt) {
    if (slot < A.P.hist && lane < 3) out[(size_t)(5 + 3 * slot + lane) * A.maxb] = 0.0;
    return;
  }
  // an instance whose solve has ended loads nothing (its dots are zeros)
  float gt[LB_PER_THREAD], v1[LB_PER_THREAD], v2[LB_PER_THREAD], dv[LB_PER_THREAD];
  float gm = 0.f;
#pragma unroll
  for (int q = 0; q < LB_PER_THREAD; ++q) {
    const int e = b * LB_VB + q * LB_BLOCK + lane;
    const bool ok = e < n && run;
    const float g0 = ok ? lb_gt(A, I, e) : 0.f;
    gm = fmaxf(gm, fabsf(g0));
    gt[q] = ok ? (wu ? g0 : g0 * A.W[v0 + e]) : 0.f;
    if (z == 0) {
      v1[q] = ok ? A.G[v0 + e] : 0.f;    // G
      v2[q] = ok ? A.Dv[v0 + e] : 0.f;   // d
      dv[q] = 0.f;
    } else {
      v1[q] = ok ? A.S[(size_t)slot * A.vtot + v0 + e] : 0.f;
      v2[q] = ok ? A.Y[(size_t)slot * A.vtot + v0 + e] : 0.f;
      dv[q] = ok ? A.Dv[v0 + e] : 0.f;   // d (for d.y_i)
    }
  }
  // lane j < nd writes dot j's partial of this block
  const double t = z == 0 ? lb_base_dots(gt, v1, v2, lane, gm) : lb_slot_dots(gt, v1, v2, dv, lane);
  const int nd = z == 0 ? 5 : 3;
  if (lane < nd) out[(size_t)((z == 0 ? 0 : 5 + 3 * slot) + lane) * A.maxb] = t;
}

__global__ void __launch_bounds__(LB_BLOCK) k_lbfgs_dots(LbArgs A) {
  // the instance, its vector offset and its state are read together
  const int k = blockIdx.y;
  const InstDev I = A.inst[k];
  lb_dots_wave(A, I, k, blockIdx.x, blockIdx.z, threadIdx.x);
}

// Batches of many instances: grid (maxb, count, LB_SEQ_SPLIT), wavefront z
// of an (instance, vector block) forms the three dots of each history slot
// of its share in turn (the next slot's s, y loads in flight while the
// current slot's dots are formed), wavefront 0 also the five base dots.  The
// per-slot grid of k_lbfgs_dots reads g~ and d once per slot; over a batch
// that traffic bounds the pass.  Same per-lane sums and reductions, so the
// same bits.
__global__ void __launch_bounds__(LB_BLOCK) k_lbfgs_dots_seq(LbArgs A) {
  const int k = blockIdx.y, b = blockIdx.x, z = blockIdx.z;
  const int per = (A.P.hist + LB_SEQ_SPLIT - 1) / LB_SEQ_SPLIT;
  const int sl0 = z * per, sl1 = min(A.P.hist, sl0 + per);   // history slots of this wavefront
  const int lane = threadIdx.x;
  const InstDev I = A.inst[k];
  const long long v0 = A.voff[k];
  const LbState& S = A.st[k];
  const int st_status = S.status, st_phase = S.phase, st_count = S.count;
  const int n = I.ns + I.nt_pad;
  if (b * LB_VB >= n) return;
  const bool wu = A.w_unit[k] != 0;
  const bool run = st_status == LB_RUNNING;
  const int cnt = (run && st_phase != 0) ? st_count : 0;
  const int sc1 = min(cnt, sl1);   // slots [sl0, sc1) hold pairs, [max(sl0, cnt), sl1) are zeros
  double* out = A.part + (size_t)k * A.ndot * A.maxb + b;
  float gt[LB_PER_THREAD], g[LB_PER_THREAD], dv[LB_PER_THREAD], sc[LB_PER_THREAD], yc[LB_PER_THREAD];
  auto load_slot = [&](int slot, float* s_, float* y_) {
#pragma unroll
    for (int q = 0; q < LB_PER_THREAD; ++q) {
      const int e = b * LB_VB + q * LB_BLOCK + lane;
      const bool ok = e < n && run;
      s_[q] = ok ? A.S[(size_t)slot * A.vtot + v0 + e] : 0.f;
      y_[q] = ok ? A.Y[(size_t)slot * A.vtot + v0 + e] : 0.f;
    }
  };
  float gm = 0.f;
#pragma unroll
  for (int q = 0; q < LB_PER_THREAD; ++q) {
    const int e = b * LB_VB + q * LB_BLOCK + lane;
    const bool ok = e < n && run;
    const float g0 = ok ? lb_gt(A, I, e) : 0.f;
    gm = fmaxf(gm, fabsf(g0));
    gt[q] = ok ? (wu ? g0 : g0 * A.W[v0 + e]) : 0.f;
    g[q] = (ok && z == 0) ? A.G[v0 + e] : 0.f;
    dv[q] = ok ? A.Dv[v0 + e] : 0.f;
  }
  if (sl0 < sc1) load_slot(sl0, sc, yc);
  if (z == 0) {
    const double t0 = lb_base_dots(gt, g, dv, lane, gm);
    if (lane < 5) out[(size_t)lane * A.maxb] = t0;
  }
  for (int slot = sl0; slot < sc1; ++slot) {
    float sn[LB_PER_THREAD], yn[LB_PER_THREAD];
    if (slot + 1 < sc1) load_slot(slot + 1, sn, yn);
    const double t = lb_slot_dots(gt, sc, yc, dv, lane);
    if (lane < 3) out[(size_t)(5 + 3 * slot + lane) * A.maxb] = t;
    if (slot + 1 < sc1) {
#pragma unroll
      for (int q = 0; q < LB_PER_THREAD; ++q) {
        sc[q] = sn[q];
        yc[q] = yn[q];
      }
    }
  }
  for (int slot = max(sl0, cnt); slot < sl1; ++slot)
    if (lane < 3) out[(size_t)(5 + 3 * slot + lane) * A.maxb] = 0.0;
}

__device__ double lb_cubic(double t0, double f0, double d0, double t1, double f1, double d1) {
  const double lo = fmin(t0, t1), hi = fmax(t0, t1), w = hi - lo;
  const double d1c = d0 + d1 - 3.0 * (f0 - f1) / (t0 - t1);
  const double disc = d1c * d1c - d0 * d1;
  double t = 0.5 * (lo + hi);
  if (disc >= 0.0) {
    const double d2 = copysign(sqrt(disc), t1 - t0);
    const double den = d1 - d0 + 2.0 * d2;
    if (den != 0.0) {
      const double c = t1 - (t1 - t0) * (d1 + d2 - d1c) / den;
      if (isfinite(c)) t = c;
    }
  }
  if (t < lo + 0.1 * w || t > hi - 0.1 * w) t = 0.5 * (lo + hi);
  return t;
}

// ring slot of the j-th oldest pair
__device__ __forceinline__ int lb_slot(const LbState& S, int hist, int j) {
  return (S.head - S.count + j + hist) % hist;
}

// float64 value of lane l (l uniform) in every lane
__device__ __forceinline__ double lane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Two-loop recursion on coefficients; d = -H G.  Returns d.G.  Run by all 64
// lanes of the control wavefront; lane i owns pair slot i: its coefficients
// and a running sum of the Gram terms its own inner product needs.  When a
// step fixes the coefficient of slot p, that value is broadcast (readlane)
// and every lane adds its term with slot p, so no step needs a reduction:
//   first loop (newest to oldest): s_p.q = s_p.G + sum_i cy_i s_p.y_i,
//     alpha_p = rho_p s_p.q, cy_p = -alpha_p;
//   scaling by g0 = s.y / y.y of the newest pair;
//   second loop (oldest to newest): y_p.r = cg y_p.G + sum_i cy_i y_p.y_i +
//     sum_i cs_i s_i.y_p, cs_p = alpha_p - rho_p y_p.r.
// The state S (LDS) is read by all lanes, written with identical values.
__device__ double lb_direction(LbState& S, LbGram& G, int hist) {
  const int lane = threadIdx.x & 63;
  const int m = S.count;
  const bool mine = lane < hist;
  const double SGl = mine ? S.SG[lane] : 0.0;
  const double YGl = mine ? S.YG[lane] : 0.0;
  const double rhol = mine ? S.rho[lane] : 0.0;
  int p0 = S.head - m;   // slot of the oldest pair
  if (p0 < 0) p0 += hist;
  double cy = 0.0, cs = 0.0, al = 0.0;
  double acc = 0.0;   // lane l: sum over fixed slots i of cy_i s_l.y_i
  int p = p0 + m - 1;
  if (p >= hist) p -= hist;
  // each step's Gram entry is read while the previous step runs
  double gq = (mine && m > 0) ? G.sy(lane, p) : 0.0;
  for (int j = m - 1; j >= 0; --j) {
    const int pu = __builtin_amdgcn_readfirstlane(p);
    const int pn = p == 0 ? hist - 1 : p - 1;
    const double gn = (mine && j > 0) ? G.sy(lane, pn) : 0.0;
    const double a = lane_d(rhol * (SGl + acc), pu);
    if (lane == pu) {
      al = a;
      cy = -a;
    }
    if (mine) acc = fma(-a, gq, acc);
    gq = gn;
    p = pn;
  }
  double cg = 1.0;
  if (m > 0) {
    int sn = p0 + m - 1;
    if (sn >= hist) sn -= hist;
    const double g0 = G.sy(sn, sn) / G.yy(sn, sn);
    cg = g0;
    cy *= g0;
  }
  // lane l: sum_i cy_i y_l.y_i, then the s_i.y_l terms as cs_i are fixed
  double acc2 = 0.0;
  double yq = mine ? G.yy(lane, 0) : 0.0;   // each entry read while the previous step runs
  for (int i = 0; i < hist; ++i) {
    const double yn = (mine && i + 1 < hist) ? G.yy(lane, i + 1) : 0.0;
    const double ci = lane_d(cy, i);
    if (mine) acc2 = fma(ci, yq, acc2);
    yq = yn;
  }
  p = p0;
  gq = (mine && m > 0) ? G.sy(p, lane) : 0.0;
  for (int j = 0; j < m; ++j) {
    const int pu = __builtin_amdgcn_readfirstlane(p);
    const int pn = p + 1 == hist ? 0 : p + 1;
    const double gn = (mine && j + 1 < m) ? G.sy(pn, lane) : 0.0;
    const double csp = lane_d(al - rhol * (cg * YGl + acc2), pu);
    if (lane == pu) cs = csp;
    if (mine) acc2 = fma(csp, gq, acc2);
    gq = gn;
    p = pn;
  }
  const double dG = -cg * S.GG + wave_sum_dd(mine ? -cs * SGl - cy * YGl : 0.0);
  S.cg = -cg;
  if (mine) {
    S.cs[lane] = -cs;
    S.cy[lane] = -cy;
  }
  return dG;
}

// steepest ascent from the accepted point, the L-BFGS memory cleared
__device__ double lb_steepest(LbState& S, const LbParams& P) {
  const int lane = threadIdx.x & 63;
  S.count = 0;
  S.head = 0;
  if (lane < P.hist) S.cs[lane] = S.cy[lane] = 0.0;
  S.cg = -1.0;
  return -S.GG;
}

// start a line search along the direction whose slope is gtd.  Without a
// memory the first trial step is 1 / ||G|| at the start of a solve; after
// the memory was dropped (a restart, a re-centring) it is the curvature
// scale s.y / y.y of the last pair, which near the optimum is orders of
// magnitude below 1 / ||G|| (a search from there could not shrink far
// enough within its trials).
__device__ void lb_start_search(LbState& S, double gtd) {
  S.gtd0 = gtd;
  S.t = (S.count != 0) ? 1.0 : (S.h0 > 0.0 ? S.h0 : 1.0 / sqrt(S.GG));
  S.t_prev = 0.0;
  S.f_prev = S.f;
  S.dp_prev = gtd;
  S.zoom = 0;
  S.nls = 0;
  S.t_next = S.t;
  S.newdir = 1;
}

__device__ void lb_new_direction(LbState& S, LbGram& G, const LbParams& P) {
  double gtd = lb_direction(S, G, P.hist);
  if (!(gtd < 0.0)) gtd = lb_steepest(S, P);   // not a descent direction
  lb_start_search(S, gtd);
}

__device__ void lb_ctrl_logic(const LbArgs& A, int k, LbState& S, LbGram& G, const double* dots,
                              double D) {
  const LbParams& P = A.P;
  S.accept = 0;
  S.push = 0;
  S.newdir = 0;
  const bool l0 = (threadIdx.x & 63) == 0;
  S.mode_eval = A.inst_mode[k];
  __builtin_amdgcn_wave_barrier();
  if (S.status != LB_RUNNING) {
    if (l0) {
      A.inst_mode[k] = EM_SKIP;
      if (S.status == LB_RECENTER) atomicAdd(A.n_active, 1);   // resumes after the re-centring
    }
    S.t_next = 0.0;
    return;
  }
  const double ft = -D;
  const double Gtd = dots[0], GtGt = dots[1], GtG = dots[2], dd = dots[3];
  long long cs[CNT_NUM];
  if (P.stats_trace) lb_counter_sums(A, A.inst[k], cs);
  S.evals++;
  if (!P.use_screen && l0) {
    // unscreened solves evaluate every tile of the live instances without a
    // screen pass, which would otherwise keep these counts
    const InstDev& I = A.inst[k];
    unsigned long long* C = (unsigned long long*)A.counters;
    atomicAdd(&C[CNT_EVALS], 1ull);
    atomicAdd(&C[CNT_PAIRS_TOTAL], (unsigned long long)I.Le * (unsigned long long)I.nt);
    atomicAdd(&C[CNT_TILES_TOTAL], (unsigned long long)I.Le * (unsigned long long)I.njb);
    atomicAdd(&C[CNT_TILES_COMPUTED], (unsigned long long)I.Le * (unsigned long long)I.njb);
  }
  const size_t tr = (size_t)k * (P.max_iter + 1);
  if (!isfinite(D) || !isfinite(GtGt)) {
    if (S.phase == 0) S.f = ft;   // the starting point itself: reported as not finite
    S.status = LB_LSFAIL;
    if (l0) A.inst_mode[k] = EM_SKIP;
    S.t_next = 0.0;
    return;
  }
  if (S.phase == 0 || S.phase == 2) {  // first evaluation, at the starting point (2: after a re-centring)
    const bool restart = S.phase == 2;
    S.phase = 1;
    S.f = ft;
    S.accept = 1;
    S.t_acc = 0.0;
    S.GG = GtGt;
    S.gmax = dots[4];
    S.count = 0;
    S.head = 0;
    if (P.obj_trace && l0 && !restart) P.obj_trace[tr] = D;
    if (P.time_trace && l0 && !restart) P.time_trace[tr] = wall_clock64();
    if (l0 && !restart) lb_write_traces(P, cs, tr, S.gmax);
    if (S.gmax <= P.gtol) {
      S.status = LB_CONVERGED;
    } else if (S.iter >= P.max_iter) {
      S.status = LB_MAXITER;
    }
    if (S.status != LB_RUNNING) {
      if (l0) A.inst_mode[k] = EM_SKIP;
      S.t_next = 0.0;
      return;
    }
    lb_new_direction(S, G, P);
    if (l0) {
      A.inst_mode[k] = P.use_screen ? EM_SCREEN : EM_DENSE;
      atomicAdd(A.n_active, 1);
    }
    S.since_refresh = 0;
    return;
  }
  // strong-Wolfe line search on phi(t) = F(X + t d)
  const double t = S.t, dp = Gtd;
  bool ok = false;
  S.nls++;
  if (S.force) {
    // the best step of a search that ran out of trials, evaluated again
    // (sufficient increase holds there): accept it
    S.force = 0;
    ok = true;
  } else if (!S.zoom) {
    if (ft > S.f + P.c1 * t * S.gtd0 || (S.nls > 1 && ft >= S.f_prev)) {
      S.zoom = 1;
      S.t_lo = S.t_prev; S.f_lo = S.f_prev; S.dp_lo = S.dp_prev;
      S.t_hi = t; S.f_hi = ft; S.dp_hi = dp;
    } else if (fabs(dp) <= -P.c2 * S.gtd0) {
      ok = true;
    } else if (dp >= 0.0) {
      S.zoom = 1;
      S.t_lo = t; S.f_lo = ft; S.dp_lo = dp;
      S.t_hi = S.t_prev; S.f_hi = S.f_prev; S.dp_hi = S.dp_prev;
    } else {
      S.t_prev = t; S.f_prev = ft; S.dp_prev = dp;
      S.t = 4.0 * t;
    }
  } else {
    if (ft > S.f + P.c1 * t * S.gtd0 || ft >= S.f_lo) {
      S.t_hi = t; S.f_hi = ft; S.dp_hi = dp;
    } else {
      if (fabs(dp) <= -P.c2 * S.gtd0) {
        ok = true;
      } else {
        if (dp * (S.t_hi - S.t_lo) >= 0.0) {
          S.t_hi = S.t_lo; S.f_hi = S.f_lo; S.dp_hi = S.dp_lo;
        }
        S.t_lo = t; S.f_lo = ft; S.dp_lo = dp;
      }
    }
  }
  if (!ok) {
    if (S.nls >= P.max_ls) {
      if (S.zoom && S.t_lo > 0.0 && S.f - S.f_lo > 1e-9 * fabs(S.f)) {
        // out of trials inside a bracket: take its best step if it gains
        // more than the rounding noise of the objective
        S.force = 1;
        S.t = S.t_lo;
        S.t_next = S.t;
        if (l0) atomicAdd(A.n_active, 1);
        return;
      }
      if (S.count > 0 && !(S.f_restart - S.f <= 1e-9 * fabs(S.f))) {
        // no step along the quasi-Newton direction: drop the memory and
        // search along the gradient before giving up (once per real gain:
        // at the rounding floor of the objective the search stops)
        S.f_restart = S.f;
        lb_start_search(S, lb_steepest(S, P));
        if (l0) atomicAdd(A.n_active, 1);
        return;
      }
      if (P.recenter && S.n_rec < RECENTER_MAX && S.f_rec - S.f > P.recenter_tol * fabs(S.f)) {
        // the search ran out of float32 resolution around the point: ask
        // for a re-centring there (the host launches it between steps) and
        // continue from it with a fresh memory; a later one only after the
        // objective has gained more than its rounding floor since the last
        S.f_rec = S.f;
        S.n_rec++;
        S.status = LB_RECENTER;
        if (l0) {
          A.inst_mode[k] = EM_SKIP;
          atomicAdd(A.n_active, 1);
          atomicAdd(A.n_recenter, 1);
        }
        S.t_next = 0.0;
        return;
      }
      S.status = LB_LSFAIL;
      if (l0) A.inst_mode[k] = EM_SKIP;
      S.t_next = 0.0;
      return;
    }
    if (S.zoom) S.t = lb_cubic(S.t_lo, S.f_lo, S.dp_lo, S.t_hi, S.f_hi, S.dp_hi);
    S.t_next = S.t;
    if (l0) atomicAdd(A.n_active, 1);
    // the next trial of the same line search keeps the current mode
    return;
  }
  // ---- accepted: X <- trial; history; Gram matrices
  const int h = P.hist;
  S.accept = 1;
  S.t_acc = t;
  S.iter++;
  S.f = ft;
  const double sy = t * (Gtd - S.gtd0);
  const double ss = t * t * dd;
  const double yy = GtGt - 2.0 * GtG + S.GG;
  const int lane = threadIdx.x & 63;
  double SGn = lane < h ? dots[5 + 3 * lane] : 0.0;   // lane i: s_i . G_new
  double YGn = lane < h ? dots[6 + 3 * lane] : 0.0;   // lane i: y_i . G_new
  if (sy > 1e-10 * sqrt(ss * yy) && yy > 0.0) {
    const int sl = S.head;
    // lane i updates the Gram entries between the new pair and pair i
    // (every valid slot except the one being overwritten)
    bool valid = false;
    for (int j = 0; j < S.count; ++j) valid |= (lb_slot(S, h, j) == lane);
    const double old_sg = lane < h ? S.SG[lane] : 0.0, old_yg = lane < h ? S.YG[lane] : 0.0;
    if (lane < h && valid && lane != sl) {
      G.sy(sl, lane) = t * dots[7 + 3 * lane];            // s_new . y_i
      G.sy(lane, sl) = dots[5 + 3 * lane] - old_sg;        // s_i . y_new
      const double yyi = dots[6 + 3 * lane] - old_yg;      // y_new . y_i
      G.yy(sl, lane) = yyi;
      G.yy(lane, sl) = yyi;
    }
    G.sy(sl, sl) = sy;
    G.yy(sl, sl) = yy;
    S.rho[sl] = 1.0 / sy;
    S.h0 = sy / yy;
    if (lane == sl) {
      SGn = t * Gtd;
      YGn = GtGt - GtG;
    }
    S.push = 1;
    S.slot = sl;
    S.head = (S.head + 1) % h;
    if (S.count < h) S.count++;
  }
  if (lane < h) {
    S.SG[lane] = SGn;
    S.YG[lane] = YGn;
  }
  S.GG = GtGt;
  S.gmax = dots[4];
  if (P.obj_trace && l0) P.obj_trace[tr + S.iter] = D;
  if (P.time_trace && l0) P.time_trace[tr + S.iter] = wall_clock64();
  if (l0) lb_write_traces(P, cs, tr + S.iter, dots[4]);
  if (S.gmax <= P.gtol) S.status = LB_CONVERGED;
  else if (S.iter >= P.max_iter) S.status = LB_MAXITER;
  if (S.status != LB_RUNNING) {
    if (l0) A.inst_mode[k] = EM_SKIP;
    S.t_next = 0.0;
    return;
  }
  lb_new_direction(S, G, P);
  int mode = P.use_screen ? EM_SCREEN : EM_DENSE;
  if (P.use_screen && ++S.since_refresh >= P.refresh) {
    S.since_refresh = 0;
    mode = EM_SNAPSHOT;
  }
  if (l0) {
    A.inst_mode[k] = mode;
    atomicAdd(A.n_active, 1);
  }
}

// LDS of one control step (one wavefront per instance; the state lives in
// LDS during the step)
struct LbCtrlShared {
  double dots[5 + 3 * HMAX];
  LbState S;
  double gram[2 * HMAX * HMAX];
};

// LDS ordering between the lanes of the one wavefront that runs a control
// step (a wavefront-level barrier: the step needs no other wavefront)
__device__ __forceinline__ void lb_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The control step of instance k on one wavefront (lanes 0..63 of the
// calling block): sums the dot and objective partials, runs the control
// logic and writes the state and Gram matrices back.
__device__ void lb_ctrl_wave(const LbArgs& A, int k, LbCtrlShared& sh) {
  double* dots = sh.dots;
  LbState& S = sh.S;
  double* gram_s = sh.gram;
  const int h = A.P.hist;
  double* gram_g = A.gram + (size_t)k * 2 * h * h;
  // Every load of the step is issued at once, before any is used: the
  // state, the Gram matrices, the first PD block partials of the lane's dot
  // (lane j: dot j, and dot j + 64) and the first PO x 64 objective
  // partials.  Both partial tables have a fixed capacity per instance, so
  // reads past this instance's count stay in bounds (and are ignored);
  // larger instances take the rest in further rounds.
  constexpr int PD = 16, PO = 4;
  constexpr int NV = (int)(sizeof(LbState) / 16);
  static_assert(NV <= 2 * 64, "state copy assumes at most two int4 per lane");
  const int lane = threadIdx.x & 63;
  const int ng = 2 * h * h;
  const double* pk = A.part + (size_t)k * A.ndot * A.maxb;
  const bool has1 = lane < A.ndot, has2 = lane + 64 < A.ndot;
  const double* p1 = pk + (size_t)lane * A.maxb;
  const double* p2 = pk + (size_t)(lane + 64) * A.maxb;
  const double* osrc = A.obj_part + (size_t)k * A.obj_stride;
  int4 w0, w1;
  double g[32], pd[PD], pd2[PD], po[PO];
  {
    const int4* src = (const int4*)&A.st[k];
    w0 = src[lane];
    w1 = lane + 64 < NV ? src[lane + 64] : int4{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int q = u * 64 + lane;
      g[u] = q < ng ? gram_g[q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      pd[u] = (has1 && u < A.maxb) ? p1[u] : 0.0;
      pd2[u] = (has2 && u < A.maxb) ? p2[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PO; ++u) {
      const int i = u * 64 + lane;
      po[u] = i < A.obj_stride ? osrc[i] : 0.0;
    }
  }
  const InstDev I = A.inst[k];
  {
    int4* dst = (int4*)&S;
    dst[lane] = w0;
    if (lane + 64 < NV) dst[lane + 64] = w1;
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int q = u * 64 + lane;
      if (q < ng) gram_s[q] = g[u];
    }
  }
  LbGram G{gram_s, gram_s + h * h, h};
  // lane j: dot j summed over the vector blocks in block order (dot 4 is a
  // maximum), and dot j + 64 likewise
  const int nb = (I.ns + I.nt_pad + LB_VB - 1) / LB_VB;
  double acc = 0.0, acc2 = 0.0;
#pragma unroll
  for (int u = 0; u < PD; ++u) {
    if (u < nb) {
      acc = lane == 4 ? fmax(acc, pd[u]) : acc + pd[u];
      acc2 += pd2[u];
    }
  }
  for (int b0 = PD; b0 < nb; b0 += PD) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      pd[u] = (has1 && b0 + u < nb) ? p1[b0 + u] : 0.0;
      pd2[u] = (has2 && b0 + u < nb) ? p2[b0 + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      if (b0 + u < nb) {
        acc = lane == 4 ? fmax(acc, pd[u]) : acc + pd[u];
        acc2 += pd2[u];
      }
    }
  }
  if (has1) dots[lane] = acc;
  if (has2) dots[lane + 64] = acc2;
  // D: lane sums the partials i = lane (mod 64) in order, then the
  // fixed-order wavefront sum (as wherever D is formed)
  const int nob = asm_obj_parts(I);
  double os = 0.0;
#pragma unroll
  for (int u = 0; u < PO; ++u)
    if (u * 64 + lane < nob) os += po[u];
  for (int i = PO * 64 + lane; i < nob; i += 64) os += osrc[i];
  const double Dobj = wave_sum_dd(os) + (A.obj_const ? A.obj_const[k] : 0.0);
  lb_wave_sync();
  if (lane == 0) A.obj_out[k] = Dobj;
  lb_ctrl_logic(A, k, S, G, dots, Dobj);
  lb_wave_sync();
  for (int q = lane; q < 2 * h * h; q += 64) gram_g[q] = gram_s[q];
  {
    const int4* src = (const int4*)&S;
    int4* dst = (int4*)&A.st[k];
    for (int i = lane; i < (int)(sizeof(LbState) / 16); i += 64) dst[i] = src[i];
  }
}

__global__ void __launch_bounds__(64) k_lbfgs_ctrl(LbArgs A) {
  __shared__ LbCtrlShared sh;
  lb_ctrl_wave(A, blockIdx.x, sh);
}
// the vector work of one element e of instance k: record the snapshot,
// accept the trial point, push (s, y), form the new direction and the next
// trial point; returns the new trial value and, in snap_out, alpha~ after
// this step
__device__ __forceinline__ float lb_update_elem(const LbArgs& A, const InstDev& I, const LbState& S, int e,
                                                long long v0, int h, bool snap, bool wu, float& snap_out) {
  float* tp = e < I.ns ? &A.alpha[I.row_off + e] : &A.beta[I.col_off + (e - I.ns)];
  float* sp = e < I.ns ? &A.alpha_s[I.row_off + e] : &A.beta_s[I.col_off + (e - I.ns)];
  const float told = *tp;
  if (snap) *sp = told;   // the point just evaluated densely becomes the snapshot
  snap_out = snap ? told : *sp;
  const float w = wu ? 1.f : A.W[v0 + e];
  float x = A.X[v0 + e];
  if (S.accept) {
    const float gt = lb_gt(A, I, e) * w;
    // the accepted trial point, formed again exactly as when it was evaluated
    x = x + (float)S.t_acc * A.Dv[v0 + e];
    if (S.push) {
      A.S[(size_t)S.slot * A.vtot + v0 + e] = (float)S.t_acc * A.Dv[v0 + e];
      A.Y[(size_t)S.slot * A.vtot + v0 + e] = gt - A.G[v0 + e];
    }
    A.X[v0 + e] = x;
    A.G[v0 + e] = gt;
  }
  if (S.newdir) {
    // d = cg G + sum over ring slots (in age order) of cs_i s_i + cy_i y_i
    double d = S.cg * (double)A.G[v0 + e];
    const int cnt = S.count;
#pragma unroll 8
    for (int j = 0; j < cnt; ++j) {
      const int i = lb_slot(S, h, j);
      d += S.cs[i] * (double)A.S[(size_t)i * A.vtot + v0 + e] +
           S.cy[i] * (double)A.Y[(size_t)i * A.vtot + v0 + e];
    }
    A.Dv[v0 + e] = (float)d;
  }
  const float xn = w * (x + (float)S.t_next * A.Dv[v0 + e]);
  *tp = xn;
  return xn;
}

// the update of elements e0, e0 + stride, ... of instance k
__device__ __forceinline__ void lb_update_elems(const LbArgs& A, const InstDev& I, int k, int e0, int stride) {
  const LbState& S = A.st[k];
  const int n = I.ns + I.nt_pad;
  const long long v0 = A.voff[k];
  const int h = A.P.hist;
  const bool snap = S.mode_eval == EM_SNAPSHOT;
  const bool wu = A.w_unit[k] != 0;
  if (lb_update_idle(A, S)) return;
  for (int e = e0; e < n; e += stride) {
    float so;
    lb_update_elem(A, I, S, e, v0, h, snap, wu, so);
  }
}

// grid (vector blocks, count); accept, push, new direction, next trial point
__global__ void __launch_bounds__(256) k_lbfgs_update(LbArgs A) {
  const int k = blockIdx.y;
  const InstDev I = A.inst[k];
  lb_update_elems(A, I, k, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// The same update, with the group statistics of alpha - alpha~ that the
// next screened evaluation needs formed on the way (handles whose groups
// all have at most CHUNK rows).  grid (max groups + max column blocks,
// count): block g < L_e takes the rows of group g (thread t the rows
// g_start + t + 256 j, then the same fixed-order tree as k_group_stats, so
// the statistics are bit-identical to that kernel's), the others 256
// columns each.  Block (0, 0) also resets the work-list counts of the next
// screen pass, and each instance's group-0 block counts its next
// evaluation, as k_group_stats does.
template <int GT>
__global__ void __launch_bounds__(GT) k_lbfgs_update_gs(LbArgs A) {
  __shared__ double sm[4][GT / 64];
  const int k = blockIdx.y;
  const InstDev I = A.inst[k];
  const LbState& S = A.st[k];
  const long long v0 = A.voff[k];
  const int h = A.P.hist;
  const bool snap = S.mode_eval == EM_SNAPSHOT;
  const bool wu = A.w_unit[k] != 0;
  const int bx = blockIdx.x;
  if (bx == 0 && k == 0 && threadIdx.x < NBUCKET + 2) A.counts[threadIdx.x] = 0;
  if (lb_update_idle(A, S)) return;
  if (bx >= A.max_le) {
    const int c = (bx - A.max_le) * GT + threadIdx.x;
    if (c < I.nt_pad) {
      float so;
      lb_update_elem(A, I, S, I.ns + c, v0, h, snap, wu, so);
    }
    return;
  }
  if (bx >= I.Le) return;
  const int gidx = I.grp_off + bx;
  const int r0 = A.g_start[gidx], n = A.g_size[gidx];
  double up = 0, dn = 0, am = 0, ams = 0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    float as;
    const double a = lb_update_elem(A, I, S, r0 + q, v0, h, snap, wu, as);
    const double d = a - (double)as;
    if (d > 0) up += d * d; else dn += d * d;
    am = fmax(am, fabs(a));
    ams = fmax(ams, fabs((double)as));
  }
  gs_reduce<GT>(up, dn, am, ams, sm);
  if (threadIdx.x == 0) {
    GroupStats g;
    g.up = sqrt(up);
    g.dn = sqrt(dn);
    g.all = sqrt(up + dn);
    g.amax = am;
    g.amax_s = ams;
    screen_group_consts(n, g.sg, g.fa, g.fb);
    A.gstats[gidx] = g;
    if (bx == 0) {
      const int m = A.inst_mode[k];
      if (m != EM_SKIP) atomicAdd((unsigned long long*)&A.counters[CNT_EVALS], 1ull);
      if (m == EM_SNAPSHOT) atomicAdd((unsigned long long*)&A.counters[CNT_REFRESH], 1ull);
    }
  }
}

// Variable scales of the iteration (see the top of this file): w = 1 /
// sqrt(M m_e) for the marginal m_e of element e, M = (n_src + n_tgt) / 2,
// formed in float64 and rounded once; exactly 1 for uniform marginals with
// n_src = n_tgt; 1 on padding columns and where a marginal is 0.
__global__ void __launch_bounds__(256) k_lbfgs_weights(const InstDev* __restrict__ inst,
                                                       const long long* __restrict__ voff,
                                                       const float* __restrict__ a_int,
                                                       const float* __restrict__ b_int,
                                                       const int* __restrict__ a_uniform,
                                                       const int* __restrict__ b_uniform, float* __restrict__ W) {
  const int k = blockIdx.y;
  const InstDev I = inst[k];
  const long long v0 = voff[k];
  const double M = 0.5 * ((double)I.ns + (double)I.nt);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < I.ns + I.nt_pad; e += gridDim.x * blockDim.x) {
    double m;
    if (e < I.ns) m = a_uniform[k] ? 1.0 / I.ns : (double)a_int[I.row_off + e];
    else if (e - I.ns < I.nt) m = b_uniform[k] ? 1.0 / I.nt : (double)b_int[I.col_off + (e - I.ns)];
    else m = 0.0;
    W[v0 + e] = m > 0.0 ? (float)(1.0 / sqrt(M * m)) : 1.0f;
  }
}

// X -> trial arrays (alpha, beta), for the export at the end of a solve
__global__ void __launch_bounds__(256) k_lbfgs_export(LbArgs A) {
  const int k = blockIdx.y;
  const InstDev I = A.inst[k];
  const long long v0 = A.voff[k];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < I.ns + I.nt_pad; e += gridDim.x * blockDim.x) {
    const float xw = A.W[v0 + e] * A.X[v0 + e];
    const float x = A.xref ? (float)(A.xref[v0 + e] + (double)xw) : xw;
    if (e < I.ns) A.alpha[I.row_off + e] = x;
    else A.beta[I.col_off + (e - I.ns)] = x;
  }
}

// start of a solve: state, snapshot and set N cleared; X = trial point
// (zeros or the caller's point already gathered into alpha/beta).
__global__ void __launch_bounds__(256) k_lbfgs_init(LbArgs A, int init_user, float* alpha_s,
                                                    float* beta_s, float* zsnap, float* osnap,
                                                    uint8_t* inN, int use_screen) {
  const int k = blockIdx.y;
  const InstDev I = A.inst[k];
  const int n = I.ns + I.nt_pad;
  const long long v0 = A.voff[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    LbState& S = A.st[k];
    S.status = LB_RUNNING;
    S.phase = 0;
    S.iter = S.evals = S.nls = S.zoom = 0;
    S.count = S.head = 0;
    S.accept = S.push = S.newdir = 0;
    S.force = 0;
    S.f_restart = INFINITY;
    S.f_rec = INFINITY;
    S.n_rec = 0;
    S.h0 = 0.0;
    if (A.obj_const) A.obj_const[k] = 0.0;
    S.since_refresh = 0;
    S.t_next = 0.0;
    S.GG = 0.0;
    for (int i = 0; i < HMAX; ++i) S.SG[i] = S.YG[i] = S.rho[i] = S.cs[i] = S.cy[i] = 0.0;
    for (int q = 0; q < 2 * A.P.hist * A.P.hist; ++q) A.gram[(size_t)k * 2 * A.P.hist * A.P.hist + q] = 0.0;
    // zero start: the zero snapshot is exact (z~ = 0 since C >= 0); a user
    // start is evaluated densely and taken as the first snapshot
    A.inst_mode[k] = !use_screen ? EM_DENSE : (init_user ? EM_SNAPSHOT : EM_SCREEN);
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    float* tp = e < I.ns ? &A.alpha[I.row_off + e] : &A.beta[I.col_off + (e - I.ns)];
    if (!init_user) *tp = 0.f;
    if (A.xref) A.xref[v0 + e] = 0.0;
    const bool pad = e >= I.ns && (e - I.ns) >= I.nt;
    if (pad) *tp = 0.f;
    A.X[v0 + e] = *tp / A.W[v0 + e];
    A.G[v0 + e] = 0.f;
    A.Dv[v0 + e] = 0.f;
    if (e < I.ns) alpha_s[I.row_off + e] = 0.f;
    else beta_s[I.col_off + (e - I.ns)] = 0.f;
  }
  const long long np = (long long)I.Le * I.nt_pad;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < np;
       q += (long long)gridDim.x * blockDim.x) {
    zsnap[I.pair_off + q] = 0.f;
    osnap[I.pair_off + q] = 0.f;
    inN[I.pair_off + q] = 0;
  }
}

// Re-centring (materialised cost).  A float32 iterate moves on a grid of
// spacing ulp(alpha) ~ 6e-8 |alpha|, while near the optimum the dual's
// remaining increase can need finer moves than that: the line search then
// finds no step although D* is not reached.  The point is therefore split as
// xref + current (xref in float64): the evaluations see the current part and
// the reduced cost c'_ij = fl32(c_ij - xref_i - xref_j) (psi depends on
// alpha_i + beta_j - c_ij only, so it is the same function, up to one
// rounding of c'), and D adds a.xref_alpha + b.xref_beta.  The current part is
// small, so its float32 grid is fine.  Runs between solver steps, for the
// instances whose control step asked for it (status LB_RECENTER).
//
// Vector part, one workgroup per instance: xref += w x, x = 0, the trial
// point and snapshot point zero, the snapshot norms and N cleared (N = {}
// until the next refresh; the first evaluation takes a new snapshot), the
// objective constant advanced by the marginals' dot with the move (fixed
// order), and the state restarted (phase 2: a fresh memory at this point).
__global__ void __launch_bounds__(1024) k_recenter_vec(LbArgs A, const float* __restrict__ a_int,
                                                       const float* __restrict__ b_int,
                                                       const int* __restrict__ a_uniform,
                                                       const int* __restrict__ b_uniform, float* zsnap,
                                                       float* osnap, uint8_t* inN, float* cmax_w) {
  __shared__ double red[16];
  const int k = blockIdx.x;
  LbState& S = A.st[k];
  if (S.status != LB_RECENTER) return;
  const InstDev I = A.inst[k];
  const long long v0 = A.voff[k];
  double part = 0.0;
  for (int e = threadIdx.x; e < I.ns + I.nt_pad; e += blockDim.x) {
    const float d = A.W[v0 + e] * A.X[v0 + e];   // the accepted point as evaluated
    A.xref[v0 + e] += (double)d;
    A.X[v0 + e] = 0.f;
    A.Dv[v0 + e] = 0.f;
    double m = 0.0;
    if (e < I.ns) {
      m = a_uniform[k] ? 1.0 / I.ns : (double)a_int[I.row_off + e];
      A.alpha[I.row_off + e] = 0.f;
      A.alpha_s[I.row_off + e] = 0.f;
    } else {
      const int c = e - I.ns;
      m = c < I.nt ? (b_uniform[k] ? 1.0 / I.nt : (double)b_int[I.col_off + c]) : 0.0;
      A.beta[I.col_off + c] = 0.f;
      A.beta_s[I.col_off + c] = 0.f;
    }
    part += m * (double)d;
  }
  const long long np = (long long)I.Le * I.nt_pad;
  for (long long q = threadIdx.x; q < np; q += blockDim.x) {
    zsnap[I.pair_off + q] = 0.f;
    osnap[I.pair_off + q] = 0.f;
    inN[I.pair_off + q] = 0;
  }
  part = wave_sum_dd(part);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    A.obj_const[k] += t;
    cmax_w[k] = 0.f;
    S.phase = 2;
    S.count = S.head = 0;
    S.nls = S.zoom = 0;
    S.accept = S.push = S.newdir = S.force = 0;
    S.since_refresh = 0;
    S.t_next = 0.0;
    A.inst_mode[k] = A.P.use_screen ? EM_SNAPSHOT : EM_DENSE;
  }
}

// Cost part, grid (column blocks, rows, count): c' = fl32(c - xref_i -
// xref_j) from the original pool for the instances just re-centred (phase 2
// and still waiting), and their largest |c'| (the rounding margin of the
// screen's upper bound takes it in place of max C).  The last launch of a
// re-centring also sets them running.
__global__ void __launch_bounds__(256) k_recenter_cost(LbArgs A, const float* __restrict__ C, float* __restrict__ Cw,
                                                       const int* __restrict__ row_grp, const int* __restrict__ g_start,
                                                       const int* __restrict__ g_size, float* cmax_w, int all) {
  const int k = blockIdx.z;
  const LbState& S = A.st[k];
  if (!all && (S.status != LB_RECENTER || S.phase != 2)) return;
  const InstDev I = A.inst[k];
  const long long v0 = A.voff[k];
  float mx = 0.f;
  for (int r = blockIdx.y; r < I.ns; r += gridDim.y) {
    const int g = row_grp[I.row_off + r];
    const int gs = g_start[I.grp_off + g], gn = g_size[I.grp_off + g];
    const double xr = A.xref[v0 + r];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < I.nt; c += gridDim.x * blockDim.x) {
      const size_t q = c_index(I, gs, gn, r, c);
      const float v = (float)((double)C[q] - xr - A.xref[v0 + I.ns + c]);
      Cw[q] = v;
      mx = fmaxf(mx, fabsf(v));
    }
  }
  // one atomic per workgroup (the maximum is order-free): a wavefront-level
  // atomic from every wavefront of a large grid serialised on one address
  __shared__ float wm[4];
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float m = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
    atomicMax((unsigned int*)&cmax_w[k], __float_as_uint(m));
  }
}

// (all = 1: every instance, rebuilding the working cost of a solver state
// restored from a checkpoint, whose reference is xref; an instance never
// re-centred has xref = 0 and gets C itself)

// Re-centred instances resume (after the cost kernel).
__global__ void k_recenter_resume(LbArgs A, int count) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) {
    LbState& S = A.st[k];
    if (S.status == LB_RECENTER && S.phase == 2) S.status = LB_RUNNING;
  }
}

// Continuing a solve from the state an earlier one left (ot_gs_solve with
// resume; the state may come from a checkpoint).  One wavefront per
// instance.  An instance that stopped at the iteration limit takes the part
// of its last control step the limit cut short - the new direction from the
// accepted point and the evaluation mode, exactly as after an acceptance -
// if the new limit lets it go on.  Every live instance's next evaluation is
// a snapshot: the snapshot on the handle need not belong to this state, and
// a snapshot evaluation is dense, so the iterates stay the same bits
// (Lemma 2).  The accept / push flags of the last step were already applied
// by its update, so they are cleared: the update that follows forms only
// the direction (if new) and the trial point, and records no snapshot.
__global__ void __launch_bounds__(64) k_lbfgs_resume(LbArgs A) {
  __shared__ LbState S;
  __shared__ double gram_s[2 * HMAX * HMAX];
  const int k = blockIdx.x, lane = threadIdx.x;
  const int h = A.P.hist;
  const LbParams& P = A.P;
  constexpr int NV = (int)(sizeof(LbState) / 16);
  {
    const int4* src = (const int4*)&A.st[k];
    int4* dst = (int4*)&S;
    for (int i = lane; i < NV; i += 64) dst[i] = src[i];
    const double* gram_g = A.gram + (size_t)k * 2 * h * h;
    for (int q = lane; q < 2 * h * h; q += 64) gram_s[q] = gram_g[q];
  }
  __syncthreads();
  const int st0 = S.status;
  const bool cont = st0 == LB_MAXITER && S.iter < P.max_iter;
  __syncthreads();
  S.accept = 0;
  S.push = 0;
  S.newdir = 0;
  S.mode_eval = EM_SKIP;
  __builtin_amdgcn_wave_barrier();
  bool live = st0 == LB_RUNNING;
  if (cont) {
    S.status = LB_RUNNING;
    LbGram G{gram_s, gram_s + h * h, h};
    lb_new_direction(S, G, P);
    if (P.use_screen && ++S.since_refresh >= P.refresh) S.since_refresh = 0;
    live = true;
  } else if (!live) {
    S.t_next = 0.0;
  }
  __syncthreads();
  double* gram_g = A.gram + (size_t)k * 2 * h * h;
  for (int q = lane; q < 2 * h * h; q += 64) gram_g[q] = gram_s[q];
  {
    const int4* src = (const int4*)&S;
    int4* dst = (int4*)&A.st[k];
    for (int i = lane; i < NV; i += 64) dst[i] = src[i];
  }
  if (lane == 0) {
    A.inst_mode[k] = live ? (P.use_screen ? EM_SNAPSHOT : EM_DENSE) : EM_SKIP;
    if (live) atomicAdd(A.n_active, 1);
  }
}

}  // namespace otgs
