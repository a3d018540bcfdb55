// A second solver under the same screened evaluations: accelerated gradient
// ascent on the dual.  The screening of Algorithms 1-2 only changes how an
// evaluation is computed, never its result (Lemma 2), so it composes with
// any solver that evaluates D and its gradient (Theorem 1 and the remark
// after it, Sec. 3.4); this one shows it with a method of a different kind
// than L-BFGS.
//
// The method (the paper fixes none; the steps are Nesterov's momentum in the
// form of Beck and Teboulle's FISTA, with backtracking on the step and the
// function-value restart of O'Donoghue and Candes), in the marginal-scaled
// variables u of the L-BFGS solver (x = w u, q(u) = w grad D(w u)):
//   start: u_0, D_0, L = ||q(u_0)||_2, v = u_0, t = 1;
//   trial u+ = v + q(v) / L; while D(u+) < D(v) + ||q(v)||^2 / (2 L): L <- 2 L;
//   if D(u+) < D_k and v is not u_k: t = 1, v = u_k, trial again;
//   else accept u_{k+1} = u+, t' = (1 + sqrt(1 + 4 t^2)) / 2,
//        v = u_{k+1} + ((t - 1) / t') (u_{k+1} - u_k), t = t', L <- shrink L.
// Accepted objectives never decrease.  Every evaluation (at v or at a trial)
// runs through the same screen / tile / assembly kernels as the L-BFGS
// solver's, so a screened solve follows the dense one bit for bit.
//
// One solver step = one evaluation + k_agd_dots (||q||^2 and max |grad D|
// per vector block, float64) + k_agd_ctrl (one wavefront per instance: the
// scalar logic above, deciding the vector action) + k_agd_update (the
// action on the vectors and the next evaluation point).
#include "otgs_internal.h"

namespace otgs {

enum AgdPhase { AG_START = 0, AG_AT_V = 1, AG_AT_TRIAL = 2 };
// what the update does with the vectors after a control step
enum AgdAction {
  AA_NONE = 0,
  AA_START = 1,        // q(u_0) -> Qk, Qv; trial from v = u_0
  AA_AT_V = 2,         // q(v) -> Qv; trial from v
  AA_RETRY = 3,        // trial from v with the doubled L
  AA_RESTART = 4,      // v <- u_k, Qv <- Qk; trial from v
  AA_ACCEPT_STEP = 5,  // u_k <- u+, Qk <- q(u+); v = u+ (no momentum): Qv <- q(u+), trial from v
  AA_ACCEPT_EXTRAP = 6,// u_k <- u+, Qk <- q(u+); v = u+ + mom (u+ - u_k), evaluated next
  AA_ACCEPT_FINAL = 7  // u_k <- u+, Qk <- q(u+); the solve ends
};

struct AgdState {
  int status, phase, iter, evals;
  int bt, at_k, since_refresh, action;
  double L, t, mom;
  double Dk, qq_k;      // D and ||q||^2 at the accepted point u_k
  double Dv, qq_v;      // at the point v the trials start from
  double gmax;          // max |grad D| at u_k (unscaled)
  double inv_l;         // 1 / L of the trial the update forms
};

struct AgdArgs {
  LbArgs A;          // vectors, scales, evaluation outputs, traces, counters
  AgdState* st;
  int max_bt;        // doublings of L per trial before the solve stops
  int momentum;      // 0: no extrapolation
  double shrink;     // L <- shrink L after an accepted step
};

// vector roles in the L-BFGS solver's buffers (scaled variables)
//   U  = X          accepted point u_k
//   Qk = G          q at u_k
//   V  = Dv         point v the trials start from
//   Qv = S slot 0   q at v
//   Ut = Y slot 0   trial point u+
struct AgdVec {
  float *U, *Qk, *V, *Qv, *Ut;
};
__device__ __forceinline__ AgdVec agd_vec(const LbArgs& A, long long v0) {
  return AgdVec{A.X + v0, A.G + v0, A.Dv + v0, A.S + v0, A.Y + v0};
}

// ascent gradient of the evaluation just done at element e (scaled variables)
__device__ __forceinline__ float agd_q(const LbArgs& A, const InstDev& I, int e, float w) {
  return -lb_gt(A, I, e) * w;
}

// grid (vector blocks, count), one wavefront per block: dot 0 = sum q^2
// (float64, each lane its LB_PER_THREAD elements in order, then the
// fixed-order wavefront sum), dot 1 = max |grad D|; partials [k][dot][maxb]
__global__ void __launch_bounds__(LB_BLOCK) k_agd_dots(AgdArgs G) {
  const LbArgs& A = G.A;
  const int k = blockIdx.y, b = blockIdx.x, lane = threadIdx.x;
  const InstDev I = A.inst[k];
  const long long v0 = A.voff[k];
  const int n = I.ns + I.nt_pad;
  if (b * LB_VB >= n) return;
  const bool wu = A.w_unit[k] != 0;
  const bool run = G.st[k].status == LB_RUNNING;
  double qq = 0.0;
  float gm = 0.f;
#pragma unroll
  for (int q = 0; q < LB_PER_THREAD; ++q) {
    const int e = b * LB_VB + q * LB_BLOCK + lane;
    if (e < n && run) {
      const float g0 = lb_gt(A, I, e);
      const float qe = -g0 * (wu ? 1.f : A.W[v0 + e]);
      gm = fmaxf(gm, fabsf(g0));
      qq += (double)qe * qe;
    }
  }
  qq = wave_sum_dd(qq);
  const double g4 = wave_max_d((double)gm);
  double* out = A.part + (size_t)k * A.ndot * A.maxb + b;
  if (lane == 0) out[0] = qq;
  if (lane == 1) out[A.maxb] = g4;
}

// one wavefront per instance
__global__ void __launch_bounds__(64) k_agd_ctrl(AgdArgs G) {
  const LbArgs& A = G.A;
  const LbParams& P = A.P;
  const int k = blockIdx.x, lane = threadIdx.x;
  const InstDev I = A.inst[k];
  AgdState S = G.st[k];
  const bool l0 = lane == 0;
  S.action = AA_NONE;
  if (S.status != LB_RUNNING) {
    if (l0) {
      A.inst_mode[k] = EM_SKIP;
      G.st[k] = S;
    }
    return;
  }
  // the two dots over the vector blocks in block order, and D from the
  // assembly partials (fixed-order sums, as the L-BFGS control step forms D)
  const int nb = (I.ns + I.nt_pad + LB_VB - 1) / LB_VB;
  const double* pk = A.part + (size_t)k * A.ndot * A.maxb;
  double qq = 0.0, gmax = 0.0;
  if (l0) {
    for (int b = 0; b < nb; ++b) {
      qq += pk[b];
      gmax = fmax(gmax, pk[A.maxb + b]);
    }
  }
  qq = __shfl(qq, 0);
  gmax = __shfl(gmax, 0);
  const int nob = asm_obj_parts(I);
  const double* osrc = A.obj_part + (size_t)k * A.obj_stride;
  double os = 0.0;
  for (int i = lane; i < nob; i += 64) os += osrc[i];
  const double D = wave_sum_dd(os);
  long long cs[CNT_NUM];
  if (P.stats_trace) lb_counter_sums(A, I, cs);
  if (!l0) return;
  A.obj_out[k] = D;
  S.evals++;
  if (!P.use_screen) {
    unsigned long long* C = (unsigned long long*)A.counters;
    atomicAdd(&C[CNT_EVALS], 1ull);
    atomicAdd(&C[CNT_PAIRS_TOTAL], (unsigned long long)I.Le * (unsigned long long)I.nt);
    atomicAdd(&C[CNT_TILES_TOTAL], (unsigned long long)I.Le * (unsigned long long)I.njb);
    atomicAdd(&C[CNT_TILES_COMPUTED], (unsigned long long)I.Le * (unsigned long long)I.njb);
  }
  const size_t tr = (size_t)k * (P.max_iter + 1);
  int next = P.use_screen ? EM_SCREEN : EM_DENSE;
  bool ends = false;
  if (!isfinite(D) || !isfinite(qq)) {
    if (S.phase == AG_START) S.Dk = D;
    S.status = LB_LSFAIL;
    ends = true;
  } else if (S.phase == AG_START) {
    S.Dk = S.Dv = D;
    S.qq_k = S.qq_v = qq;
    S.gmax = gmax;
    S.L = sqrt(qq);
    S.t = 1.0;
    S.at_k = 1;
    S.bt = 0;
    if (P.obj_trace) P.obj_trace[tr] = D;
    if (P.time_trace) P.time_trace[tr] = wall_clock64();
    lb_write_traces(P, cs, tr, gmax);
    if (gmax <= P.gtol || !(S.L > 0.0)) {
      S.status = LB_CONVERGED;
      ends = true;
    } else if (P.max_iter <= 0) {
      S.status = LB_MAXITER;
      ends = true;
    } else {
      S.action = AA_START;
      S.phase = AG_AT_TRIAL;
    }
  } else if (S.phase == AG_AT_V) {
    S.Dv = D;
    S.qq_v = qq;
    S.bt = 0;
    S.action = AA_AT_V;
    S.phase = AG_AT_TRIAL;
  } else if (D < S.Dv + S.qq_v / (2.0 * S.L)) {
    // not enough ascent for this step length: halve it
    if (++S.bt > G.max_bt) {
      S.status = LB_LSFAIL;
      ends = true;
    } else {
      S.L *= 2.0;
      S.action = AA_RETRY;
    }
  } else if (D < S.Dk && !S.at_k) {
    // below the accepted point: drop the momentum and step from u_k
    S.t = 1.0;
    S.at_k = 1;
    S.Dv = S.Dk;
    S.qq_v = S.qq_k;
    S.bt = 0;
    S.action = AA_RESTART;
  } else {
    S.iter++;
    S.Dk = D;
    S.qq_k = qq;
    S.gmax = gmax;
    if (P.obj_trace) P.obj_trace[tr + S.iter] = D;
    if (P.time_trace) P.time_trace[tr + S.iter] = wall_clock64();
    lb_write_traces(P, cs, tr + S.iter, gmax);
    const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * S.t * S.t));
    S.mom = G.momentum ? (S.t - 1.0) / tn : 0.0;
    S.t = tn;
    S.L *= G.shrink;
    S.bt = 0;
    if (P.use_screen && ++S.since_refresh >= P.refresh) {
      S.since_refresh = 0;
      next = EM_SNAPSHOT;
    }
    if (gmax <= P.gtol) {
      S.status = LB_CONVERGED;
      S.action = AA_ACCEPT_FINAL;
      ends = true;
    } else if (S.iter >= P.max_iter) {
      S.status = LB_MAXITER;
      S.action = AA_ACCEPT_FINAL;
      ends = true;
    } else if (S.mom == 0.0) {
      S.at_k = 1;
      S.Dv = D;
      S.qq_v = qq;
      S.action = AA_ACCEPT_STEP;
    } else {
      S.at_k = 0;
      S.action = AA_ACCEPT_EXTRAP;
      S.phase = AG_AT_V;
    }
  }
  S.inv_l = S.L > 0.0 ? 1.0 / S.L : 0.0;
  G.st[k] = S;
  if (ends) {
    A.inst_mode[k] = EM_SKIP;
  } else {
    A.inst_mode[k] = next;
    atomicAdd(A.n_active, 1);
  }
}

// grid (vector blocks, count): the action of the control step on each
// element, and the next evaluation point x = w * point (internal order)
__global__ void __launch_bounds__(256) k_agd_update(AgdArgs G) {
  const LbArgs& A = G.A;
  const int k = blockIdx.y;
  const AgdState& S = G.st[k];
  const int action = S.action;
  if (action == AA_NONE) return;
  const InstDev I = A.inst[k];
  const long long v0 = A.voff[k];
  const int n = I.ns + I.nt_pad;
  const bool wu = A.w_unit[k] != 0;
  const float il = (float)S.inv_l, mom = (float)S.mom;
  const AgdVec V = agd_vec(A, v0);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const float w = wu ? 1.f : A.W[v0 + e];
    float* tp = e < I.ns ? &A.alpha[I.row_off + e] : &A.beta[I.col_off + (e - I.ns)];
    const bool pad = e >= I.ns && (e - I.ns) >= I.nt;
    float pt;   // next point to evaluate (scaled)
    bool eval = true;
    switch (action) {
      case AA_START: {
        const float q = agd_q(A, I, e, w);
        V.Qk[e] = q;
        V.Qv[e] = q;
        pt = V.V[e] + q * il;
        V.Ut[e] = pt;
        break;
      }
      case AA_AT_V: {
        const float q = agd_q(A, I, e, w);
        V.Qv[e] = q;
        pt = V.V[e] + q * il;
        V.Ut[e] = pt;
        break;
      }
      case AA_RETRY:
        pt = V.V[e] + V.Qv[e] * il;
        V.Ut[e] = pt;
        break;
      case AA_RESTART: {
        const float u = V.U[e], qk = V.Qk[e];
        V.V[e] = u;
        V.Qv[e] = qk;
        pt = u + qk * il;
        V.Ut[e] = pt;
        break;
      }
      case AA_ACCEPT_STEP: {
        const float un = V.Ut[e], q = agd_q(A, I, e, w);
        V.U[e] = un;
        V.Qk[e] = q;
        V.V[e] = un;
        V.Qv[e] = q;
        pt = un + q * il;
        V.Ut[e] = pt;
        break;
      }
      case AA_ACCEPT_EXTRAP: {
        const float un = V.Ut[e], uo = V.U[e], q = agd_q(A, I, e, w);
        V.U[e] = un;
        V.Qk[e] = q;
        pt = un + mom * (un - uo);
        V.V[e] = pt;
        break;
      }
      default: {   // AA_ACCEPT_FINAL
        V.U[e] = V.Ut[e];
        V.Qk[e] = agd_q(A, I, e, w);
        eval = false;
        pt = 0.f;
        break;
      }
    }
    if (eval) *tp = pad ? 0.f : w * pt;
  }
}

// start of a solve (after k_lbfgs_init has set X = u_0, the trial point, the
// snapshot and the first mode): v = u_0 and the state
__global__ void __launch_bounds__(256) k_agd_init(AgdArgs G) {
  const LbArgs& A = G.A;
  const int k = blockIdx.y;
  const InstDev I = A.inst[k];
  const long long v0 = A.voff[k];
  const int n = I.ns + I.nt_pad;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    AgdState S;
    S.status = LB_RUNNING;
    S.phase = AG_START;
    S.iter = S.evals = S.bt = S.since_refresh = 0;
    S.at_k = 1;
    S.action = AA_NONE;
    S.L = S.t = 1.0;
    S.mom = 0.0;
    S.Dk = S.qq_k = S.Dv = S.qq_v = S.gmax = 0.0;
    S.inv_l = 1.0;
    G.st[k] = S;
  }
  const AgdVec V = agd_vec(A, v0);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    V.V[e] = V.U[e];
    V.Qk[e] = V.Qv[e] = V.Ut[e] = 0.f;
  }
}

}  // namespace otgs
