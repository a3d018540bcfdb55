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
#include "otgs_internal.h"

namespace otgs {

constexpr int HMAX = 32;
constexpr int LB_BLOCK = 256;
constexpr int LB_PER_THREAD = 8;
constexpr int LB_VB = LB_BLOCK * LB_PER_THREAD;   // vector elements per dots block

enum LbStatus { LB_RUNNING = 0, LB_CONVERGED = 1, LB_LSFAIL = 2, LB_MAXITER = 3 };

struct LbParams {
  int hist, max_iter, max_ls, refresh, use_screen, use_lower;
  double c1, c2, gtol;
  double* obj_trace;      // [count * (max_iter + 1)] or NULL
  long long* time_trace;  // [count * (max_iter + 1)] or NULL
};

struct LbState {
  int status, phase, iter, evals, nls, zoom;
  int count, head;            // history ring
  int accept, push, slot, newdir;
  int since_refresh, pad0;
  double f, gtd0, gmax;
  double t, t_prev, f_prev, dp_prev;
  double t_lo, f_lo, dp_lo, t_hi, f_hi, dp_hi;
  double t_acc, t_next;
  double GG, cg;
  double SG[HMAX], YG[HMAX], rho[HMAX];
  double SY[HMAX][HMAX], YY[HMAX][HMAX];
  double cs[HMAX], cy[HMAX];
};

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
  double* part;  // [count][maxb][ndot]
  int maxb;
  int ndot;
};

__device__ __forceinline__ int lb_ndot(int hist) { return 5 + 3 * hist; }

// dot slots: 0 Gt.d, 1 Gt.Gt, 2 Gt.G, 3 d.d, 4 max|Gt| (as a double),
// 5 + 3i: Gt.s_i, 6 + 3i: Gt.y_i, 7 + 3i: d.y_i
__device__ __forceinline__ double block_sum_d(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

__device__ __forceinline__ float block_max_f(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  float s = 0.f;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = fmaxf(s, red[i]);
  return s;
}

// element e of instance k: trial gradient of F (= -grad D)
__device__ __forceinline__ float lb_gt(const LbArgs& A, const InstDev& I, int e) {
  return e < I.ns ? -A.ga[I.row_off + e] : -A.gb[I.col_off + (e - I.ns)];
}

// grid (maxb, count), block LB_BLOCK
__global__ void __launch_bounds__(LB_BLOCK) k_lbfgs_dots(LbArgs A) {
  __shared__ double red_d[LB_BLOCK / 64];
  __shared__ float red_f[LB_BLOCK / 64];
  const int k = blockIdx.y, b = blockIdx.x;
  const InstDev I = A.inst[k];
  const LbState& S = A.st[k];
  if (b == 0 && k == 0 && threadIdx.x == 0) *A.n_active = 0;
  const int n = I.ns + I.nt_pad;
  const long long v0 = A.voff[k];
  double* out = A.part + ((size_t)k * A.maxb + b) * A.ndot;
  const bool live = S.status == LB_RUNNING && S.phase != 0;
  float gt[LB_PER_THREAD], gv[LB_PER_THREAD], dv[LB_PER_THREAD];
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  float gm = 0.f;
#pragma unroll
  for (int q = 0; q < LB_PER_THREAD; ++q) {
    const int e = b * LB_VB + q * LB_BLOCK + threadIdx.x;
    gt[q] = gv[q] = dv[q] = 0.f;
    if (e < n && S.status == LB_RUNNING) {
      gt[q] = lb_gt(A, I, e);
      gv[q] = A.G[v0 + e];
      dv[q] = A.Dv[v0 + e];
    }
    a0 += (double)gt[q] * dv[q];
    a1 += (double)gt[q] * gt[q];
    a2 += (double)gt[q] * gv[q];
    a3 += (double)dv[q] * dv[q];
    gm = fmaxf(gm, fabsf(gt[q]));
  }
  double r;
  r = block_sum_d(a0, red_d); if (threadIdx.x == 0) out[0] = r;
  r = block_sum_d(a1, red_d); if (threadIdx.x == 0) out[1] = r;
  r = block_sum_d(a2, red_d); if (threadIdx.x == 0) out[2] = r;
  r = block_sum_d(a3, red_d); if (threadIdx.x == 0) out[3] = r;
  const float m = block_max_f(gm, red_f);
  if (threadIdx.x == 0) out[4] = (double)m;
  // history dots (only valid ring slots are read)
  for (int i = 0; i < A.P.hist; ++i) {
    double s0 = 0, s1 = 0, s2 = 0;
    const bool valid = live && S.count > 0 && (i < S.count);
    if (valid) {
      const float* Si = A.S + (size_t)i * A.vtot + v0;
      const float* Yi = A.Y + (size_t)i * A.vtot + v0;
#pragma unroll
      for (int q = 0; q < LB_PER_THREAD; ++q) {
        const int e = b * LB_VB + q * LB_BLOCK + threadIdx.x;
        if (e < n) {
          const double sv = Si[e], yv = Yi[e];
          s0 += (double)gt[q] * sv;
          s1 += (double)gt[q] * yv;
          s2 += (double)dv[q] * yv;
        }
      }
    }
    r = block_sum_d(s0, red_d); if (threadIdx.x == 0) out[5 + 3 * i] = r;
    r = block_sum_d(s1, red_d); if (threadIdx.x == 0) out[6 + 3 * i] = r;
    r = block_sum_d(s2, red_d); if (threadIdx.x == 0) out[7 + 3 * i] = r;
  }
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

// Two-loop recursion on coefficients; d = -H G.  Returns d.G.
__device__ double lb_direction(LbState& S, int hist) {
  const int m = S.count;
  double cy[HMAX], cs[HMAX], al[HMAX];
  for (int i = 0; i < hist; ++i) cy[i] = cs[i] = al[i] = 0.0;
  // q = G + sum cy_i y_i
  for (int j = m - 1; j >= 0; --j) {
    const int sj = lb_slot(S, hist, j);
    double sq = S.SG[sj];
    for (int i = 0; i < hist; ++i) sq += cy[i] * S.SY[sj][i];
    al[sj] = S.rho[sj] * sq;
    cy[sj] -= al[sj];
  }
  double cg = 1.0;
  if (m > 0) {
    const int sn = lb_slot(S, hist, m - 1);
    const double g0 = S.SY[sn][sn] / S.YY[sn][sn];
    cg = g0;
    for (int i = 0; i < hist; ++i) cy[i] *= g0;
  }
  for (int j = 0; j < m; ++j) {
    const int sj = lb_slot(S, hist, j);
    double yr = cg * S.YG[sj];
    for (int i = 0; i < hist; ++i) yr += cy[i] * S.YY[sj][i] + cs[i] * S.SY[i][sj];
    const double be = S.rho[sj] * yr;
    cs[sj] += al[sj] - be;
  }
  S.cg = -cg;
  double dG = -cg * S.GG;
  for (int i = 0; i < hist; ++i) {
    S.cs[i] = -cs[i];
    S.cy[i] = -cy[i];
    dG += S.cs[i] * S.SG[i] + S.cy[i] * S.YG[i];
  }
  return dG;
}

__device__ void lb_new_direction(LbState& S, const LbParams& P) {
  double gtd = lb_direction(S, P.hist);
  if (!(gtd < 0.0)) {  // not a descent direction: restart from steepest descent
    S.count = 0;
    S.head = 0;
    for (int i = 0; i < P.hist; ++i) S.cs[i] = S.cy[i] = 0.0;
    S.cg = -1.0;
    gtd = -S.GG;
  }
  S.gtd0 = gtd;
  S.t = (S.count == 0) ? 1.0 / sqrt(S.GG) : 1.0;
  S.t_prev = 0.0;
  S.f_prev = S.f;
  S.dp_prev = gtd;
  S.zoom = 0;
  S.nls = 0;
  S.t_next = S.t;
  S.newdir = 1;
}

// one wavefront per instance
__global__ void __launch_bounds__(64) k_lbfgs_ctrl(LbArgs A) {
  __shared__ double dots[5 + 3 * HMAX];
  const int k = blockIdx.x;
  const InstDev I = A.inst[k];
  LbState& S = A.st[k];
  const int nb = (I.ns + I.nt_pad + LB_VB - 1) / LB_VB;
  for (int j = threadIdx.x; j < A.ndot; j += 64) {
    const double* p = A.part + (size_t)k * A.maxb * A.ndot + j;
    double s = 0.0;
    if (j == 4) {
      for (int b = 0; b < nb; ++b) s = fmax(s, p[(size_t)b * A.ndot]);
    } else {
      for (int b = 0; b < nb; ++b) s += p[(size_t)b * A.ndot];
    }
    dots[j] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const LbParams& P = A.P;
  S.accept = 0;
  S.push = 0;
  S.newdir = 0;
  if (S.status != LB_RUNNING) {
    A.inst_mode[k] = EM_SKIP;
    S.t_next = 0.0;
    return;
  }
  const double D = A.obj[k];
  const double ft = -D;
  const double Gtd = dots[0], GtGt = dots[1], GtG = dots[2], dd = dots[3];
  S.evals++;
  const size_t tr = (size_t)k * (P.max_iter + 1);
  if (!isfinite(D) || !isfinite(GtGt)) {
    S.status = LB_LSFAIL;
    A.inst_mode[k] = EM_SKIP;
    S.t_next = 0.0;
    return;
  }
  if (S.phase == 0) {  // first evaluation, at the starting point
    S.phase = 1;
    S.f = ft;
    S.accept = 1;
    S.t_acc = 0.0;
    S.GG = GtGt;
    S.gmax = dots[4];
    S.count = 0;
    S.head = 0;
    if (P.obj_trace) P.obj_trace[tr] = D;
    if (P.time_trace) P.time_trace[tr] = wall_clock64();
    if (S.gmax <= P.gtol) {
      S.status = LB_CONVERGED;
    } else if (P.max_iter <= 0) {
      S.status = LB_MAXITER;
    }
    if (S.status != LB_RUNNING) {
      A.inst_mode[k] = EM_SKIP;
      S.t_next = 0.0;
      return;
    }
    lb_new_direction(S, P);
    A.inst_mode[k] = P.use_screen ? EM_SCREEN : EM_DENSE;
    atomicAdd(A.n_active, 1);
    return;
  }
  // strong-Wolfe line search on phi(t) = F(X + t d)
  const double t = S.t, dp = Gtd;
  bool ok = false;
  S.nls++;
  if (!S.zoom) {
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
      S.status = LB_LSFAIL;
      A.inst_mode[k] = EM_SKIP;
      S.t_next = 0.0;
      return;
    }
    if (S.zoom) S.t = lb_cubic(S.t_lo, S.f_lo, S.dp_lo, S.t_hi, S.f_hi, S.dp_hi);
    S.t_next = S.t;
    atomicAdd(A.n_active, 1);
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
  double SGn[HMAX], YGn[HMAX];
  for (int i = 0; i < h; ++i) {
    SGn[i] = dots[5 + 3 * i];
    YGn[i] = dots[6 + 3 * i];
  }
  if (sy > 1e-10 * sqrt(ss * yy) && yy > 0.0) {
    const int sl = S.head;
    // pairs that stay: every valid slot except the one being overwritten
    for (int j = 0; j < S.count; ++j) {
      const int i = lb_slot(S, h, j);
      if (i == sl) continue;
      S.SY[sl][i] = t * dots[7 + 3 * i];            // s_new . y_i
      S.SY[i][sl] = dots[5 + 3 * i] - S.SG[i];       // s_i . y_new
      const double yyi = dots[6 + 3 * i] - S.YG[i];  // y_new . y_i
      S.YY[sl][i] = yyi;
      S.YY[i][sl] = yyi;
    }
    S.SY[sl][sl] = sy;
    S.YY[sl][sl] = yy;
    S.rho[sl] = 1.0 / sy;
    SGn[sl] = t * Gtd;
    YGn[sl] = GtGt - GtG;
    S.push = 1;
    S.slot = sl;
    S.head = (S.head + 1) % h;
    if (S.count < h) S.count++;
  }
  for (int i = 0; i < h; ++i) {
    S.SG[i] = SGn[i];
    S.YG[i] = YGn[i];
  }
  S.GG = GtGt;
  S.gmax = dots[4];
  if (P.obj_trace) P.obj_trace[tr + S.iter] = D;
  if (P.time_trace) P.time_trace[tr + S.iter] = wall_clock64();
  if (S.gmax <= P.gtol) S.status = LB_CONVERGED;
  else if (S.iter >= P.max_iter) S.status = LB_MAXITER;
  if (S.status != LB_RUNNING) {
    A.inst_mode[k] = EM_SKIP;
    S.t_next = 0.0;
    return;
  }
  lb_new_direction(S, P);
  int mode = P.use_screen ? EM_SCREEN : EM_DENSE;
  if (P.use_screen && ++S.since_refresh >= P.refresh) {
    S.since_refresh = 0;
    mode = EM_SNAPSHOT;
  }
  A.inst_mode[k] = mode;
  atomicAdd(A.n_active, 1);
}

// grid (vector blocks, count); accept, push, new direction, next trial point
__global__ void __launch_bounds__(256) k_lbfgs_update(LbArgs A) {
  const int k = blockIdx.y;
  const InstDev I = A.inst[k];
  const LbState& S = A.st[k];
  const int n = I.ns + I.nt_pad;
  const long long v0 = A.voff[k];
  const int h = A.P.hist;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    float* tp = e < I.ns ? &A.alpha[I.row_off + e] : &A.beta[I.col_off + (e - I.ns)];
    float x = A.X[v0 + e];
    if (S.accept) {
      const float gt = lb_gt(A, I, e);
      x = *tp;
      if (S.push) {
        A.S[(size_t)S.slot * A.vtot + v0 + e] = (float)S.t_acc * A.Dv[v0 + e];
        A.Y[(size_t)S.slot * A.vtot + v0 + e] = gt - A.G[v0 + e];
      }
      A.X[v0 + e] = x;
      A.G[v0 + e] = gt;
    }
    if (S.newdir) {
      double d = S.cg * (double)A.G[v0 + e];
      for (int j = 0; j < S.count; ++j) {
        const int i = lb_slot(S, h, j);
        d += S.cs[i] * (double)A.S[(size_t)i * A.vtot + v0 + e] +
             S.cy[i] * (double)A.Y[(size_t)i * A.vtot + v0 + e];
      }
      A.Dv[v0 + e] = (float)d;
    }
    *tp = x + (float)S.t_next * A.Dv[v0 + e];
  }
}

// X -> trial arrays (alpha, beta), for the export at the end of a solve
__global__ void __launch_bounds__(256) k_lbfgs_export(LbArgs A) {
  const int k = blockIdx.y;
  const InstDev I = A.inst[k];
  const long long v0 = A.voff[k];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < I.ns + I.nt_pad; e += gridDim.x * blockDim.x) {
    if (e < I.ns) A.alpha[I.row_off + e] = A.X[v0 + e];
    else A.beta[I.col_off + (e - I.ns)] = A.X[v0 + e];
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
    S.since_refresh = 0;
    S.t_next = 0.0;
    S.GG = 0.0;
    for (int i = 0; i < HMAX; ++i) S.SG[i] = S.YG[i] = S.rho[i] = S.cs[i] = S.cy[i] = 0.0;
    for (int i = 0; i < HMAX; ++i)
      for (int j = 0; j < HMAX; ++j) S.SY[i][j] = S.YY[i][j] = 0.0;
    // zero start: the zero snapshot is exact (z~ = 0 since C >= 0); a user
    // start is evaluated densely and taken as the first snapshot
    A.inst_mode[k] = !use_screen ? EM_DENSE : (init_user ? EM_SNAPSHOT : EM_SCREEN);
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    float* tp = e < I.ns ? &A.alpha[I.row_off + e] : &A.beta[I.col_off + (e - I.ns)];
    if (!init_user) *tp = 0.f;
    const bool pad = e >= I.ns && (e - I.ns) >= I.nt;
    if (pad) *tp = 0.f;
    A.X[v0 + e] = *tp;
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

}  // namespace otgs
