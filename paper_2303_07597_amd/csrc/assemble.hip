// The assembly of an evaluation: the fixed-order reductions of the tiles'
// partials into grad_alpha = a - T 1 and grad_beta = b - T^T 1, and the
// float64 partials of the objective of the smooth relaxed dual (Eq. 4)
// whose fixed-order sum is D (formed here when finalising, else by the
// solver's control step).
#include "otgs_internal.h"

namespace otgs {

struct ReduceArgs {
  const InstDev* inst;
  const int* row_grp;
  const int* perm_row;
  const int* perm_col;
  const float* rowpart;
  const float* colsum;
  const float* excess;
  const uint8_t* tile_on;   // NULL: every tile was evaluated (dense)
  const float* a_int;
  const float* b_int;
  const float* a_cal;       // the marginals in the caller's order
  const float* b_cal;
  // the caller's alpha and beta (NULL: none): the objective's a.alpha and
  // b.beta are then summed over caller rows and columns, so that every
  // evaluation of ot_gs_dual_grad forms D in the same order whether its
  // tiles read the caller's arrays or the internal copies
  const float* alpha_cal;
  const float* beta_cal;
  const float* alpha;       // internal order (caller order with caller_order)
  const float* beta;
  float* ga_int;            // internal-order gradients (may be NULL)
  float* gb_int;
  float* ga_out;            // caller-order gradients (may be NULL)
  float* gb_out;
  double* obj;              // [count]
  double* obj_part;         // [count][obj_stride] assembly partials of D
  long long obj_stride;
  int max_ns;               // largest n_src over the instances (grid layout)
  const int* a_uniform;     // per instance flags
  const int* b_uniform;
  int* err;
  unsigned int* done;       // finalize: assembly blocks finished, per instance (reset by the last)
  double* obj_out;          // finalize: caller's copy of D (may be NULL)
  int finalize;             // 1: the last assembly block of an instance forms D
  const int* inst_mode;     // EvalMode per instance
  int* zero_first;          // solver steps: the step's count of live instances, zeroed here (may be NULL)
  // dense evaluations straight from the caller's arrays: alpha and beta are
  // in the caller's order (read through perm_row / perm_col and checked for
  // NaN / Inf here), and block (0, 0) runs the evaluation prologue after
  // the tiles (which read every mode as dense)
  int caller_order;
  Prologue pro;
};

constexpr int ASM_BLOCK = 256;
constexpr int ASM_LPR = 8;                      // lanes per row
constexpr int ASM_ROWS = ASM_BLOCK / ASM_LPR;   // rows per assembly block
constexpr int ASM_U = 16;                      // loads per lane in flight

// Blocks of the assembly kernel per instance: row blocks, then column blocks.
__host__ __device__ inline int asm_row_blocks(int ns) { return (ns + ASM_ROWS - 1) / ASM_ROWS; }
__host__ __device__ inline int asm_col_blocks(int ntp) { return (ntp + ASM_BLOCK - 1) / ASM_BLOCK; }
// The partials of D of an instance: one per row block, then one per column
// block, in that order (their fixed-order sum is D).
__host__ __device__ inline int asm_obj_parts(const InstDev& I) {
  return asm_row_blocks(I.ns) + asm_col_blocks(I.nt_pad);
}
// Column blocks also publish the row blocks' partials when each takes at
// most this many of them.
constexpr int ASM_RPMAX = 32;

// Compensated float32 sums (Knuth's TwoSum): s + c carries the sum of the
// terms added so far with the rounding error of every addition kept in c,
// so a gradient entry a - sum, which cancels to a small number near the
// optimum, is formed as (a - s) - c without the sum's float32 rounding.
struct Csum {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float v) {
    const float t = s + v;
    const float bv = t - s;
    c += (s - (t - bv)) + (v - bv);
    s = t;
  }
  __device__ __forceinline__ void add(const Csum& o) {
    add(o.s);
    c += o.c;
  }
  // x - (s + c)
  __device__ __forceinline__ float from(float x) const { return (x - s) - c; }
};

// Row sum of slot q of a row: jb = q, q + ASM_LPR, ... added in that order.
// Each batch issues all its ASM_U loads before the first add; indices past
// the end are clamped to the last slot (a valid address) and not added.
// With MASK, a tile the screen skipped adds an exact zero (its slot holds
// stale data, discarded by the select).
template <bool MASK>
__device__ __forceinline__ Csum asm_row_sum(const float* rp, int ns, int njb, const uint8_t* on, int q) {
  Csum s;
  for (int j0 = q; j0 < njb; j0 += ASM_U * ASM_LPR) {
    float v[ASM_U];
    uint8_t f[ASM_U];
#pragma unroll
    for (int u = 0; u < ASM_U; ++u) {
      const int jb = min(j0 + u * ASM_LPR, njb - 1);
      v[u] = rp[(size_t)jb * ns];
      if (MASK) f[u] = on[jb];
    }
#pragma unroll
    for (int u = 0; u < ASM_U; ++u)
      if (j0 + u * ASM_LPR < njb) s.add((!MASK || f[u]) ? v[u] : 0.f);
  }
  return s;
}

// Column c over the groups of its instance, in group order: sum of the
// column partials and of excess^2 (float64); batches as in asm_row_sum.
template <bool MASK>
__device__ __forceinline__ void asm_col_sum(const float* cs, const float* ex, int nt_pad, int Le,
                                            const uint8_t* on, int njb, Csum& s, double& e2) {
  s = Csum();
  e2 = 0.0;
  for (int g0 = 0; g0 < Le; g0 += ASM_U) {
    float cv[ASM_U], ev[ASM_U];
    uint8_t f[ASM_U];
#pragma unroll
    for (int u = 0; u < ASM_U; ++u) {
      const int g = min(g0 + u, Le - 1);
      cv[u] = cs[(size_t)g * nt_pad];
      ev[u] = ex[(size_t)g * nt_pad];
      if (MASK) f[u] = on[(size_t)g * njb];
    }
#pragma unroll
    for (int u = 0; u < ASM_U; ++u) {
      if (g0 + u < Le) {
        const bool keep = !MASK || f[u];
        const double e = ev[u];
        s.add(keep ? cv[u] : 0.f);
        e2 += keep ? e * e : 0.0;
      }
    }
  }
}


// Assembly, grid (max row blocks + max column blocks, count):
//  row block b:    grad_alpha_r = a_r - sum_jb rowpart[jb][r] (8 slots per row
//                  take jb = q mod 8 in order, then a fixed pairwise tree; the
//                  sums compensated, see Csum);
//  column block b: grad_beta_c = b_c - sum_l colsum[l][c] in group order (compensated) and
//                  the block's share of b.beta - sum_l excess_lc^2 / (2 gamma).
// D's float64 partials are one per row block (its rows' share of a.alpha)
// and one per column block, and D is their sum in block order.  Only
// evaluated tiles are summed (skipped ones are exact zeros).  Inside a solve
// every block writes its own partial and the control kernel adds them.
// When finalising, the column blocks also form the row blocks' partials
// (column block cb those of row blocks cb, cb + ncb, ...), so that only the
// column blocks publish partials and pay the agent-scope release before
// their count; the last of them to finish adds all partials.  An instance
// with more than ASM_RPMAX row blocks per column block keeps each row
// block's partial in that block, which then takes part in the count.
__global__ void __launch_bounds__(ASM_BLOCK) k_assemble(ReduceArgs A) {
  __shared__ double red[ASM_BLOCK / 64];
  __shared__ double rpart[ASM_RPMAX];
  __shared__ float lds_s[ASM_LPR][ASM_ROWS], lds_c[ASM_LPR][ASM_ROWS];
  const int k = blockIdx.y;
  if (A.zero_first && blockIdx.x == 0 && k == 0 && threadIdx.x == 0) *A.zero_first = 0;
  if (A.caller_order && blockIdx.x == 0 && k == 0) prologue_body(A.pro);
  // inside a batched solve, an instance whose solve has ended (mode SKIP)
  // has no tiles evaluated and nothing reads its gradient or D: its blocks
  // leave at once (calls that finalize D never see SKIP)
  if (!A.finalize && A.inst_mode[k] == EM_SKIP) return;
  const InstDev I = A.inst[k];
  // per-instance blocks and partials, so that an instance's objective does
  // not depend on the other instances of a batch
  const int nbr = asm_row_blocks(I.ns);
  const int nbc = asm_col_blocks(I.nt_pad);
  // (inside a solve nothing is finalised: every block keeps its own partial)
  const bool cols_publish = A.finalize && (nbr + nbc - 1) / nbc <= ASM_RPMAX;
  const int b = blockIdx.x;
  if (b >= nbr + nbc) return;
  const bool a_uni = A.a_uniform[k];
  double part = 0.0;
  if (b < nbr) {
    // thread t takes row t mod 32 and slot q = t / 32, so that one load
    // instruction of a wavefront reads two runs of 32 consecutive partials
    const int r = b * ASM_ROWS + threadIdx.x % ASM_ROWS;
    const int q = threadIdx.x / ASM_ROWS;
    const bool rok = r < I.ns;
    const bool lead = q == 0 && rok;         // slot 0 forms the row's results
    // the row's own operands are loaded together with its partials
    const float a_r = lead ? A.a_int[I.row_off + r] : 0.f;
    const int pm_r = (lead && A.ga_out) ? A.perm_row[I.row_off + r] : 0;
    const bool own = !cols_publish && lead;  // this block forms its share of a.alpha
    const float al_r = own ? (A.alpha_cal ? A.alpha_cal : A.alpha)[I.row_off + r] : 0.f;
    const float am_r = (own && A.alpha_cal) ? A.a_cal[I.row_off + r] : a_r;
    Csum s;
    if (rok) {
      const float* rp = A.rowpart + I.r_off + r;
      if (A.tile_on)
        s = asm_row_sum<true>(rp, I.ns, I.njb, A.tile_on + I.tile_off + (size_t)A.row_grp[I.row_off + r] * I.njb, q);
      else
        s = asm_row_sum<false>(rp, I.ns, I.njb, nullptr, q);
    }
    lds_s[q][threadIdx.x % ASM_ROWS] = s.s;
    lds_c[q][threadIdx.x % ASM_ROWS] = s.c;
    __syncthreads();
    if (threadIdx.x < 64) {
      if (q == 0) {
        // fixed-order combine of the slots of a row: pairs (0,1), (2,3),
        // (4,5), (6,7), then pairs of pairs, each added lower slot first
        Csum p[ASM_LPR];
#pragma unroll
        for (int i = 0; i < ASM_LPR; ++i) {
          p[i].s = lds_s[i][threadIdx.x];
          p[i].c = lds_c[i][threadIdx.x];
        }
#pragma unroll
        for (int o = 1; o < ASM_LPR; o <<= 1)
#pragma unroll
          for (int i = 0; i < ASM_LPR; i += 2 * o) p[i].add(p[i + o]);
        if (rok) {
          const float gval = p[0].from(a_r);
          if (A.ga_int) A.ga_int[I.row_off + r] = gval;
          if (A.ga_out) A.ga_out[I.row_off + pm_r] = gval;
          if (own) {
            if (A.caller_order && !isfinite(al_r)) atomicOr(A.err, 8);
            const double av = a_uni ? 1.0 / (double)I.ns : (double)am_r;
            part = av * (double)al_r;
          }
        }
      }
      if (!cols_publish) {
        // the block's share of a.alpha, added as the column blocks add it
        // for a row block when they publish its partial
        double v = part + 0.0;
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        const double g1 = __shfl_down(v, 8), g2 = __shfl_down(v, 16), g3 = __shfl_down(v, 24);
        part = threadIdx.x == 0 ? (((0.0 + v) + g1) + g2) + g3 : 0.0;
      }
    }
    if (cols_publish) return;
  } else {
    const int cb = b - nbr;
    if (cols_publish) {
      // the partials of the row blocks assigned to this block, 32 threads
      // (one row each) per row block: the same sums in the same order as a
      // row block forms its own (a value plus +0.0, pairs, pairs of pairs
      // and the tree of eight rows, then the four totals added in order).
      // With caller-order duals the share of caller rows (a.alpha is a sum
      // over all rows in any one-to-one order, so no index load precedes
      // the alpha loads).
      const int nrb = (nbr - cb + nbc - 1) / nbc;   // row blocks cb, cb + nbc, ... below nbr
      const float* al = (A.alpha_cal ? A.alpha_cal : A.alpha) + I.row_off;
      const float* am = (A.alpha_cal ? A.a_cal : A.a_int) + I.row_off;
      for (int i0 = 0; i0 < nrb; i0 += ASM_BLOCK / ASM_ROWS) {
        const int i = i0 + (int)threadIdx.x / ASM_ROWS;
        const int r = (cb + i * nbc) * ASM_ROWS + (int)threadIdx.x % ASM_ROWS;
        const bool mine = i < nrb && r < I.ns;
        const float al_r = mine ? al[r] : 0.f;
        const float am_r = mine ? am[r] : 0.f;
        if (mine && A.caller_order && !isfinite(al_r)) atomicOr(A.err, 8);
        double v = mine ? (a_uni ? 1.0 / (double)I.ns : (double)am_r) * (double)al_r : 0.0;
        v = v + 0.0;
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        const double g1 = __shfl_down(v, 8), g2 = __shfl_down(v, 16), g3 = __shfl_down(v, 24);
        if (threadIdx.x % ASM_ROWS == 0 && i < nrb) rpart[i] = (((0.0 + v) + g1) + g2) + g3;
      }
    }
    const int c = cb * ASM_BLOCK + threadIdx.x;
    if (c < I.nt_pad) {
      const bool cok = c < I.nt;
      const float b_c = cok ? A.b_int[I.col_off + c] : 0.f;
      const int pm_c = (cok && A.gb_out) ? A.perm_col[I.col_off + c] : 0;
      // b.beta as a.alpha: caller column c's share with caller-order duals
      const float be_c = cok ? (A.beta_cal ? A.beta_cal[I.scol_off + c] : A.beta[I.col_off + c]) : 0.f;
      const float bm_c = (cok && A.beta_cal) ? A.b_cal[I.scol_off + c] : b_c;
      if (A.caller_order && !isfinite(be_c)) atomicOr(A.err, 8);
      const bool b_uni = A.b_uniform[k];
      const float* cs = A.colsum + (size_t)I.pair_off + c;
      const float* ex = A.excess + (size_t)I.pair_off + c;
      Csum s;
      double e2;
      if (A.tile_on)
        asm_col_sum<true>(cs, ex, I.nt_pad, I.Le, A.tile_on + I.tile_off + c / TJ, I.njb, s, e2);
      else
        asm_col_sum<false>(cs, ex, I.nt_pad, I.Le, nullptr, I.njb, s, e2);
      const float gval = cok ? s.from(b_c) : 0.f;
      if (A.gb_int) A.gb_int[I.col_off + c] = gval;
      if (A.gb_out && cok) A.gb_out[I.scol_off + pm_c] = gval;
      if (cok) {
        const double bv = b_uni ? 1.0 / (double)I.nt : (double)bm_c;
        part = bv * (double)be_c - e2 * (0.5 / I.gamma64);
      }
    }
  }
  // fixed-order block sum
  part = wave_sum_dd(part);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  __shared__ int last;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < ASM_BLOCK / 64; ++w) t += red[w];
    double* op = A.obj_part + (size_t)k * A.obj_stride;
    op[b] = t;
    if (cols_publish)
      for (int i = 0; b - nbr + i * nbc < nbr; ++i) op[b - nbr + i * nbc] = rpart[i];
    last = 0;
    if (A.finalize) {
      // the last publishing block of the instance to finish forms D from the
      // partials (release: this block's partials are visible before its count)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      last = atomicAdd(&A.done[k], 1u) == (unsigned)((cols_publish ? nbc : nbr + nbc) - 1);
    }
  }
  __syncthreads();
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  if (threadIdx.x < 64) {
    const volatile double* parts = A.obj_part + (size_t)k * A.obj_stride;
    double t = 0.0;
    for (int i = threadIdx.x; i < nbr + nbc; i += 64) t += parts[i];
    t = wave_sum_dd(t);
    if (threadIdx.x == 0) {
      if (!isfinite(t)) atomicOr(A.err, 4);
      A.obj[k] = t;
      if (A.obj_out) A.obj_out[k] = t;
      A.done[k] = 0;
    }
  }
}

}  // namespace otgs
