// Barycentric mapping of the source samples onto the targets with the plan
// (Sec. 2.1: the source matrix is moved to the target side as n T^T X_S):
// y_j = (1 / b_j) sum_i T_ij x_i, which is n_tgt T^T X_S for uniform b, with
// T_ij = kappa_lj [alpha_i + beta_j - c_ij]_+ the plan of Sec. 2.3.  At a
// solution the columns of T sum to b_j, so y_j is a convex combination of
// source samples.
#include "otgs_internal.h"

namespace otgs {

constexpr int MAP_ROWS = 64;      // source rows per round
constexpr int MAP_DMAX = 256;     // feature dimensions

// One workgroup per (32-target column block, instance): for every group in
// order and its rows in order, 64 rows at a time, the entries of T of the
// block go to LDS (each thread 8 of them, computed as the plan computes
// them) together with the rows' features, then thread (column c, dimension
// slice s) adds T_ic x_i over the rows into its dimensions s, s + 8, ...
// Groups with no active block in the column block are passed over.  The
// order of every sum is fixed, so the result is deterministic.
__global__ void __launch_bounds__(256) k_transport(const InstDev* __restrict__ inst, const int* __restrict__ perm_row,
                                                   const int* __restrict__ perm_col, const int* __restrict__ g_start,
                                                   const int* __restrict__ g_size, const float* __restrict__ C,
                                                   const float* __restrict__ alpha, const float* __restrict__ beta,
                                                   const float* __restrict__ kappa, const float* __restrict__ b_int,
                                                   const int* __restrict__ b_uniform, const float* __restrict__ xs,
                                                   int dim, float* __restrict__ y) {
  __shared__ float Tt[MAP_ROWS][TJ];
  __shared__ float Xs[MAP_ROWS][MAP_DMAX];
  const int k = blockIdx.y, jb = blockIdx.x;
  const InstDev I = inst[k];
  if (jb >= I.njb) return;
  const int t = threadIdx.x;
  const int c = t & (TJ - 1), sl = t >> 5;    // column of the block, dimension slice 0..7
  const int col = jb * TJ + c;
  const bool cok = col < I.nt;
  const float bj = cok ? beta[I.col_off + col] : 0.f;
  constexpr int DS = MAP_DMAX / 8;
  float acc[DS];
#pragma unroll
  for (int m = 0; m < DS; ++m) acc[m] = 0.f;
  for (int ge = 0; ge < I.Le; ++ge) {
    const float kap = cok ? kappa[(size_t)I.pair_off + (size_t)ge * I.nt_pad + col] : 0.f;
    if (!__syncthreads_or(kap > 0.f)) continue;
    const int gs = g_start[I.grp_off + ge], gn = g_size[I.grp_off + ge];
    for (int r0 = 0; r0 < gn; r0 += MAP_ROWS) {
      // entries of T: thread t has rows t/32 + 8 m of the round, column c
#pragma unroll
      for (int m = 0; m < MAP_ROWS / 8; ++m) {
        const int rr = sl + 8 * m, r = r0 + rr;
        float v = 0.f;
        if (r < gn && cok && kap > 0.f) {
          const float f = (alpha[I.row_off + gs + r] + bj) - C[c_index(I, gs, gn, gs + r, col)];
          v = kap * fmaxf(f, 0.f);
        }
        Tt[rr][c] = v;
      }
      for (int e = t; e < MAP_ROWS * dim; e += blockDim.x) {
        const int rr = e / dim, q = e - rr * dim, r = r0 + rr;
        Xs[rr][q] = r < gn ? xs[((size_t)I.row_off + perm_row[I.row_off + gs + r]) * dim + q] : 0.f;
      }
      __syncthreads();
      const int nr = min(MAP_ROWS, gn - r0);
      for (int rr = 0; rr < nr; ++rr) {
        const float w = Tt[rr][c];
        if (w != 0.f) {
#pragma unroll
          for (int m = 0; m < DS; ++m) {
            const int q = sl + 8 * m;
            if (q < dim) acc[m] = fmaf(w, Xs[rr][q], acc[m]);
          }
        }
      }
      __syncthreads();
    }
  }
  if (!cok) return;
  const double bb = b_uniform[k] ? 1.0 / I.nt : (double)b_int[I.col_off + col];
  const float inv = bb > 0.0 ? (float)(1.0 / bb) : 0.f;
  float* yo = y + ((size_t)I.scol_off + perm_col[I.col_off + col]) * dim;
#pragma unroll
  for (int m = 0; m < DS; ++m) {
    const int q = sl + 8 * m;
    if (q < dim) yo[q] = acc[m] * inv;
  }
}

}  // namespace otgs

using namespace otgs;

extern "C" int ot_gs_transport(ot_gs_handle* h, const float* alpha, const float* beta, const float* x_src,
                               int dim, float* y_out, void* stream) {
  if (!h || !alpha || !beta || !x_src || !y_out) return fail(OT_GS_EINVAL, "transport: NULL argument");
  if (dim < 1 || dim > MAP_DMAX) return fail(OT_GS_EINVAL, "transport: dim must lie in [1, %d]", MAP_DMAX);
  if (h->onthefly)
    return fail(OT_GS_EINVAL, "transport: needs a materialised cost (for the on-the-fly cost use ot_gs_plan_csr)");
  hipStream_t s = (hipStream_t)stream;
  TRY(gather(h, alpha, beta, s));
  TRY(evaluate(h, OT_GS_DENSE, nullptr, nullptr, s, true));
  int maxjb = 1;
  for (int k = 0; k < h->count; ++k) maxjb = std::max(maxjb, h->inst[k].d.njb);
  hipLaunchKernelGGL(k_transport, dim3(maxjb, h->count), dim3(256), 0, s, h->d_inst, (const int*)h->perm_row,
                     (const int*)h->perm_col, (const int*)h->g_start, (const int*)h->g_size, (const float*)h->C,
                     (const float*)h->alpha, (const float*)h->beta, (const float*)h->kappa,
                     (const float*)h->b_int, (const int*)h->b_uniform, x_src, dim, y_out);
  LAUNCHCHK();
  return OT_GS_OK;
}
