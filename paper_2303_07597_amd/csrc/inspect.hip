// Device helpers of the inspection and verification entry points: the
// screening state (snapshot and set N of Algorithm 1) exported in the
// caller's layout, and the bitwise comparison of a screened evaluation with
// a dense one at the same point (Lemma 2: every skipped block is zero, so
// the two must agree exactly).
#include "otgs_internal.h"

namespace otgs {

template <class T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ p, long long n, T v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// Snapshot point and per-pair snapshot state of instance blockIdx.y in the
// caller's layout: alpha~ [n_src] and beta~ [n_tgt] in the caller's order;
// z~, o~ and the N flag (1 in N, else 0) as [n_groups x n_tgt] row-major
// (row = label, column = the caller's target index) at lab_pair_off[k].
// Pairs of empty labels are not written (the caller's arrays are cleared
// first).  Any output may be NULL.
__global__ void __launch_bounds__(256) k_export_screen(
    const InstDev* __restrict__ inst, const int* __restrict__ perm_row, const int* __restrict__ perm_col,
    const int* __restrict__ g_label, const long long* __restrict__ lab_pair_off, const float* __restrict__ alpha_s,
    const float* __restrict__ beta_s, const float* __restrict__ zsnap, const float* __restrict__ osnap,
    const uint8_t* __restrict__ inN, float* __restrict__ a_out, float* __restrict__ b_out,
    float* __restrict__ z_out, float* __restrict__ o_out, uint8_t* __restrict__ n_out) {
  const int k = blockIdx.y;
  const InstDev I = inst[k];
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  if (a_out)
    for (long long r = t0; r < I.ns; r += st) a_out[I.row_off + perm_row[I.row_off + r]] = alpha_s[I.row_off + r];
  if (b_out)
    for (long long c = t0; c < I.nt; c += st) b_out[I.scol_off + perm_col[I.col_off + c]] = beta_s[I.col_off + c];
  const long long np = (long long)I.Le * I.nt;
  for (long long q = t0; q < np; q += st) {
    const int ge = (int)(q / I.nt), c = (int)(q % I.nt);
    const size_t src = (size_t)I.pair_off + (size_t)ge * I.nt_pad + c;
    const size_t dst = (size_t)lab_pair_off[k] + (size_t)g_label[I.grp_off + ge] * I.nt + perm_col[I.col_off + c];
    if (z_out) z_out[dst] = zsnap[src];
    if (o_out) o_out[dst] = osnap[src];
    if (n_out) n_out[dst] = inN[src] == PAIR_IN_N ? 1 : 0;
  }
}

// Counts the entries of instance blockIdx.y where two evaluations differ in
// any bit: gradients of the rows and of the (unpadded) columns, and either
// the per-instance objective (obj_n == 1) or its assembly partials.  caller:
// the gradients are in the caller's order (column offset scol_off), else in
// the internal one (col_off).  modes (may be NULL): instances whose mode is
// EM_SKIP were not evaluated and are not compared.
__global__ void __launch_bounds__(256) k_bits_differ(const InstDev* __restrict__ inst, const int* __restrict__ modes,
                                                     int caller, const float* __restrict__ ga1,
                                                     const float* __restrict__ ga2, const float* __restrict__ gb1,
                                                     const float* __restrict__ gb2, const double* __restrict__ o1,
                                                     const double* __restrict__ o2, long long obj_n,
                                                     unsigned long long* __restrict__ count) {
  const int k = blockIdx.y;
  if (modes && modes[k] == EM_SKIP) return;
  const InstDev I = inst[k];
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  unsigned n = 0;
  for (long long r = t0; r < I.ns; r += st)
    n += __float_as_uint(ga1[I.row_off + r]) != __float_as_uint(ga2[I.row_off + r]);
  const long long c0 = caller ? I.scol_off : I.col_off;
  for (long long c = t0; c < I.nt; c += st)
    n += __float_as_uint(gb1[c0 + c]) != __float_as_uint(gb2[c0 + c]);
  for (long long q = t0; q < obj_n; q += st)
    n += __double_as_longlong(o1[k * obj_n + q]) != __double_as_longlong(o2[k * obj_n + q]);
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
  if ((threadIdx.x & 63) == 0 && n) atomicAdd(count, (unsigned long long)n);
}

// Verification inside a solve: save every instance's evaluation mode and
// make the live ones DENSE (restore = 0), or put the saved modes back
// (restore = 1).
__global__ void k_verify_modes(int* __restrict__ inst_mode, int* __restrict__ saved, int count, int restore) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) {
    if (restore) {
      inst_mode[k] = saved[k];
    } else {
      const int m = inst_mode[k];
      saved[k] = m;
      inst_mode[k] = m == EM_SKIP ? EM_SKIP : EM_DENSE;
    }
  }
}

}  // namespace otgs
