// Setup kernels: group layout of the source rows (stable counting sort by
// label), clustering of the target columns by nearest source class, the cost
// in the internal layout, marginals.  All run once per handle.
#include "otgs_internal.h"

namespace otgs {

// ---------------------------------------------------------------- sorting

// Histogram of integer keys in [0, K) of each segment; one block per segment.
__global__ void k_histogram(const SegDesc* __restrict__ segs, const int* __restrict__ keys,
                            int* __restrict__ counts, int* __restrict__ err) {
  extern __shared__ int h[];
  const SegDesc s = segs[blockIdx.x];
  for (int l = threadIdx.x; l < s.K; l += blockDim.x) h[l] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < s.n; i += blockDim.x) {
    const int key = keys[s.key_off + i];
    if (key < 0 || key >= s.K) {
      atomicOr(err, 1);
      continue;
    }
    atomicAdd(&h[key], 1);
  }
  __syncthreads();
  for (int l = threadIdx.x; l < s.K; l += blockDim.x) counts[s.kt_off + l] = h[l];
}

// Stable scatter: position of element i = start[key] + number of earlier
// elements with the same key.  One wavefront per segment walks the keys in
// order, 64 at a time; lanes holding equal keys are found with ballots over
// the key bits.  out_perm[pos] = i, out_key[pos] = keymap[key].
__global__ void __launch_bounds__(WAVE) k_stable_scatter(
    const SegDesc* __restrict__ segs, const int* __restrict__ keys,
    const int* __restrict__ start, const int* __restrict__ keymap,
    int* __restrict__ out_perm, int* __restrict__ out_key) {
  extern __shared__ int cur[];
  const SegDesc s = segs[blockIdx.x];
  const int lane = threadIdx.x;
  for (int l = lane; l < s.K; l += WAVE) cur[l] = start[s.kt_off + l];
  __syncthreads();
  int nbits = 1;
  while ((1 << nbits) < s.K) ++nbits;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int base = 0; base < s.n; base += WAVE) {
    const int i = base + lane;
    const bool v = i < s.n;
    const int key = v ? keys[s.key_off + i] : 0;
    unsigned long long peers = __ballot(v);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (key >> b) & 1;
      const unsigned long long m = __ballot(v && bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    int pos = 0;
    if (v) {
      pos = cur[key] + rank;
      out_perm[s.out_off + pos] = i;
      if (out_key) out_key[s.out_off + pos] = keymap ? keymap[s.kt_off + key] : key;
    }
    __syncthreads();
    if (v && rank == 0) cur[key] += __popcll(peers);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- cost

// max over a nonnegative float array, per instance (grid.y); flags negative,
// NaN or Inf values.  Result as float bits through an integer atomic max,
// which orders nonnegative floats correctly and is order independent.
__global__ void k_cost_max(const float* const* __restrict__ costs, const long long* __restrict__ sizes,
                           unsigned int* __restrict__ maxbits, int* __restrict__ err) {
  const int k = blockIdx.y;
  const float* c = costs[k];
  const long long n = sizes[k];
  float m = 0.f;
  bool bad = false;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float x = c[i];
    bad |= !(x >= 0.f) || isinf(x);
    m = fmaxf(m, x);
  }
  if (bad) atomicOr(err, 2);
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(&maxbits[k], __float_as_uint(m));
}

// Squared Euclidean cost from features in the caller's order (materialised
// provider): c_ij = sum_k (x_ik - y_jk)^2 in float32, 16x16 threads per 64x64
// block with both feature tiles staged in LDS.  The sum is compensated, so
// the stored value is within about one rounding of the exact cost of the
// float32 features (plain float32 accumulation over d terms errs by up to
// d + 2 roundings): each difference t = x - y is split exactly into
// t + t_lo (TwoSum), each square into t*t + p_lo (fma), and the running sum
// carries its own rounding errors (TwoSum) in a second word, the
// compensated dot product of Ogita, Rump and Oishi (SIAM J. Sci. Comput.,
// 2005).  The cross term 2 t t_lo is added to the second word; t_lo^2 is
// below the final rounding.  One-time setup work; the kernel is not on the
// evaluation path.
__global__ void __launch_bounds__(256) k_cost_features(const float* __restrict__ xs,
                                                       const float* __restrict__ xt, int ns,
                                                       int nt, int d, float* __restrict__ C) {
  constexpr int TB = 64, KB = 32;
  __shared__ float sx[KB][TB + 1];
  __shared__ float sy[KB][TB + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * TB, j0 = blockIdx.x * TB;
  float acc[4][4] = {}, cmp[4][4] = {};
  for (int k0 = 0; k0 < d; k0 += KB) {
    for (int e = threadIdx.x; e < TB * KB; e += 256) {
      const int rr = e / KB, kk = e % KB;
      const int gi = i0 + rr, gj = j0 + rr, gk = k0 + kk;
      sx[kk][rr] = (gi < ns && gk < d) ? xs[(size_t)gi * d + gk] : 0.f;
      sy[kk][rr] = (gj < nt && gk < d) ? xt[(size_t)gj * d + gk] : 0.f;
    }
    __syncthreads();
    const int kmax = min(KB, d - k0);
    for (int kk = 0; kk < kmax; ++kk) {
      float xv[4], yv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = sx[kk][ty + 16 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u) yv[u] = sy[kk][tx + 16 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float x = xv[u], y = yv[v];
          const float t = x - y;                           // TwoSum(x, -y)
          const float tv = t - x;
          const float t_lo = (x - (t - tv)) + (-y - tv);
          const float p = t * t;                           // TwoProduct by fma
          const float p_lo = fmaf(t, t, -p);
          const float s0 = acc[u][v];
          const float s1 = s0 + p;                         // TwoSum(s0, p)
          const float sv = s1 - s0;
          const float e = (s0 - (s1 - sv)) + (p - sv);
          acc[u][v] = s1;
          cmp[u][v] += e + fmaf(2.f * t, t_lo, p_lo);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = i0 + ty + 16 * u, gj = j0 + tx + 16 * v;
      if (gi < ns && gj < nt) C[(size_t)gi * nt + gj] = acc[u][v] + cmp[u][v];
    }
}

// For every target column j (grid.x) of instance k (grid.y): the nonempty
// group holding the source row of least cost (first such group on ties).
__global__ void k_col_assign(const InstDev* __restrict__ inst, const float* const* __restrict__ costs,
                             const int* __restrict__ perm_row, const int* __restrict__ row_grp,
                             int* __restrict__ colkey) {
  const InstDev I = inst[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= I.nt) return;
  const float* c = costs[blockIdx.y];
  float best = INFINITY;
  int bg = 0;
  for (int r = 0; r < I.ns; ++r) {
    const float v = c[(size_t)perm_row[I.row_off + r] * I.nt + j];
    const int g = row_grp[I.row_off + r];
    if (v < best) {
      best = v;
      bg = g;
    }
  }
  colkey[I.scol_off + j] = bg;
}

// Internal cost: C_int(r, c) = fl32(C[perm_row[r]][perm_col[c]] * scale) in the
// tile-major layout, 0 on padding columns.  grid.x: columns / 256, grid.y:
// rows (strided), grid.z: instance.
__global__ void k_relayout_cost(const InstDev* __restrict__ inst, const float* const* __restrict__ costs,
                                const float* __restrict__ scales, const int* __restrict__ perm_row,
                                const int* __restrict__ perm_col, const int* __restrict__ row_grp,
                                const int* __restrict__ g_start, const int* __restrict__ g_size,
                                float* __restrict__ Cint) {
  const InstDev I = inst[blockIdx.z];
  const float s = scales[blockIdx.z];
  for (int r = blockIdx.y; r < I.ns; r += gridDim.y) {
    const int g = row_grp[I.row_off + r];
    const int gs = g_start[I.grp_off + g], gn = g_size[I.grp_off + g];
    const float* src = costs[blockIdx.z] + (size_t)perm_row[I.row_off + r] * I.nt;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < I.nt_pad; c += gridDim.x * blockDim.x) {
      float v = 0.f;
      if (c < I.nt) v = src[perm_col[I.col_off + c]] * s;
      Cint[c_index(I, gs, gn, r, c)] = v;
    }
  }
}

// Marginals in the internal order (float32); uniform ones are 1/n.
__global__ void k_marginals(const InstDev* __restrict__ inst, const float* const* __restrict__ a_src,
                            const float* const* __restrict__ b_src, const int* __restrict__ perm_row,
                            const int* __restrict__ perm_col, float* __restrict__ a_int,
                            float* __restrict__ b_int, float* __restrict__ a_cal, float* __restrict__ b_cal) {
  const InstDev I = inst[blockIdx.y];
  const float* a = a_src[blockIdx.y];
  const float* b = b_src[blockIdx.y];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < I.ns; r += gridDim.x * blockDim.x) {
    a_int[I.row_off + r] = a ? a[perm_row[I.row_off + r]] : 1.0f / (float)I.ns;
    a_cal[I.row_off + r] = a ? a[r] : 1.0f / (float)I.ns;
  }
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < I.nt_pad; c += gridDim.x * blockDim.x) {
    b_int[I.col_off + c] = (c < I.nt) ? (b ? b[perm_col[I.col_off + c]] : 1.0f / (float)I.nt) : 0.f;
    if (c < I.nt) b_cal[I.scol_off + c] = b ? b[c] : 1.0f / (float)I.nt;
  }
}

}  // namespace otgs

namespace otgs {

// ---------------------------------------------------------------- on-the-fly cost
//
// Features are packed for the FP32 matrix-core instruction v_mfma_f32_32x32x2f32
// (A operand: lane l gives row l%32, dim 2m + l/32; B operand: column l%32,
// dim 2m + l/32).  Dimensions are padded with zeros to DP (a multiple of 16)
// and stored per block of 32 rows (or columns) as [DP/16][2][32][8]: for
// chunk m8 (dims 16 m8 .. 16 m8 + 15), lane (c, h) finds its 8 values
// (dims 2 (8 m8 + u) + h, u < 8) contiguously at ((2 m8 + h) 32 + c) 8, so a
// wavefront's operand load is 1 KB of consecutive memory.
__host__ __device__ inline size_t otf_block_index(int DP, int c, int dim) {
  const int m = dim >> 1, h = dim & 1;
  return ((size_t)((m >> 3) * 2 + h) * 32 + c) * 8 + (m & 7);
}

// Source features: internal row r (group ge, local row q) goes to the block
// of rows of its group; groups are padded to whole 32-row blocks.  Also the
// squared norms in float32 (fixed order over dims).  grid (row blocks, count)
__global__ void k_otf_pack_x(const InstDev* __restrict__ inst, const float* const* __restrict__ xs,
                             const int* __restrict__ perm_row, const int* __restrict__ row_grp,
                             const int* __restrict__ g_start, const int* __restrict__ g_xblk,
                             float* __restrict__ Xp, float* __restrict__ xn, int* __restrict__ err) {
  const InstDev I = inst[blockIdx.y];
  const float* x = xs[blockIdx.y];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < I.ns; r += gridDim.x * blockDim.x) {
    const int g = row_grp[I.row_off + r];
    const int q = r - g_start[I.grp_off + g];
    float* blk = Xp + I.x_off + ((size_t)g_xblk[I.grp_off + g] + q / 32) * 32 * I.dp;
    const float* src = x + (size_t)perm_row[I.row_off + r] * I.dim;
    float s = 0.f;
    for (int k = 0; k < I.dp; ++k) {
      const float v = k < I.dim ? src[k] : 0.f;
      if (!isfinite(v)) atomicOr(err, 2);
      s = fmaf(v, v, s);
      blk[otf_block_index(I.dp, q % 32, k)] = v;
    }
    if (!isfinite(s)) atomicOr(err, 2);
    xn[I.row_off + r] = s;
  }
}

// Target features, column c of the internal order (perm_col maps to the
// caller's column; NULL: natural order), block c / 32; padding columns 0.
__global__ void k_otf_pack_y(const InstDev* __restrict__ inst, const float* const* __restrict__ xt,
                             const int* __restrict__ perm_col, float* __restrict__ Yp,
                             float* __restrict__ yn, int* __restrict__ err) {
  const InstDev I = inst[blockIdx.y];
  const float* y = xt[blockIdx.y];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < I.nt_pad; c += gridDim.x * blockDim.x) {
    float* blk = Yp + I.y_off + (size_t)(c / 32) * 32 * I.dp;
    const int src_c = c < I.nt ? (perm_col ? perm_col[I.col_off + c] : c) : -1;
    float s = 0.f;
    for (int k = 0; k < I.dp; ++k) {
      const float v = (src_c >= 0 && k < I.dim) ? y[(size_t)src_c * I.dim + k] : 0.f;
      if (!isfinite(v)) atomicOr(err, 2);
      s = fmaf(v, v, s);
      blk[otf_block_index(I.dp, c % 32, k)] = v;
    }
    if (!isfinite(s)) atomicOr(err, 2);
    yn[I.col_off + c] = s;
  }
}

}  // namespace otgs
