// Learned warm start: per-sample features and a three-layer network
// (Linear - GELU - Linear - GELU - Linear, GELU with the exact normal CDF)
// that maps them to initial dual values, trained with Adam on converged
// duals.  The products run on bf16 matrix cores (v_mfma_f32_32x32x16_bf16):
// operands are rounded to bfloat16 (nearest even) as they are loaded,
// accumulation and everything else is float32; reductions have a fixed order.
#include "otgs_internal.h"

namespace otgs {

typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ short bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite values)
  return (short)(u >> 16);
}

__device__ __forceinline__ float bf16_round(float f) {
  return __uint_as_float(((uint32_t)(unsigned short)bf16_bits(f)) << 16);
}

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---------------------------------------------------------------- products

enum GemmEpi { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD = 2 };

// C = A B with A(i, k) = A[i a_rs + k a_cs], B(k, j) = B[k b_rs + j b_cs],
// C[i ldc + j] (M x N).  Split-K: workgroup z covers k in
// [z kchunk, (z + 1) kchunk) and writes C + z part_stride (EPI_STORE only).
struct GemmArgs {
  int M, N, K, kchunk;
  const float* A;
  long long a_rs, a_cs;
  const float* B;
  long long b_rs, b_cs;
  float* C;
  long long ldc, part_stride;
  const float* bias;   // EPI_BIAS_GELU: bias[j]; C gets GELU(z), Z gets z
  float* Z;
  const float* Zin;    // EPI_GELU_GRAD: C = (A B) GELU'(Zin)
};

// 64 x 64 output tile per workgroup of four wavefronts (32 x 32 each), K
// in stages of GK (32 or 128) through LDS.  Each stage the 256 threads load
// the 64 x GK slices of A and B along whichever index is contiguous in memory
// (so the loads coalesce for plain and transposed operands alike), round
// them to bfloat16 and store them in the matrix-core operand layout (k
// contiguous per row of A and per column of B, rows padded against bank
// conflicts); each wavefront then reads 16-byte fragments and issues one
// v_mfma_f32_32x32x16_bf16 per 16 k.  The next stage's global loads are in
// flight in registers while the current stage multiplies.  The MFMA
// sequence over k is that of a direct 16-step loop (steps past the end of
// the chunk are not issued), so the results do not depend on the staging.
// GK = 128 takes a 256-deep chunk in two stages (few workgroups: the
// split-K weight gradients, 4096-row batches); GK = 32 keeps the registers
// and LDS of a workgroup small, for grids of thousands of workgroups where
// occupancy hides the latency.
template <int EPI, int GK>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  constexpr int GLD = GK + 8;           // padded row length (bf16) of an LDS tile
  constexpr int GU = 64 * GK / 256;     // elements per thread and operand per stage
  constexpr int RS = 256 / GK;          // rows per load instruction along k
  __shared__ short As[64 * GLD];
  __shared__ short Bs[64 * GLD];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int bi = blockIdx.y * 64, bj = blockIdx.x * 64;
  const int i0 = 32 * (w >> 1), j0 = 32 * (w & 1);   // the wavefront's sub-tile in the block
  const int ka = blockIdx.z * g.kchunk, kb = min(ka + g.kchunk, g.K);
  const bool a_krow = g.a_cs == 1;   // A(i, k): k contiguous
  const bool b_kcol = g.b_rs == 1;   // B(k, j): k contiguous
  // element u of this thread in a stage: (row or column, k) of the tile;
  // each load instruction covers min(GK, 64) consecutive k of one or more
  // rows, or 64 consecutive rows of one k, whichever runs along memory
  auto a_at = [&](int u, int& r, int& k) {
    if (a_krow) {
      r = t / GK + RS * u;
      k = t % GK;
    } else {
      r = t & 63;
      k = (t >> 6) + 4 * u;
    }
  };
  auto b_at = [&](int u, int& c, int& k) {
    if (b_kcol) {
      c = t / GK + RS * u;
      k = t % GK;
    } else {
      c = t & 63;
      k = (t >> 6) + 4 * u;
    }
  };
  float ra[GU], rb[GU];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      int r, k;
      a_at(u, r, k);
      const int gr = bi + r, gk = k0 + k;
      ra[u] = (gr < g.M && gk < kb) ? g.A[(long long)gr * g.a_rs + (long long)gk * g.a_cs] : 0.f;
      int c, k2;
      b_at(u, c, k2);
      const int gc = bj + c, gk2 = k0 + k2;
      rb[u] = (gc < g.N && gk2 < kb) ? g.B[(long long)gk2 * g.b_rs + (long long)gc * g.b_cs] : 0.f;
    }
  };
  floatx16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (ka < kb) load(ka);
  for (int k0 = ka; k0 < kb; k0 += GK) {
    // ---- the staged slices into LDS as bfloat16
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      int r, k;
      a_at(u, r, k);
      As[r * GLD + k] = bf16_bits(ra[u]);
      int c, k2;
      b_at(u, c, k2);
      Bs[c * GLD + k2] = bf16_bits(rb[u]);
    }
    __syncthreads();
    // ---- the next stage's loads in flight during this stage's products
    if (k0 + GK < kb) load(k0 + GK);
    // ---- one 16-deep product per 16 k of the chunk (lane: row / column
    // lane & 31, k offset 8 (lane >> 5))
    const int nh = (min(GK, kb - k0) + 15) / 16;
#pragma unroll
    for (int h = 0; h < GK / 16; ++h) {
      if (h < nh) {
        const int ko = 16 * h + 8 * (lane >> 5);
        const shortx8 av = *reinterpret_cast<const shortx8*>(&As[(i0 + (lane & 31)) * GLD + ko]);
        const shortx8 bv = *reinterpret_cast<const shortx8*>(&Bs[(j0 + (lane & 31)) * GLD + ko]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                      __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int c = bj + j0 + (lane & 31);
  const bool cok = c < g.N;
  float* C = g.C + (EPI == EPI_STORE ? (long long)blockIdx.z * g.part_stride : 0);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int row = bi + i0 + 8 * (q / 4) + 4 * (lane >> 5) + (q % 4);
    if (row >= g.M || !cok) continue;
    const long long e = (long long)row * g.ldc + c;
    if (EPI == EPI_STORE) {
      C[e] = acc[q];
    } else if (EPI == EPI_BIAS_GELU) {
      const float z = acc[q] + g.bias[c];
      g.Z[e] = z;
      C[e] = gelu_f(z);
    } else {
      C[e] = acc[q] * gelu_grad_f(g.Zin[e]);
    }
  }
}

// out[e] = sum_z parts[z stride + e], z ascending
__global__ void k_sum_parts(const float* __restrict__ parts, int nparts, long long stride, long long n,
                            float* __restrict__ out) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < nparts; ++z) s += parts[z * stride + e];
    out[e] = s;
  }
}

// The same sums for few elements and many partials (the column sums of a
// layer): 16 threads per element each add the partials z = j, j + 16, ...
// in order, then the element's first thread adds the 16 sums in order.
__global__ void __launch_bounds__(1024) k_sum_parts_wide(const float* __restrict__ parts, int nparts,
                                                         long long stride, long long n, float* __restrict__ out) {
  __shared__ float sm[16][64];
  const int c = threadIdx.x & 63, j = threadIdx.x >> 6;
  const long long e = (long long)blockIdx.x * 64 + c;
  float s = 0.f;
  if (e < n)
    for (int z = j; z < nparts; z += 16) s += parts[(long long)z * stride + e];
  sm[j][c] = s;
  __syncthreads();
  if (j == 0 && e < n) {
    float t = 0.f;
    for (int q = 0; q < 16; ++q) t += sm[q][c];
    out[e] = t;
  }
}

// ---------------------------------------------------------------- head and loss

// out_i = sum_k r(H2[i, k]) r(w3[k]) + b3, one wavefront per row (each lane a
// fixed set of k, then a fixed butterfly).  With a target y: e_i = out_i - y_i,
// dout_i = 2 e_i / n_total, and per-workgroup float64 partials of sum e^2.
__global__ void __launch_bounds__(256) k_mlp_head(const float* __restrict__ H2, const float* __restrict__ w3,
                                                  const float* __restrict__ b3, int n, int w,
                                                  float* __restrict__ out, const float* __restrict__ y,
                                                  float inv_total, float* __restrict__ dout,
                                                  double* __restrict__ loss_part) {
  __shared__ double sl[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + wv;
  double e2 = 0.0;
  if (i < n) {
    float s = 0.f;
    for (int k = lane; k < w; k += 64) s = fmaf(bf16_round(H2[(long long)i * w + k]), bf16_round(w3[k]), s);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    const float o_ = s + b3[0];
    if (lane == 0) {
      out[i] = o_;
      if (y) {
        const float e = o_ - y[i];
        dout[i] = 2.f * e * inv_total;
        e2 = (double)e * (double)e;
      }
    }
  }
  if (lane == 0) sl[wv] = e2;
  __syncthreads();
  if (threadIdx.x == 0 && loss_part) loss_part[blockIdx.x] = ((sl[0] + sl[1]) + sl[2]) + sl[3];
}

// dZ2[i, k] = dout_i r(w3[k]) GELU'(Z2[i, k])
__global__ void k_mlp_dz2(const float* __restrict__ dout, const float* __restrict__ w3,
                          const float* __restrict__ Z2, int n, int w, float* __restrict__ dZ2) {
  const long long tot = (long long)n * w;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / w), k = (int)(e % w);
    dZ2[e] = dout[i] * bf16_round(w3[k]) * gelu_grad_f(Z2[e]);
  }
}

// Column sums over rows [z rows_per, (z + 1) rows_per) of A [n x w] (row
// weights `wt` if given, operands then rounded to bf16 as in the product
// they stand for), one partial per z; rows ascending.
__global__ void k_colsum_parts(const float* __restrict__ A, const float* __restrict__ wt, int n, int w,
                               int rows_per, float* __restrict__ parts) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= w) return;
  const int r0 = blockIdx.y * rows_per, r1 = min(n, r0 + rows_per);
  float s = 0.f;
  if (wt) {
    for (int i = r0; i < r1; ++i) s = fmaf(bf16_round(A[(long long)i * w + k]), wt[i], s);
  } else {
    for (int i = r0; i < r1; ++i) s += A[(long long)i * w + k];
  }
  parts[(long long)blockIdx.y * w + k] = s;
}

// sum of n floats (fixed order) into out[0]; one workgroup
__global__ void k_sum_vec(const float* __restrict__ v, int n, float* __restrict__ out) {
  __shared__ float sm[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += v[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

// sum of n doubles (fixed order) into out[slot], scaled
__global__ void k_sum_loss(const double* __restrict__ v, int n, double scale, double* __restrict__ out) {
  __shared__ double sm[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += v[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0] * scale;
}

// Adam with bias-corrected moments; c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
  }
}

// ---------------------------------------------------------------- features

struct FeatDesc {
  int n, m, L, pad;
  const float* xs;
  const float* xt;
  const int* labels;
  long long src_row, tgt_row;   // first feature row of the instance's sources / targets
  long long cent_off;           // [L][d] centroid block of the instance
  long long cls_off;            // first class slot of the instance in the count arrays
  float scale, lg, lm, pad2;    // cost scale, log gamma, log mu
};

// source class centroids: grid (class, instance), thread = dimension
__global__ void k_ws_src_centroid(const FeatDesc* __restrict__ fd, int d, float* __restrict__ cs,
                                  int* __restrict__ ccount) {
  const FeatDesc D = fd[blockIdx.y];
  const int l = blockIdx.x;
  if (l >= D.L) return;
  int cnt = 0;
  for (int dim = threadIdx.x; dim < d; dim += blockDim.x) {
    float s = 0.f;
    cnt = 0;
    for (int i = 0; i < D.n; ++i)
      if (D.labels[i] == l) {
        s += D.xs[(long long)i * d + dim];
        ++cnt;
      }
    cs[D.cent_off + (long long)l * d + dim] = cnt ? s / (float)cnt : 0.f;
  }
  if (threadIdx.x == 0) {
    int c2 = 0;
    for (int i = 0; i < D.n; ++i) c2 += D.labels[i] == l;
    ccount[D.cls_off + l] = c2;
  }
}

// nearest source centroid of every target (ties: smallest class)
__global__ void k_ws_tgt_assign(const FeatDesc* __restrict__ fd, int d, const float* __restrict__ cs,
                                const int* __restrict__ ccount, int* __restrict__ pseudo,
                                float* __restrict__ dmin) {
  const FeatDesc D = fd[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D.m) return;
  float best = INFINITY;
  int bl = 0;
  for (int l = 0; l < D.L; ++l) {
    if (ccount[D.cls_off + l] == 0) continue;
    float s = 0.f;
    for (int k = 0; k < d; ++k) {
      const float t = D.xt[(long long)j * d + k] - cs[D.cent_off + (long long)l * d + k];
      s = fmaf(t, t, s);
    }
    if (s < best) {
      best = s;
      bl = l;
    }
  }
  pseudo[D.tgt_row + j] = bl;
  dmin[D.tgt_row + j] = best;
}

// target pseudo-class centroids: grid (class, instance), thread = dimension
__global__ void k_ws_tgt_centroid(const FeatDesc* __restrict__ fd, int d, const int* __restrict__ pseudo,
                                  float* __restrict__ ct, int* __restrict__ tcount) {
  const FeatDesc D = fd[blockIdx.y];
  const int l = blockIdx.x;
  if (l >= D.L) return;
  for (int dim = threadIdx.x; dim < d; dim += blockDim.x) {
    float s = 0.f;
    int cnt = 0;
    for (int j = 0; j < D.m; ++j)
      if (pseudo[D.tgt_row + j] == l) {
        s += D.xt[(long long)j * d + dim];
        ++cnt;
      }
    ct[D.cent_off + (long long)l * d + dim] = cnt ? s / (float)cnt : 0.f;
  }
  if (threadIdx.x == 0) {
    int c2 = 0;
    for (int j = 0; j < D.m; ++j) c2 += pseudo[D.tgt_row + j] == l;
    tcount[D.cls_off + l] = c2;
  }
}

// one feature row per sample; row layout [x sqrt(s) (d), own, other, frac,
// side, log gamma, log mu, log n, log m]
__global__ void k_ws_features(const FeatDesc* __restrict__ fd, int d, const float* __restrict__ cs,
                              const int* __restrict__ ccount, const float* __restrict__ ct,
                              const int* __restrict__ tcount, const int* __restrict__ pseudo,
                              const float* __restrict__ dmin, float* __restrict__ F) {
  const FeatDesc D = fd[blockIdx.y];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= D.n + D.m) return;
  const int din = d + 8;
  const float rs = sqrtf(D.scale);
  const bool src = q < D.n;
  const int i = src ? q : q - D.n;
  const float* x = src ? D.xs + (long long)i * d : D.xt + (long long)i * d;
  float* row = F + (long long)(src ? D.src_row + i : D.tgt_row + i) * din;
  const int l = src ? D.labels[i] : pseudo[D.tgt_row + i];
  const float* own_c = (src ? cs : ct) + D.cent_off + (long long)l * d;
  float own = 0.f;
  for (int k = 0; k < d; ++k) {
    const float t = x[k] - own_c[k];
    own = fmaf(t, t, own);
    row[k] = x[k] * rs;
  }
  float other;
  if (src) {
    other = INFINITY;
    for (int t = 0; t < D.L; ++t) {
      if (tcount[D.cls_off + t] == 0) continue;
      float s = 0.f;
      for (int k = 0; k < d; ++k) {
        const float u = x[k] - ct[D.cent_off + (long long)t * d + k];
        s = fmaf(u, u, s);
      }
      other = fminf(other, s);
    }
  } else {
    other = dmin[D.tgt_row + i];
  }
  const int cnt = src ? ccount[D.cls_off + l] : tcount[D.cls_off + l];
  row[d + 0] = own * D.scale;
  row[d + 1] = other * D.scale;
  row[d + 2] = (float)cnt / (float)(src ? D.n : D.m);
  row[d + 3] = src ? 0.f : 1.f;
  row[d + 4] = D.lg;
  row[d + 5] = D.lm;
  row[d + 6] = logf((float)D.n);
  row[d + 7] = logf((float)D.m);
}

}  // namespace otgs
