// The hot path: fused dual-gradient tiles of the smooth relaxed dual (Eq. 4):
// per tile the row partials of T 1, the column sums of T and the per-pair
// group statistics (assemble.hip reduces them into the gradients and D).
//
// Gradient tile (group l, TJ = 32 target columns j): lane 32 h + c takes
// column c and the rows of parity h, streams the tile's cost (one
// contiguous [rows x 32] block of the tile-major pool), forms
// f = (alpha_i + beta_j) - c_ij and p = max(f, 0) in registers, accumulates
// z^2 = sum p^2 and s1 = sum p; the two parities and the 16 wavefronts
// combine their partial sums through LDS in a fixed order; then
//     kappa = (z - mu gamma) / (gamma z)   if z > mu gamma, else 0
// is the group soft threshold of Eq. 5 (T_ij = kappa p_ij), the column sum of
// the block is kappa s1, the block's share of psi is (z - mu gamma)^2/(2 gamma)
// and the row sums sum_j kappa_j p_ij are wavefront reductions over lanes.
// Whole groups of up to WHOLE_MAX = 2048 rows keep p in registers (R loads
// per lane, row buckets R = 2, 4, 8, ..., 64; small groups run as teams of
// 2, 4 or 8 wavefronts per tile); larger groups are cut in CHUNK = 1024-row
// chunks: one pass writes per-chunk column sums, a combine step forms kappa,
// a second pass re-reads the chunk and forms the row sums.
// Every reduction has a fixed order and there are no floating-point atomics,
// so a tile gives bit-identical results whichever mode requested it; skipped
// tiles contribute exact zeros, hence screened == dense bit for bit.
#include "otgs_internal.h"

namespace otgs {

struct GradArgs {
  const InstDev* inst;
  const int* g_start;
  const int* g_size;
  const int* g_chunk0;    // first chunk row of a split group (-1: not split)
  const int* g_xblk;      // on-the-fly: first packed 32-row feature block of a group
  const float* Xp;        // on-the-fly: packed source / target features, norms
  const float* Yp;
  const float* xn;
  const float* yn;
  const TileDesc* list;   // work list
  const int* count;       // number of entries (device)
  const float* C;
  const float* alpha;     // internal order
  const float* beta;      // internal order, padded
  float* rowpart;
  float* colsum;
  float* excess;          // [z - mu gamma]_+ per pair (objective: excess^2/(2 gamma))
  float* zsnap;           // snapshot outputs (snapshot != 0)
  float* osnap;
  float* part;            // split chunks: [3][chunk pair] column partial sums
  long long part_stride;  // elements per partial kind
  float* kappa;           // split groups: kappa per pair
  const int* inst_mode;   // EM_SNAPSHOT: also record z~ and o~
  int write_kappa;        // also store kappa per pair (plan recovery)
  int single_inst;        // one instance: a kernel of the other snapshot mode has no work
  const TileRec* rec;     // whole-group materialized tiles: records of the list's entries
  int n_static;           // entries of a static list (-1: read the device count)
  // caller-order duals (dense evaluations straight from the caller's
  // arrays): alpha / beta index of internal row / column i is row_map[i] /
  // col_map[i]; NULL: alpha and beta are in the internal order
  const int* row_map;
  const int* col_map;
};

__device__ __forceinline__ float tile_alpha(const GradArgs& A, int i) {
  return A.alpha[A.row_map ? A.row_map[i] : i];
}
__device__ __forceinline__ float tile_beta(const GradArgs& A, int c) {
  return A.beta[A.col_map ? A.col_map[c] : c];
}

// Does a tile kernel of snapshot kind `snap` take a tile of an instance in
// mode m?  Instances whose solve has ended (EM_SKIP) are never evaluated.
__device__ __forceinline__ bool mode_takes(int m, bool snap) {
  return m != EM_SKIP && (m == EM_SNAPSHOT) == snap;
}


// Sum over the 16 lanes of each lane row (DPP row shifts); lane 15 of every
// row ends with the row's total.  Fixed order: deterministic.
__device__ __forceinline__ float row16_sum(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x112, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x118, 0xf, 0xf, false));
  return x;
}

// Row sums of a register tile: v[k] holds row k's value in every lane; the
// sum over the 64 lanes of each row is formed with a transposed butterfly:
// a permlane32 swap pairs row i with row i + RP/2 (lower lanes keep row i,
// upper lanes row i + RP/2), a permlane16 swap pairs rows i and i + RP/4 the
// same way, and DPP row shifts finish within 16 lanes.  Afterwards lane
// 16 q + 15 holds the total of row i + q RP/4 in x[i].
template <int RP>
__device__ __forceinline__ void transposed_row_sums(float (&v)[RP], float (&x)[RP / 4]) {
  constexpr int H = RP / 2, Q = RP / 4;
  float w[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + H]),
                                                    false, false);
    w[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w[i]), __float_as_uint(w[i + Q]),
                                                    false, false);
    x[i] = row16_sum(__uint_as_float(r[0]) + __uint_as_float(r[1]));
  }
}

// PHASE 0: whole group; 1: split chunk, column partials; 2: split chunk, rows.
// Lane layout: lane = 32 h + c, c the column of the tile (TJ = 32), h the row
// parity.  Load k of wavefront w covers the two tile rows 2 (w + NW k) + h:
// 64 consecutive floats of the tile-major pool.  R loads per lane cover
// 2 NW R >= rows of the tile.  SNAP: also form o~ = ||[f]_-||.
//
// A tile is processed in two steps: tile_loads issues the loads of alpha,
// beta and the R cost values of every lane, tile_body forms p, the sums,
// kappa and the row sums once they have arrived.  Kernels either run the two
// back to back or issue the next tile's loads before the current body.

// Geometry of a tile: every index its loads and its body need (wavefront
// uniform).  Whole-group tiles take it from their precomputed record,
// split-group chunks from the descriptor, the instance and the group tables.
struct TileGeo {
  long long c0;     // cost pool index of the tile stream's first entry
  long long rp0;    // row-partial index of the group's first row, this column block
  long long pr0;    // pair index of the block's first column
  long long part0;  // split chunk (PHASE 1): partial index of the block's first column
  int a0;           // alpha index of the group's first row
  int b0;           // beta index of the block's first column
  int r0, r1;       // rows of the tile, relative to the group start
  int ncol;         // valid columns of the block
  float thr, gamma;
};

__device__ __forceinline__ TileGeo geo_rec(const TileRec& r) {
  TileGeo g;
  g.c0 = r.c0;
  g.rp0 = r.rp0;
  g.pr0 = r.pr0;
  g.part0 = 0;
  g.a0 = r.a0;
  g.b0 = r.b0;
  g.r0 = 0;
  g.r1 = r.gn;
  g.ncol = r.ncol;
  g.thr = r.thr;
  g.gamma = r.gamma;
  return g;
}

template <int PHASE>
__device__ __forceinline__ TileGeo geo_desc(const GradArgs& A, const TileDesc& d) {
  const InstDev I = A.inst[d.inst];
  const int gi = I.grp_off + d.grp;
  const int gs = A.g_start[gi], gn = A.g_size[gi];
  TileGeo g;
  g.c0 = (long long)c_index(I, gs, gn, gs, d.jb * TJ);
  g.rp0 = I.r_off + (long long)d.jb * I.ns + gs;
  g.pr0 = (long long)I.pair_off + (long long)d.grp * I.nt_pad + d.jb * TJ;
  g.part0 = PHASE == 1 ? I.chunk_off + (long long)(A.g_chunk0[gi] + d.aux) * I.nt_pad + d.jb * TJ : 0;
  g.a0 = I.row_off + gs;
  g.b0 = I.col_off + d.jb * TJ;
  g.r0 = PHASE != 0 ? d.aux * CHUNK : 0;
  g.r1 = PHASE != 0 ? min(g.r0 + CHUNK, gn) : gn;
  g.ncol = min(TJ, I.nt - d.jb * TJ);
  g.thr = I.thr;
  g.gamma = I.gamma;
  return g;
}

// Issue the loads of a tile.  A wavefront plays K of the NW "virtual"
// wavefronts of the canonical layout (K = 1: itself): team t of NW / K real
// wavefronts takes one tile, real wavefront v of the team plays the virtual
// wavefronts v + (NW / K) j, j < K.  Virtual wavefront w' reads at load k the
// two tile rows 2 (w' + NW k) + h, so every tile is summed exactly as by NW
// wavefronts (same partials, same order, same bits) whatever K is.
// Alpha of virtual wavefront j, load k, parity h sits in slot s = 2 R j + 2 k + h,
// lane s mod 64 of register s / 64 (-inf past the tile: f = -inf, p = 0
// without a mask); beta of the lane's
// column; the R K cost values by raw buffer loads (loads past the tile
// re-read the last valid row pair, a cache hit).  An inactive team (no tile
// this round) loads nothing.
template <int R, int K>
__device__ __forceinline__ void tile_loads(const GradArgs& A, const TileGeo& g, bool act,
                                           float (&av)[av_regs(R, K)], float& bj, float (&p)[K][R]) {
  static_assert(K == 1 || 2 * R * K <= WAVE, "teams keep their alpha values in one register");
  constexpr int NA = av_regs(R, K);
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int WT = NW / K;
  const int v = w % WT;
  if (!act) {
#pragma unroll
    for (int a = 0; a < NA; ++a) av[a] = -INFINITY;
    bj = -INFINITY;
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
      for (int k = 0; k < R; ++k) p[j][k] = 0.f;
    return;
  }
  // alpha / beta indices first (with caller-order maps these are loads, and
  // the alpha / beta loads wait for them), then every cost load, then the
  // alpha / beta loads: the map round trip overlaps the cost stream
  int ia[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    // (K = 1: slots past 2 R hold -inf; j stays wavefront-uniform)
    const int sl = a * WAVE + lane;
    const int j = K == 1 ? 0 : sl / (2 * R), k = K == 1 ? (sl >> 1) : (sl >> 1) % R;
    const int rwj = g.r0 + 2 * (v + WT * j);
    const int nkj = rwj < g.r1 ? min(R, (g.r1 - rwj + 2 * NW - 1) / (2 * NW)) : 0;
    const int arow = rwj + 2 * NW * k + (lane & 1);
    const bool ok = sl < 2 * R * K && k < nkj && arow < g.r1;
    ia[a] = !ok ? -1 : (A.row_map ? A.row_map[g.a0 + arow] : g.a0 + arow);
  }
  const int ib = A.col_map ? A.col_map[g.b0 + (lane & (TJ - 1))] : g.b0 + (lane & (TJ - 1));
  __builtin_amdgcn_sched_barrier(0);
  // one descriptor at the tile's first row; every load a scalar byte offset
  const float* Ct = A.C + g.c0 + (long long)g.r0 * TJ;
  const __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void*)Ct, (short)0, 0x7fffffff, 0x00020000);
  const int stride_b = 2 * NW * TJ * 4;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int rwj = g.r0 + 2 * (v + WT * j);
    const int nkj = rwj < g.r1 ? min(R, (g.r1 - rwj + 2 * NW - 1) / (2 * NW)) : 0;
    const int base = __builtin_amdgcn_readfirstlane((rwj - g.r0) * TJ * 4);
    const int klast = __builtin_amdgcn_readfirstlane(nkj > 0 ? nkj - 1 : 0);
#pragma unroll
    for (int k = 0; k < R; ++k)
      p[j][k] = __uint_as_float(
          __builtin_amdgcn_raw_buffer_load_b32(rsrc, lane * 4, base + min(k, klast) * stride_b, 0));
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int a = 0; a < NA; ++a) av[a] = ia[a] >= 0 ? A.alpha[ia[a]] : -INFINITY;
  bj = A.beta[ib];
}

// red: this team's [3][NW][TJ] partials; aw: per real wavefront alpha slot;
// kap_s: this team's TJ kappas.  act = false: the team has no tile this
// round and only takes part in the workgroup barriers.
template <int R, int K, int PHASE, bool SNAP>
__device__ __forceinline__ void tile_body(const GradArgs& A, const TileGeo& g, bool act,
                                          const float (&av)[av_regs(R, K)], float bj, float (&p)[K][R],
                                          float (*red)[NW][TJ], float (*aw)[WAVE * av_regs(R, K)],
                                          float* kap_s) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int h = lane >> 5, c = lane & (TJ - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int WT = NW / K;
  const int v = w % WT;
  const int r1 = g.r1;
  const bool colok = act && c < g.ncol;
  constexpr bool snap = SNAP && PHASE != 2;
  // this wavefront's alpha values through its own LDS slot (written and read
  // by the same wavefront: no barrier)
#pragma unroll
  for (int a = 0; a < av_regs(R, K); ++a) aw[w][a * WAVE + lane] = av[a];
  // a padding column gets beta = -inf: with alpha = -inf past the tile,
  // every entry outside the tile has f = -inf and p exactly 0 (the entries
  // inside are computed exactly as written); snapshots mask explicitly
  // because they also sum [f]_-
  const float bjm = colok ? bj : -INFINITY;
  static_assert(WT > 1, "teams of at least two wavefronts");
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int rwj = g.r0 + 2 * (v + WT * j);
    const int nkj = (act && rwj < r1) ? min(R, (r1 - rwj + 2 * NW - 1) / (2 * NW)) : 0;
    float z2 = 0.f, s1 = 0.f, o2 = 0.f;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      // loads past the last row (k >= nk) re-read valid memory and meet
      // alpha = -inf, so they need no branch either (snapshots skip them)
      float pk = 0.f;
      if (!snap || k < nkj) {
        const float ak = aw[w][2 * R * j + 2 * k + h];
        const float f = (ak + bjm) - p[j][k];
        pk = fmaxf(f, 0.f);
        if (snap) {
          const bool ok = (rwj + 2 * NW * k + h < r1) && colok;
          pk = ok ? pk : 0.f;
          const float nkv = ok ? fminf(f, 0.f) : 0.f;
          o2 = fmaf(nkv, nkv, o2);
        }
        if (PHASE != 2) {
          z2 = fmaf(pk, pk, z2);
          s1 += pk;
        }
      }
      p[j][k] = pk;
    }
    if (PHASE != 2) {
      // the two row parities of a column; virtual wavefront v + WT j's partials
      z2 += __shfl_xor(z2, 32);
      s1 += __shfl_xor(s1, 32);
      if (snap) o2 += __shfl_xor(o2, 32);
      if (h == 0) {
        red[0][v + WT * j][c] = z2;
        red[1][v + WT * j][c] = s1;
        if (snap) red[2][v + WT * j][c] = o2;
      }
    }
  }

  float kap = 0.f;
  if (PHASE != 2) {
    __syncthreads();
    // wavefront 0 of the team sums the NW virtual partials in order and
    // forms kappa; the others take kappa from LDS
    if (v == 0) {
      float Z2 = 0.f, S1 = 0.f, O2 = 0.f;
#pragma unroll 4
      for (int u = 0; u < NW; ++u) {
        Z2 += red[0][u][c];
        S1 += red[1][u][c];
      }
      if (snap) {
#pragma unroll 4
        for (int u = 0; u < NW; ++u) O2 += red[2][u][c];
      }
      if (PHASE == 1) {
        // column partial sums of chunk `aux` of a split group
        if (h == 0 && act) {
          const long long q = g.part0 + c;
          A.part[q] = Z2;
          A.part[q + A.part_stride] = S1;
          A.part[q + 2 * A.part_stride] = O2;
        }
      } else {
        const float z = sqrtf(Z2);
        float num = 0.f;
        if (z > g.thr) {
          num = z - g.thr;
          kap = num / (g.gamma * z);
        }
        if (h == 0) {
          if (act) {
            const size_t pr = (size_t)(g.pr0 + c);
            A.colsum[pr] = kap * S1;
            A.excess[pr] = num;
            if (A.write_kappa) A.kappa[pr] = kap;
            if (snap) {
              A.zsnap[pr] = z;
              A.osnap[pr] = sqrtf(O2);
            }
          }
          kap_s[c] = kap;
        }
      }
    }
    if (PHASE == 1) return;
    __syncthreads();
    kap = kap_s[c];
  } else {
    kap = act ? A.kappa[(size_t)(g.pr0 + c)] : 0.f;
  }
  if (!act) return;

  // row partials of this column block, rows relative to the group start
  float* __restrict__ rp = A.rowpart + g.rp0;
  if (__ballot(kap > 0.f) == 0ull) {
    // every block of the tile is zero: its row sums are exact zeros (slot
    // s = 2 k + h of load k, parity h; 2 R slots per virtual wavefront)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int rwj = g.r0 + 2 * (v + WT * j);
      const int nkj = rwj < r1 ? min(R, (r1 - rwj + 2 * NW - 1) / (2 * NW)) : 0;
#pragma unroll
      for (int a = 0; a < (2 * R + WAVE - 1) / WAVE; ++a) {
        const int kk = (a * WAVE + lane) >> 1;
        const int arow = rwj + 2 * NW * kk + (lane & 1);
        if (kk < nkj && arow < r1) rp[arow] = 0.f;
      }
    }
    return;
  }
  // Row sums, two loads (four rows) at a time: a permlane16 swap pairs the
  // lane rows of loads k0 = 2m and k1 = 2m + 1, DPP shifts finish inside 16
  // lanes; lane 16 q + 15 then holds the row of load k0 + (q & 1), parity
  // q >> 1.
  const int q = lane >> 4;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int rwj = g.r0 + 2 * (v + WT * j);
    const int nkj = rwj < r1 ? min(R, (r1 - rwj + 2 * NW - 1) / (2 * NW)) : 0;
#pragma unroll
    for (int m = 0; m < (R + 1) / 2; ++m) {
      const float va = kap * p[j][2 * m];
      const float vb = (2 * m + 1 < R) ? kap * p[j][(2 * m + 1 < R) ? 2 * m + 1 : 0] : 0.f;
      const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(va), __float_as_uint(vb), false, false);
      const float x = row16_sum(__uint_as_float(sw[0]) + __uint_as_float(sw[1]));
      const int k = 2 * m + (q & 1);
      const int row = rwj + 2 * NW * k + (q >> 1);
      if ((lane & 15) == 15 && k < nkj && row < r1) rp[row] = x;
    }
  }
}

template <int R, int K, int PHASE, bool SNAP>
__device__ __forceinline__ void grad_tile(const GradArgs& A, const TileGeo& g, bool act,
                                          float (*red)[NW][TJ], float (*aw)[WAVE * av_regs(R, K)],
                                          float* kap_s) {
  float av[av_regs(R, K)], bj, p[K][R];
  tile_loads<R, K>(A, g, act, av, bj, p);
  // keep every load of the wavefront in flight before any is consumed
  __builtin_amdgcn_sched_barrier(0);
  tile_body<R, K, PHASE, SNAP>(A, g, act, av, bj, p, red, aw, kap_s);
}

// Whole-group tiles read the list's records.  A workgroup issues the loads
// of its first record, the tile count (dynamic lists) and the mode of a
// single instance together; the grid never exceeds the list's capacity, so
// the first record is in bounds even past the current count.
struct RecStart {
  int n, mode0;
  TileRec r;
};

__device__ __forceinline__ RecStart rec_start(const GradArgs& A) {
  RecStart q;
  q.r = A.rec[blockIdx.x];
  q.mode0 = A.inst_mode[0];
  q.n = A.n_static >= 0 ? A.n_static : *A.count;
  return q;
}

// Whole-group tiles (PHASE 0) with the next tile's loads in flight while the
// current tile's body runs (same arithmetic as grad_tile).
template <int R>
struct TileLoad {
  TileGeo g;
  float av[av_regs(R, 1)], bj;
  float v[1][R];
};

template <int R, bool SNAP>
__global__ void __launch_bounds__(BLOCK) k_grad_tiles_pf(GradArgs A) {
  static_assert(R <= RMAX, "two tiles in registers only up to RMAX loads per lane");
  __shared__ float red[3][NW][TJ];
  __shared__ float aw[NW][WAVE * av_regs(R, 1)];
  __shared__ float kap_s[TJ];
  const RecStart q = rec_start(A);
  if (A.single_inst && !mode_takes(q.mode0, SNAP)) return;
  const int n = q.n;
  // skip tiles of the other mode (their loads would be wasted)
  auto next_match = [&](int from) {
    int u = from;
    if (!A.single_inst)
      while (u < n && !mode_takes(A.inst_mode[A.rec[u].inst], SNAP)) u += gridDim.x;
    return u;
  };
  int t = next_match(blockIdx.x);
  if (t >= n) return;
  TileLoad<R> cur, nxt;
  cur.g = geo_rec(t == (int)blockIdx.x ? q.r : A.rec[t]);
  tile_loads<R, 1>(A, cur.g, true, cur.av, cur.bj, cur.v);
  for (;;) {
    const int tn = next_match(t + gridDim.x);
    if (tn < n) {
      nxt.g = geo_rec(A.rec[tn]);
      tile_loads<R, 1>(A, nxt.g, true, nxt.av, nxt.bj, nxt.v);
    }
    tile_body<R, 1, 0, SNAP>(A, cur.g, true, cur.av, cur.bj, cur.v, red, aw, kap_s);
    __syncthreads();
    if (tn >= n) break;
    t = tn;
    cur = nxt;
  }
}

// Whole-group tiles (PHASE 0, R <= 16) whose cost tile is copied into LDS
// by direct buffer-to-LDS loads: the copy of the next tile runs while the
// current one's body runs from registers.  Same arithmetic as grad_tile.
constexpr int DMA_RMAX = 16;

template <int R, bool SNAP>
__global__ void __launch_bounds__(BLOCK, 8) k_grad_tiles_dma(GradArgs A) {
  static_assert(R <= DMA_RMAX, "LDS tile buffer sized for R <= 16");
  __shared__ float red[3][NW][TJ];
  __shared__ float aw[NW][WAVE * av_regs(R, 1)];
  __shared__ float kap_s[TJ];
  __shared__ __attribute__((aligned(16))) float buf[2 * NW * R * TJ];   // 32 R rows of 32 floats
  const RecStart q0 = rec_start(A);
  if (A.single_inst && !mode_takes(q0.mode0, SNAP)) return;
  const int n = q0.n;
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  auto match = [&](int u) {
    if (!A.single_inst)
      while (u < n && !mode_takes(A.inst_mode[A.rec[u].inst], SNAP)) u += gridDim.x;
    return u;
  };
  // the tile's rows are one contiguous [gn x 32] stream: 1 KB pieces (8
  // rows), piece q to LDS bytes [1024 q, 1024 q + 1024); pieces past the
  // tile read the pool's following rows (in bounds) and land inside buf.
  // alpha and beta of the tile are loaded into registers alongside.
  auto issue = [&](const TileGeo& g, float (&av)[1], float& bj) {
    const int rw = 2 * w;
    const int nk = rw < g.r1 ? min(R, (g.r1 - rw + 2 * NW - 1) / (2 * NW)) : 0;
    const int arow = rw + 2 * NW * (lane >> 1) + (lane & 1);
    av[0] = ((lane >> 1) < nk && arow < g.r1) ? tile_alpha(A, g.a0 + arow) : -INFINITY;
    bj = tile_beta(A, g.b0 + (lane & (TJ - 1)));
    const float* Ct = A.C + g.c0;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)Ct, (short)0, 0x7fffffff, 0x00020000);
    const int npc = __builtin_amdgcn_readfirstlane((g.r1 + 7) / 8);
    for (int q = w; q < npc; q += NW)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void*)(buf + q * 256), 16,
                                               lane * 16, q * 1024, 0, 0);
  };
  int t = match(blockIdx.x);
  if (t >= n) return;
  TileGeo g = geo_rec(t == (int)blockIdx.x ? q0.r : A.rec[t]);
  float av[1], bj;
  issue(g, av, bj);
  for (;;) {
    __builtin_amdgcn_s_waitcnt(0);   // this wavefront's copies have landed
    __syncthreads();                 // and everybody else's
    float v[1][R];
#pragma unroll
    for (int k = 0; k < R; ++k) v[0][k] = buf[(2 * w + 2 * NW * k) * TJ + lane];   // rows 2 (w + 16 k) + h
    __syncthreads();                 // buffer free for the next tile
    const int tn = match(t + gridDim.x);
    float avn[1] = {0.f}, bjn = 0.f;
    TileGeo gn_ = g;
    if (tn < n) {
      gn_ = geo_rec(A.rec[tn]);
      issue(gn_, avn, bjn);
    }
    tile_body<R, 1, 0, SNAP>(A, g, true, av, bj, v, red, aw, kap_s);
    __syncthreads();
    if (tn >= n) break;
    t = tn;
    g = gn_;
    av[0] = avn[0];
    bj = bjn;
  }
}

// One instantiation per row bucket R (a multiple of 4) for whole-group tiles
// (PHASE 0, over records), R = RMAX for the two passes over split-group
// chunks (descriptors).  SNAP kernels take only the tiles of instances
// evaluated at a snapshot, the others the rest (separate kernels keep the
// common path's register count low enough for two workgroups per compute
// unit).  K > 1 (small groups, PHASE 0): K teams of NW / K wavefronts, team
// t of workgroup b taking list entries b K + t, b K + t + K gridDim.x, ...;
// every team runs each round (an idle one only joins the barriers).
template <int R, int PHASE, bool SNAP, int K = 1>
__global__ void __launch_bounds__(BLOCK, R * K <= 16 ? 8 : 1) k_grad_tiles(GradArgs A) {
  static_assert(K == 1 || PHASE == 0, "teams only for whole-group tiles");
  static_assert(PHASE == 0 || R == RMAX, "split-group chunks run with RMAX loads per lane");
  __shared__ float red[K][3][NW][TJ];
  __shared__ float aw[NW][WAVE * av_regs(R, K)];
  __shared__ float kap_s[K][TJ];
  if (PHASE == 0 && K > 1) {
    const int team = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6) / (NW / K));
    const int n = A.n_static >= 0 ? A.n_static : *A.count;
    const int mode0 = A.inst_mode[0];
    if (A.single_inst && !mode_takes(mode0, SNAP)) return;
    for (int t0 = blockIdx.x * K; t0 < n; t0 += gridDim.x * K) {
      const int t = t0 + team;
      bool act = t < n;
      TileRec r = {};
      if (act) {
        r = A.rec[t];
        act = A.single_inst || mode_takes(A.inst_mode[r.inst], SNAP);
      }
      grad_tile<R, K, 0, SNAP>(A, geo_rec(r), act, red[team], aw, kap_s[team]);
      __syncthreads();
    }
    return;
  }
  if (PHASE == 0) {
    const RecStart q = rec_start(A);
    if (A.single_inst && !mode_takes(q.mode0, SNAP)) return;
    for (int t = blockIdx.x; t < q.n; t += gridDim.x) {
      const TileRec r = t == (int)blockIdx.x ? q.r : A.rec[t];
      if (!A.single_inst && !mode_takes(A.inst_mode[r.inst], SNAP)) continue;
      grad_tile<R, 1, 0, SNAP>(A, geo_rec(r), true, red[0], aw, kap_s[0]);
      __syncthreads();
    }
    return;
  }
  // the row-sum pass of split groups has one variant for every mode
  if (A.single_inst && (PHASE == 2 ? A.inst_mode[0] == EM_SKIP : !mode_takes(A.inst_mode[0], SNAP))) return;
  const int n = *A.count;
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const TileDesc d = A.list[t];
    const int m = A.inst_mode[d.inst];
    if (PHASE == 2 ? m == EM_SKIP : !mode_takes(m, SNAP)) continue;
    grad_tile<R, 1, PHASE, SNAP>(A, geo_desc<PHASE>(A, d), true, red[0], aw, kap_s[0]);
    __syncthreads();
  }
}

// Whole-group tiles of both kinds in one launch (evaluations where some
// instance may be at a snapshot): the mode of a tile's instance picks the
// body, so no launch is spent on a kind that has no tile.  K teams as in
// k_grad_tiles.
template <int R, int K = 1>
__global__ void __launch_bounds__(BLOCK, 8) k_grad_tiles_mixed(GradArgs A) {
  static_assert(R * K <= 16, "both bodies in one kernel only for R K <= 16");
  __shared__ float red[K][3][NW][TJ];
  __shared__ float aw[NW][WAVE * av_regs(R, K)];
  __shared__ float kap_s[K][TJ];
  if (K > 1) {
    const int team = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6) / (NW / K));
    const int n = A.n_static >= 0 ? A.n_static : *A.count;
    const int mode0 = A.inst_mode[0];
    if (A.single_inst && mode0 == EM_SKIP) return;
    // K >= 4 (groups of at most 128 rows, rounds of small tiles): the next
    // round's record is fetched while the current round runs (with K = 2
    // the extra registers would spill)
    constexpr bool PF = K >= 4;
    const int step = gridDim.x * K;
    TileRec rn = {};
    if (PF && blockIdx.x * K + team < n) rn = A.rec[blockIdx.x * K + team];
    for (int t0 = blockIdx.x * K; t0 < n; t0 += step) {
      const int t = t0 + team;
      bool act = t < n;
      TileRec r = {};
      int m = mode0;
      if (PF) {
        r = rn;
        if (t + step < n) rn = A.rec[t + step];
      }
      if (act) {
        if (!PF) r = A.rec[t];
        if (!A.single_inst) m = A.inst_mode[r.inst];
        act = m != EM_SKIP;
      }
      if (m == EM_SNAPSHOT) grad_tile<R, K, 0, true>(A, geo_rec(r), act, red[team], aw, kap_s[team]);
      else grad_tile<R, K, 0, false>(A, geo_rec(r), act, red[team], aw, kap_s[team]);
      __syncthreads();
    }
    return;
  }
  const RecStart q = rec_start(A);
  for (int t = blockIdx.x; t < q.n; t += gridDim.x) {
    const TileRec r = t == (int)blockIdx.x ? q.r : A.rec[t];
    const int m = A.single_inst ? q.mode0 : A.inst_mode[r.inst];
    if (m == EM_SKIP) {
      if (A.single_inst) return;
      continue;
    }
    if (m == EM_SNAPSHOT) grad_tile<R, 1, 0, true>(A, geo_rec(r), true, red[0], aw, kap_s[0]);
    else grad_tile<R, 1, 0, false>(A, geo_rec(r), true, red[0], aw, kap_s[0]);
    __syncthreads();
  }
}

// Split groups: combine the chunk partials of every listed (group, column
// block) in chunk order and finalise kappa, the column sums, the objective
// share and the snapshot, exactly as the single-pass tile does.  One
// wavefront per entry (blockDim 64); entries are group tiles (aux unused).
__global__ void __launch_bounds__(WAVE) k_split_combine(GradArgs A) {
  const int n = *A.count;
  const int lane = threadIdx.x;
  if (lane >= TJ) return;   // one lane per column of the tile
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const TileDesc d = A.list[t];
    if (A.inst_mode[d.inst] == EM_SKIP) continue;
    const InstDev I = A.inst[d.inst];
    const int gn = A.g_size[I.grp_off + d.grp];
    const int nch = (gn + CHUNK - 1) / CHUNK;
    const int col = d.jb * TJ + lane;
    const long long q0 =
        I.chunk_off + (long long)A.g_chunk0[I.grp_off + d.grp] * I.nt_pad + col;
    float Z2 = 0.f, S1 = 0.f, O2 = 0.f;
    for (int c = 0; c < nch; ++c) {
      const long long q = q0 + (long long)c * I.nt_pad;
      Z2 += A.part[q];
      S1 += A.part[q + A.part_stride];
      O2 += A.part[q + 2 * A.part_stride];
    }
    const float z = sqrtf(Z2);
    float num = 0.f, kap = 0.f;
    if (z > I.thr) {
      num = z - I.thr;
      kap = num / (I.gamma * z);
    }
    const size_t pr = (size_t)I.pair_off + (size_t)d.grp * I.nt_pad + col;
    A.kappa[pr] = kap;
    A.colsum[pr] = kap * S1;
    A.excess[pr] = num;
    if (A.inst_mode[d.inst] == EM_SNAPSHOT) {
      A.zsnap[pr] = z;
      A.osnap[pr] = sqrtf(O2);
    }
  }
}

// ---------------------------------------------------------------- assembly

// Host-directed evaluation prologue: every instance gets `mode`; for dense
// evaluations the counters are advanced here (screened ones count in the
// screen pass).
struct Prologue {
  int* inst_mode;
  int count, mode;
  long long* counters;
  long long pairs_valid, tiles;
};

__device__ __forceinline__ void prologue_body(const Prologue& P) {
  for (int k = threadIdx.x; k < P.count; k += blockDim.x) P.inst_mode[k] = P.mode;
  if (threadIdx.x == 0 && P.mode == EM_DENSE) {
    unsigned long long* C = (unsigned long long*)P.counters;
    atomicAdd(&C[CNT_EVALS], (unsigned long long)P.count);
    atomicAdd(&C[CNT_PAIRS_TOTAL], (unsigned long long)P.pairs_valid);
    atomicAdd(&C[CNT_TILES_TOTAL], (unsigned long long)P.tiles);
    atomicAdd(&C[CNT_TILES_COMPUTED], (unsigned long long)P.tiles);
  }
}


// caller-order (alpha, beta) -> internal order; padding columns get 0.
// Flags non-finite inputs.  grid.y instance.  With do_prologue, workgroup
// (0, 0) also runs the evaluation prologue.
__global__ void __launch_bounds__(256) k_gather_duals(const InstDev* __restrict__ inst,
                                                      const int* __restrict__ perm_row,
                                                      const int* __restrict__ perm_col,
                                                      const float* __restrict__ alpha,
                                                      const float* __restrict__ beta,
                                                      float* __restrict__ al_int,
                                                      float* __restrict__ be_int,
                                                      int* __restrict__ err, Prologue P, int do_prologue) {
  if (do_prologue && blockIdx.x == 0 && blockIdx.y == 0) prologue_body(P);
  const InstDev I = inst[blockIdx.y];
  bool bad = false;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < I.ns; r += gridDim.x * blockDim.x) {
    const float v = alpha[I.row_off + perm_row[I.row_off + r]];
    bad |= !isfinite(v);
    al_int[I.row_off + r] = v;
  }
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < I.nt_pad; c += gridDim.x * blockDim.x) {
    float v = 0.f;
    if (c < I.nt) v = beta[I.scol_off + perm_col[I.col_off + c]];
    bad |= !isfinite(v);
    be_int[I.col_off + c] = v;
  }
  if (bad) atomicOr(err, 8);   // a NaN or Inf dual value (reported by checked calls)
}

// caller-order index of every internal row and column (padding columns:
// the instance's first target, a valid address whose value is masked)
__global__ void __launch_bounds__(256) k_build_maps(const InstDev* __restrict__ inst,
                                                    const int* __restrict__ perm_row,
                                                    const int* __restrict__ perm_col, int* __restrict__ row_map,
                                                    int* __restrict__ col_map) {
  const InstDev I = inst[blockIdx.y];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < I.ns; r += gridDim.x * blockDim.x)
    row_map[I.row_off + r] = I.row_off + perm_row[I.row_off + r];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < I.nt_pad; c += gridDim.x * blockDim.x)
    col_map[I.col_off + c] = I.scol_off + (c < I.nt ? perm_col[I.col_off + c] : 0);
}

__global__ void k_prologue(int* inst_mode, int count, int mode, long long* counters,
                           long long pairs_valid, long long tiles) {
  prologue_body(Prologue{inst_mode, count, mode, counters, pairs_valid, tiles});
}

// internal order -> caller order
__global__ void __launch_bounds__(256) k_scatter_duals(const InstDev* __restrict__ inst,
                                                       const int* __restrict__ perm_row,
                                                       const int* __restrict__ perm_col,
                                                       const float* __restrict__ al_int,
                                                       const float* __restrict__ be_int,
                                                       float* __restrict__ alpha,
                                                       float* __restrict__ beta) {
  const InstDev I = inst[blockIdx.y];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < I.ns; r += gridDim.x * blockDim.x)
    alpha[I.row_off + perm_row[I.row_off + r]] = al_int[I.row_off + r];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < I.nt; c += gridDim.x * blockDim.x)
    beta[I.scol_off + perm_col[I.col_off + c]] = be_int[I.col_off + c];
}

// Dense plan in the caller's order (Sec. 2.3): T[i][j] = kappa_lj max(f_ij, 0)
// with kappa_lj written per pair by a preceding dense evaluation.
// grid.x columns / 256, grid.y rows (strided), grid.z instance.
__global__ void __launch_bounds__(256) k_plan_dense(const InstDev* __restrict__ inst,
                                                    const int* __restrict__ perm_row,
                                                    const int* __restrict__ perm_col,
                                                    const int* __restrict__ row_grp,
                                                    const int* __restrict__ g_start,
                                                    const int* __restrict__ g_size,
                                                    const float* __restrict__ C,
                                                    const float* __restrict__ alpha,
                                                    const float* __restrict__ beta,
                                                    const float* __restrict__ kappa,
                                                    const long long* __restrict__ t_off,
                                                    float* __restrict__ T) {
  const InstDev I = inst[blockIdx.z];
  for (int r = blockIdx.y; r < I.ns; r += gridDim.y) {
    const int g = row_grp[I.row_off + r];
    const int gs = g_start[I.grp_off + g], gn = g_size[I.grp_off + g];
    const float a = alpha[I.row_off + r];
    float* trow = T + t_off[blockIdx.z] + (size_t)perm_row[I.row_off + r] * I.nt;
    const float* krow = kappa + I.pair_off + (size_t)g * I.nt_pad;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < I.nt; c += gridDim.x * blockDim.x) {
      const float f = (a + beta[I.col_off + c]) - C[c_index(I, gs, gn, r, c)];
      trow[perm_col[I.col_off + c]] = krow[c] * fmaxf(f, 0.f);
    }
  }
}


// Plan recovery in compressed sparse row form, per (row, 32-target column
// block) segment: CSR_COUNT writes the number of nonzero entries of row i in
// column block jb to cnt[i * cstride + jb] (i the caller row, stacked over
// the instances); CSR_FILL writes entry (i, j) at seg[i * cstride + jb] plus
// its rank among the row's nonzero entries of the block (internal column
// order), as the caller's column j and the value.
enum PlanMode { PLAN_DENSE = 1, CSR_COUNT = 2, CSR_FILL = 3 };

struct CsrSink {
  int* cnt;             // CSR_COUNT: [rows][cstride]
  const long long* seg; // CSR_FILL: [rows][cstride] segment offsets
  long long cstride;
  int* col;
  float* val;
};

// One entry per lane of a 64-lane group whose half h (lanes 32 h ..
// 32 h + 31, column c) shares one row: the half's nonzero pattern by ballot.
template <int MODE>
__device__ __forceinline__ void csr_emit(const CsrSink& K, bool ok, int grow, int jb, int c, int h, int dcol,
                                         float v) {
  const unsigned long long b = __ballot(ok && v > 0.f);
  const unsigned m = (unsigned)(h ? (b >> 32) : b);
  if (MODE == CSR_COUNT) {
    if (c == 0 && ok) K.cnt[(size_t)grow * K.cstride + jb] = __popc(m);
  } else {
    if (ok && v > 0.f) {
      const long long sg = K.seg[(size_t)grow * K.cstride + jb];
      if (sg >= 0) {   // rows whose count disagrees with the caller's row_ptr are skipped
        const long long pos = sg + __popc(m & ((1u << c) - 1u));
        K.col[pos] = dcol;
        K.val[pos] = v;
      }
    }
  }
}

// Materialized cost: one wavefront per two rows of a (group, column block)
// tile at a time (lane = 32 h + c), every tile of the handle.
template <int MODE>
__global__ void __launch_bounds__(256) k_plan_csr(const InstDev* __restrict__ inst, const TileDesc* __restrict__ tiles,
                                                  int ntiles, const int* __restrict__ perm_row,
                                                  const int* __restrict__ perm_col, const int* __restrict__ g_start,
                                                  const int* __restrict__ g_size, const float* __restrict__ C,
                                                  const float* __restrict__ alpha, const float* __restrict__ beta,
                                                  const float* __restrict__ kappa, CsrSink K) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int h = lane >> 5, c = lane & (TJ - 1);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const TileDesc d = tiles[t];
    const InstDev I = inst[d.inst];
    const int gs = g_start[I.grp_off + d.grp], gn = g_size[I.grp_off + d.grp];
    const int col = d.jb * TJ + c;
    const bool colok = col < I.nt;
    const float bj = colok ? beta[I.col_off + col] : 0.f;
    const float kap = colok ? kappa[(size_t)I.pair_off + (size_t)d.grp * I.nt_pad + col] : 0.f;
    const int dcol = colok ? perm_col[I.col_off + col] : 0;
    for (int r0 = 2 * w; r0 < gn; r0 += 2 * nw) {
      const int r = r0 + h;
      const bool ok = r < gn && colok;
      float v = 0.f;
      int grow = 0;
      if (ok) {
        const float f = (alpha[I.row_off + gs + r] + bj) - C[c_index(I, gs, gn, gs + r, col)];
        v = kap * fmaxf(f, 0.f);
        grow = I.row_off + perm_row[I.row_off + gs + r];
      }
      csr_emit<MODE>(K, ok, grow, d.jb, c, h, dcol, v);
    }
  }
}

// Row totals of the segment counts (CSR_COUNT output), caller rows of
// instance blockIdx.y
__global__ void __launch_bounds__(256) k_csr_rowsum(const InstDev* __restrict__ inst, const int* __restrict__ cnt,
                                                    long long cstride, long long* __restrict__ tot) {
  const InstDev I = inst[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < I.ns; i += gridDim.x * blockDim.x) {
    const int* ci = cnt + (size_t)(I.row_off + i) * cstride;
    long long t = 0;
    for (int jb = 0; jb < I.njb; ++jb) t += ci[jb];
    tot[I.row_off + i] = t;
  }
}

// Segment offsets from the caller's row pointers: seg[i][jb] = row_ptr[i]
// plus the counts of the row's earlier column blocks.  A row whose total
// differs from row_ptr[i + 1] - row_ptr[i] (a point other than the count
// call's) gets -1 everywhere (nothing is written for it) and sets bit 16 of
// err.
__global__ void __launch_bounds__(256) k_csr_segoff(const InstDev* __restrict__ inst, const int* __restrict__ cnt,
                                                    long long cstride, const long long* __restrict__ row_ptr,
                                                    long long* __restrict__ seg, int* __restrict__ err) {
  const InstDev I = inst[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < I.ns; i += gridDim.x * blockDim.x) {
    const size_t base = (size_t)(I.row_off + i) * cstride;
    const long long r0 = row_ptr[I.row_off + i], r1 = row_ptr[I.row_off + i + 1];
    long long o = r0;
    for (int jb = 0; jb < I.njb; ++jb) {
      seg[base + jb] = o;
      o += cnt[base + jb];
    }
    if (o != r1) {
      for (int jb = 0; jb < I.njb; ++jb) seg[base + jb] = -1;
      atomicOr(err, 16);
    }
  }
}

// The scaled internal cost in the caller's order (materialized pool).
__global__ void __launch_bounds__(256) k_cost_dump(const InstDev* __restrict__ inst,
                                                   const int* __restrict__ perm_row,
                                                   const int* __restrict__ perm_col,
                                                   const int* __restrict__ row_grp,
                                                   const int* __restrict__ g_start,
                                                   const int* __restrict__ g_size,
                                                   const float* __restrict__ C,
                                                   const long long* __restrict__ t_off,
                                                   float* __restrict__ out) {
  const InstDev I = inst[blockIdx.z];
  for (int r = blockIdx.y; r < I.ns; r += gridDim.y) {
    const int g = row_grp[I.row_off + r];
    const int gs = g_start[I.grp_off + g], gn = g_size[I.grp_off + g];
    float* orow = out + t_off[blockIdx.z] + (size_t)perm_row[I.row_off + r] * I.nt;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < I.nt; c += gridDim.x * blockDim.x)
      orow[perm_col[I.col_off + c]] = C[c_index(I, gs, gn, r, c)];
  }
}

// ---------------------------------------------------------------- on-the-fly cost

// x_i . y_j for the 32 rows of a packed source block and the 32 columns of a
// packed target block, on v_mfma_f32_32x32x2f32 (two dims per instruction,
// dims in increasing order).  Both operands come from global memory, 1 KB
// contiguous per wavefront load, the next 16 dims in flight while the
// current ones are multiplied.  Result: lane l, element q holds row
// 8 (q / 4) + 4 (l / 32) + (q % 4) of the block, column l % 32.
template <bool PREFETCH = true>
__device__ __forceinline__ floatx16 otf_dot_block(const float* __restrict__ xblk,
                                                  const float* __restrict__ yblk, int DP, int lane) {
  floatx16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const float4* xa = (const float4*)(xblk + lane * 8);   // lane = 32 h + c
  const float4* ya = (const float4*)(yblk + lane * 8);
  const int nm = DP >> 4;                                // chunks of 16 dims: 128 float4
  float4 x0 = xa[0], x1 = xa[1], y0 = ya[0], y1 = ya[1];
  for (int m8 = 0; m8 < nm; ++m8) {
    float4 nx0, nx1, ny0, ny1;
    if (PREFETCH) {
      const int nx = min(m8 + 1, nm - 1) * 128;
      nx0 = xa[nx];
      nx1 = xa[nx + 1];
      ny0 = ya[nx];
      ny1 = ya[nx + 1];
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, y0.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.y, y0.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.z, y0.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.w, y0.w, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.x, y1.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.y, y1.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.z, y1.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.w, y1.w, acc, 0, 0, 0);
    if (PREFETCH) {
      x0 = nx0;
      x1 = nx1;
      y0 = ny0;
      y1 = ny1;
    } else if (m8 + 1 < nm) {
      const int nx = (m8 + 1) * 128;
      x0 = xa[nx];
      x1 = xa[nx + 1];
      y0 = ya[nx];
      y1 = ya[nx + 1];
    }
  }
  return acc;
}

// Cost of one element: C = max(s ((|x_i|^2 + |y_j|^2) - 2 x_i.y_j), 0).
__device__ __forceinline__ float otf_cost(float xn_i, float yn_j, float dot, float s) {
  return fmaxf(s * ((xn_i + yn_j) - 2.f * dot), 0.f);
}

// lane value of row r (0..31) of a 32-row block whose values sit one per lane
// in lanes 0..31 (and again in 32..63): element q of the MFMA layout needs row
// 8 (q / 4) + (q % 4) in lanes 0..31 and that row + 4 in lanes 32..63.
__device__ __forceinline__ float otf_row_value(float v, int q, int h) {
  const int r = 8 * (q / 4) + (q % 4);
  const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), r));
  const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), r + 4));
  return h ? b : a;
}

// Gradient tiles with the cost computed on matrix cores.  A team of WT
// wavefronts takes one entry of the work list; each wavefront covers up to
// BPW 32-row blocks of its tile (its p values stay in registers), so a team
// holds 32 BPW WT rows (tiles are bucketed by group size to fit; larger
// groups are cut in chunks of CHUNK = 64 NW rows, WT = NW, BPW = 2).  A
// workgroup holds K = NWV / WT teams, NWV = max(WT, 4) wavefronts.  PHASE as
// in grad_tile: 0 whole group, 1 chunk column partials, 2 chunk row sums (only
// tiles with a nonzero kappa recompute their cost).
template <int WT>
constexpr int otf_waves() { return WT < 4 ? 4 : WT; }

template <int WT, int BPW, int PHASE, bool SNAP>
__global__ void __launch_bounds__(64 * otf_waves<WT>(), (PHASE == 1 || BPW == 1) ? 8 : 1)
    k_grad_tiles_otf(GradArgs A) {
  constexpr int NWV = otf_waves<WT>();
  constexpr int K = NWV / WT;
  constexpr bool snap = SNAP && PHASE != 2;
  constexpr int TB = WT * BPW;   // row blocks of a team
  // one team of 8 or more wavefronts per workgroup: every wavefront
  // multiplies by the same target block, staged once in LDS (dynamic
  // shared memory of 32 dp floats); the row-sum pass of split groups, which
  // mostly skips, reads it from global memory
  constexpr bool YL = K == 1 && WT >= 8 && PHASE != 2;
  extern __shared__ __attribute__((aligned(16))) float ylds[];
  // per-block partial sums; a tile's sums run over its blocks in order, so
  // the result does not depend on the team shape (WT, BPW)
  __shared__ float red[3][K * TB][TJ];
  if (A.single_inst && (PHASE == 2 ? A.inst_mode[0] == EM_SKIP : !mode_takes(A.inst_mode[0], SNAP))) return;
  const int n = *A.count;
  const int lane = threadIdx.x & (WAVE - 1);
  const int h = lane >> 5, c = lane & (TJ - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int team = w / WT, v = w % WT;
  for (int t0 = blockIdx.x * K; t0 < n; t0 += gridDim.x * K) {
    const int t = t0 + team;
    TileDesc d{0, 0, 0, 0};
    bool act = t < n;
    if (act) {
      d = A.list[t];
      const int m = A.inst_mode[d.inst];
      act = PHASE == 2 ? m != EM_SKIP : mode_takes(m, SNAP);
    }
    const InstDev I = A.inst[d.inst];
    const int gs = A.g_start[I.grp_off + d.grp];
    const int gn = A.g_size[I.grp_off + d.grp];
    int r0 = 0, r1 = gn;
    if (PHASE != 0) {
      r0 = d.aux * CHUNK;
      r1 = min(r0 + CHUNK, gn);
    }
    const int col = d.jb * TJ + c;
    const bool colok = col < I.nt;
    const size_t pr = (size_t)I.pair_off + (size_t)d.grp * I.nt_pad + col;
    const float* xg = A.Xp + I.x_off + (size_t)A.g_xblk[I.grp_off + d.grp] * 32 * I.dp;
    const float* yb = A.Yp + I.y_off + (size_t)d.jb * 32 * I.dp;

    if (YL) {
      if (act) {
        const float4* src = (const float4*)yb;
        float4* dst = (float4*)ylds;
        for (int i = threadIdx.x; i < 8 * I.dp; i += blockDim.x) dst[i] = src[i];
      }
      __syncthreads();
    }
    float kap = 0.f;
    bool anyk = true;
    if (PHASE == 2 && act) {
      kap = A.kappa[pr];
      anyk = __ballot(kap > 0.f) != 0ull;
    }
    float p[BPW][16];
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
#pragma unroll
      for (int q = 0; q < 16; ++q) p[b][q] = 0.f;
      const int i0 = r0 + 32 * (v + WT * b);   // first row of the block, in the group
      if (!act || i0 >= r1 || !anyk) continue;  // wave-uniform
      float z2 = 0.f, s1 = 0.f, o2 = 0.f;
      floatx16 acc;
      if constexpr (YL)
        acc = otf_dot_block<PHASE != 1>(xg + (size_t)(i0 / 32) * 32 * I.dp, ylds, I.dp, lane);
      else
        acc = otf_dot_block<PHASE != 1>(xg + (size_t)(i0 / 32) * 32 * I.dp, yb, I.dp, lane);
      const bool rowin = i0 + c < r1;
      const float av = rowin ? A.alpha[I.row_off + gs + i0 + c] : 0.f;
      const float xv = rowin ? A.xn[I.row_off + gs + i0 + c] : 0.f;
      const float bj = A.beta[I.col_off + col];
      const float ynj = A.yn[I.col_off + col];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int rr = 8 * (q / 4) + (q % 4) + 4 * h;
        const float C = otf_cost(otf_row_value(xv, q, h), ynj, acc[q], I.cscale);
        const float f = (otf_row_value(av, q, h) + bj) - C;
        const bool ok = (i0 + rr < r1) && colok;
        const float pk = ok ? fmaxf(f, 0.f) : 0.f;
        if (PHASE != 2) {
          z2 = fmaf(pk, pk, z2);
          s1 += pk;
          if (snap) {
            const float nkv = ok ? fminf(f, 0.f) : 0.f;
            o2 = fmaf(nkv, nkv, o2);
          }
        }
        p[b][q] = pk;
      }
      if (PHASE != 2) {
        z2 += __shfl_xor(z2, 32);
        s1 += __shfl_xor(s1, 32);
        if (snap) o2 += __shfl_xor(o2, 32);
        const int slot = team * TB + v + WT * b;
        if (h == 0) {
          red[0][slot][c] = z2;
          red[1][slot][c] = s1;
          if (snap) red[2][slot][c] = o2;
        }
      }
    }

    if (PHASE != 2) {
      __syncthreads();
      if (act) {
        float Z2 = 0.f, S1 = 0.f, O2 = 0.f;
        const int nblk = (r1 - r0 + 31) / 32;
        for (int u = 0; u < nblk; ++u) {
          Z2 += red[0][team * TB + u][c];
          S1 += red[1][team * TB + u][c];
          if (snap) O2 += red[2][team * TB + u][c];
        }
        if (PHASE == 1) {
          if (v == 0 && h == 0) {
            const long long qq = I.chunk_off +
                                 (long long)(A.g_chunk0[I.grp_off + d.grp] + d.aux) * I.nt_pad + col;
            A.part[qq] = Z2;
            A.part[qq + A.part_stride] = S1;
            A.part[qq + 2 * A.part_stride] = O2;
          }
        } else {
          const float z = sqrtf(Z2);
          float num = 0.f;
          if (z > I.thr) {
            num = z - I.thr;
            kap = num / (I.gamma * z);
          }
          if (v == 0 && h == 0) {
            A.colsum[pr] = kap * S1;
            A.excess[pr] = num;
            if (A.write_kappa) A.kappa[pr] = kap;
            if (snap) {
              A.zsnap[pr] = z;
              A.osnap[pr] = sqrtf(O2);
            }
          }
          anyk = __ballot(kap > 0.f) != 0ull;
        }
      }
    }

    if (PHASE != 1 && act) {
      float* __restrict__ rp = A.rowpart + I.r_off + (size_t)d.jb * I.ns + gs;
      const int Q = lane >> 4;
#pragma unroll
      for (int b = 0; b < BPW; ++b) {
        const int i0 = r0 + 32 * (v + WT * b);
        if (i0 >= r1) continue;
        if (!anyk) {
          if (lane < 32 && i0 + lane < r1) rp[i0 + lane] = 0.f;
          continue;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          // rows of elements 2m and 2m + 1, both halves: after the swap and
          // the row-16 sums, lane 16 Q + 15 holds row 8 (qs / 4) + qs % 4 + 4 (Q / 2)
          // with qs = 2m + Q % 2
          const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(kap * p[b][2 * m]),
                                                           __float_as_uint(kap * p[b][2 * m + 1]), false, false);
          const float x = row16_sum(__uint_as_float(sw[0]) + __uint_as_float(sw[1]));
          const int qs = 2 * m + (Q & 1);
          const int row = i0 + 8 * (qs / 4) + (qs % 4) + 4 * (Q >> 1);
          if ((lane & 15) == 15 && row < r1) rp[row] = x;
        }
      }
    }
    __syncthreads();
  }
}

// Setup pass over natural-order target blocks: per (group, target) the least
// unscaled cost u = |x|^2 + |y|^2 - 2 x.y over the group's rows (nearest-class
// clustering) and the largest u of the instance (normalisation).  grid: one
// workgroup per (group, natural 32-column block) in `list` (aux unused).
__global__ void __launch_bounds__(BLOCK) k_otf_setup(GradArgs A, int n, const float* __restrict__ Ynat,
                                                     const float* __restrict__ ynnat,
                                                     float* __restrict__ colmin,
                                                     unsigned int* __restrict__ maxbits) {
  __shared__ float red[NW][TJ];
  const int lane = threadIdx.x & (WAVE - 1);
  const int h = lane >> 5, c = lane & (TJ - 1);
  const int w = threadIdx.x >> 6;
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const TileDesc d = A.list[t];
    const InstDev I = A.inst[d.inst];
    const int gs = A.g_start[I.grp_off + d.grp];
    const int gn = A.g_size[I.grp_off + d.grp];
    const float* yb = Ynat + I.y_off + (size_t)d.jb * 32 * I.dp;
    const int col = d.jb * TJ + c;
    const float ynj = ynnat[I.col_off + col];
    float mn = INFINITY, mx = 0.f;
    for (int i0 = 32 * w; i0 < gn; i0 += 32 * NW) {
      const float* xblk = A.Xp + I.x_off + ((size_t)A.g_xblk[I.grp_off + d.grp] + i0 / 32) * 32 * I.dp;
      const floatx16 acc = otf_dot_block(xblk, yb, I.dp, lane);
      const float xv = (i0 + c < gn) ? A.xn[I.row_off + gs + i0 + c] : 0.f;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int rr0 = 8 * (q / 4) + (q % 4);
        const float u = (otf_row_value(xv, q, h) + ynj) - 2.f * acc[q];
        if (i0 + rr0 + 4 * h < gn && col < I.nt) {
          mn = fminf(mn, u);
          mx = fmaxf(mx, u);
        }
      }
    }
    mn = fminf(mn, __shfl_xor(mn, 32));
    if (h == 0) red[w][c] = mn;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0) atomicMax(&maxbits[d.inst], __float_as_uint(mx));
    __syncthreads();
    if (w == 0 && h == 0 && col < I.nt) {
      float m = INFINITY;
      for (int v = 0; v < NW; ++v) m = fminf(m, red[v][c]);
      colmin[(size_t)I.pair_off + (size_t)d.grp * I.nt_pad + col] = m;
    }
    __syncthreads();
  }
}

// The cost (MODE 0) or the plan T_ij = kappa_lj [f_ij]_+ (MODE 1) of the
// tiles of `list` (all rows of each group), written in the caller's order at
// out[t_off + perm_row(i) n_tgt + perm_col(j)].  Same arithmetic as the
// gradient tiles, so the values are the ones the gradient used.
template <int MODE>
__global__ void __launch_bounds__(BLOCK) k_otf_emit(GradArgs A, int n, const int* __restrict__ perm_row,
                                                    const int* __restrict__ perm_col,
                                                    const long long* __restrict__ t_off,
                                                    float* __restrict__ out, CsrSink K) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int h = lane >> 5, c = lane & (TJ - 1);
  const int w = threadIdx.x >> 6;
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const TileDesc d = A.list[t];
    const InstDev I = A.inst[d.inst];
    const int gs = A.g_start[I.grp_off + d.grp];
    const int gn = A.g_size[I.grp_off + d.grp];
    const float* yb = A.Yp + I.y_off + (size_t)d.jb * 32 * I.dp;
    const int col = d.jb * TJ + c;
    const bool colok = col < I.nt;
    const float ynj = A.yn[I.col_off + col];
    const float bj = A.beta[I.col_off + col];
    const float kap = MODE ? A.kappa[(size_t)I.pair_off + (size_t)d.grp * I.nt_pad + col] : 0.f;
    const int dcol = colok ? perm_col[I.col_off + col] : 0;
    float* o = out + t_off[d.inst];
    for (int i0 = 32 * w; i0 < gn; i0 += 32 * NW) {
      const float* xblk = A.Xp + I.x_off + ((size_t)A.g_xblk[I.grp_off + d.grp] + i0 / 32) * 32 * I.dp;
      const floatx16 acc = otf_dot_block(xblk, yb, I.dp, lane);
      const bool rowin = i0 + c < gn;
      const float xv = rowin ? A.xn[I.row_off + gs + i0 + c] : 0.f;
      const float av = rowin ? A.alpha[I.row_off + gs + i0 + c] : 0.f;
      const int pv = rowin ? perm_row[I.row_off + gs + i0 + c] : 0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int rr0 = 8 * (q / 4) + (q % 4);
        const int prow = __float_as_int(otf_row_value(__int_as_float(pv), q, h));
        const float C = otf_cost(otf_row_value(xv, q, h), ynj, acc[q], I.cscale);
        const float v = MODE ? kap * fmaxf((otf_row_value(av, q, h) + bj) - C, 0.f) : C;
        const bool ok = i0 + rr0 + 4 * h < gn && colok;
        if (MODE >= CSR_COUNT)
          csr_emit<(MODE >= CSR_COUNT ? MODE : CSR_COUNT)>(K, ok, I.row_off + prow, d.jb, c, h, dcol, v);
        else if (ok)
          o[(size_t)prow * I.nt + dcol] = v;
      }
    }
  }
}

// nearest source class of every target column from the per-group minima
__global__ void k_otf_assign(const InstDev* __restrict__ inst, const float* __restrict__ colmin,
                             int* __restrict__ colkey) {
  const InstDev I = inst[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= I.nt) return;
  float best = INFINITY;
  int bg = 0;
  for (int g = 0; g < I.Le; ++g) {
    const float v = colmin[(size_t)I.pair_off + (size_t)g * I.nt_pad + j];
    if (v < best) {
      best = v;
      bg = g;
    }
  }
  colkey[I.scol_off + j] = bg;
}

}  // namespace otgs
