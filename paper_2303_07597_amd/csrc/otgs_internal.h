// Internal declarations shared by the HIP translation units of libotgs.
// Device layout (all arrays packed over the instances of a handle):
//   rows    - source rows sorted by label (stable), instance k at row_off;
//             perm_row maps an internal row to the caller's row.
//   columns - target columns clustered by nearest source class (stable),
//             padded to a multiple of TJ, instance k at col_off; perm_col
//             maps an internal column to the caller's column (-1 = pad).
//   groups  - nonempty label groups, instance k at grp_off: first internal
//             row and size.
//   pairs   - (group, padded column) arrays, [Le x nt_pad] at pair_off.
//   tiles   - (group, block of TJ columns), [Le x njb] at tile_off.
//   cost    - C in the internal layout at c_off, tile-major: the rows of a
//             group form njb consecutive tiles of [g x TJ] floats, so a tile
//             (group, column block) is one contiguous stream; see c_index.
//   rowpart - row partial sums of T per column block, [njb x ns] at r_off.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace otgs {

constexpr int WAVE = 64;
constexpr int TJ = 32;                 // target columns per tile (lane = 32 h + column)
constexpr int NW = 16;                 // waves per gradient workgroup
constexpr int BLOCK = NW * WAVE;       // 1024 threads
constexpr int RMAX = 32;               // loads per lane of a split-group chunk
constexpr int CHUNK = 2 * NW * RMAX;   // 1024: rows of a split-group chunk
constexpr int RSTEP = 4;               // row buckets: R = 2, 4, 8, ..., 32 loads per lane,
constexpr int RBIG = 64;               // then 40, 48, 56, 64 (one workgroup per compute unit)
constexpr int RSTEP_BIG = 8;
constexpr int WHOLE_MAX = 2 * NW * RBIG;   // 2048: largest whole-group tile (materialised cost)
constexpr int NBUCKET = 1 + RMAX / RSTEP + (RBIG - RMAX) / RSTEP_BIG;   // 13
constexpr int MAX_GROUPS = 16384;      // label range limit (LDS histogram)
constexpr int DP_MAX = 256;            // on-the-fly cost: padded feature dims

typedef float floatx16 __attribute__((ext_vector_type(16)));   // 32 x 32 matrix-core accumulator

struct InstDev {
  int ns, nt, nt_pad, njb;
  int L;          // label range
  int Le;         // nonempty groups
  int row_off;    // packed row arrays (also the caller's row offset)
  int col_off;    // packed padded column arrays
  int scol_off;   // caller's packed column offset
  int grp_off;    // packed group arrays
  int pair_off;   // packed pair arrays
  int tile_off;   // packed tile arrays
  int pad0;
  long long chunk_off;  // split-chunk partial table offset (floats)
  long long c_off;  // cost pool offset (floats)
  long long r_off;  // row-partial pool offset (floats)
  float gamma, mu, thr;  // thr = fl32(mu * gamma)
  float cmax;            // max of the internal (scaled) cost
  // on-the-fly cost (features on matrix cores); unused otherwise
  int onthefly, dim, dp, pad1;   // dp: dims padded to a multiple of 16
  long long x_off, y_off;        // packed feature pools (floats)
  float cscale, pad2;            // C = max(cscale (|x|^2 + |y|^2 - 2 x.y), 0)
  double gamma64;                // gamma as given (the objective's 1 / (2 gamma))
};

// A segment of keys for the stable counting sort: n keys in [0, K) at
// key_off, key tables (counts / starts) at kt_off, output at out_off.
struct SegDesc {
  int n, K, key_off, kt_off, out_off, pad0, pad1, pad2;
};

// A unit of work of the gradient kernel: (instance, group, column block)
// plus the row class (whole-group tiles) or the chunk index (split groups).
struct TileDesc {
  int inst, grp, jb, aux;
};

// float64 lane move by a DPP pattern (both 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// a + b where (a, b) are the two halves of a permlane swap of x with itself:
// every lane gets x of its row (or half) plus x of the partner row (half),
// in the same order in both
template <bool HALF>
__device__ __forceinline__ double swap_sum_d(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  unsigned l0, l1, h0, h1;
  if (HALF) {
    const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
  }
  const double a = __longlong_as_double((long long)(((unsigned long long)h0 << 32) | l0));
  const double c = __longlong_as_double((long long)(((unsigned long long)h1 << 32) | l1));
  return a + c;
}

// Sum over the 64 lanes, the total in every lane with identical bits: pairs
// (xor 1), quads (xor 2), half rows and rows (mirrors), row pairs and halves
// (permlane swaps).  Every step adds two partials that are equal across the
// lanes of a group (addition commutes), so the order is fixed.
__device__ __forceinline__ double wave_sum_dd(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  v += dpp_d<0x140>(v);   // row_mirror
  v = swap_sum_d<false>(v);
  v = swap_sum_d<true>(v);
  return v;
}

// Safe-screening bounds (Def. 1 with the rounding margins derived beside
// the screen pass, and the lower bound of Def. 2).
constexpr double SCR_U = 5.9604644775390625e-08;   // 2^-24

// per-group constants of the rounding-safe upper bound for a group of n rows
__device__ __forceinline__ void screen_group_consts(int n, double& sg, double& fa, double& fb) {
  const int nch = (n + CHUNK - 1) / CHUNK;
  const double nop = (double)n + 17.0 * nch + 16.0;
  const double gam = nop * SCR_U / (1.0 - nop * SCR_U);
  sg = sqrt((double)n);
  fa = (1.0 + 2.0 * SCR_U) * sqrt(1.0 + gam) * (1.0 + 1e-9);
  fb = 1.0 / ((1.0 - 2.0 * SCR_U) * sqrt(1.0 - gam));
}

// rounding-safe upper bound on the computed norm of block (l, j): zt the
// snapshot norm, (b, bs) beta_j now and at the snapshot, up the group's
// ||[alpha - alpha~]_+||, amax / amax_s the group's max |alpha|, |alpha~|
__device__ __forceinline__ double screen_upper(double zt, double b, double bs, double up, double amax,
                                               double amax_s, double sg, double fa, double fb,
                                               double cmax) {
  const double u2 = 2.01 * SCR_U;
  const double db = b - bs;
  return fa * (zt * fb + sg * (u2 * (amax_s + amax + 2.0 * cmax + fabs(bs) + fabs(b)) +
                               (db > 0 ? db : 0.0)) + up);
}

// lower bound on the norm of block (l, j) (membership in N): all and dn the
// group's ||alpha - alpha~|| and ||[alpha - alpha~]_-||, ot the snapshot
// norm of the negative part
__device__ __forceinline__ double screen_lower(double zt, double ot, double b, double bs, double all,
                                               double dn, double sg) {
  const double db = b - bs;
  const double kt = sqrt(zt * zt + ot * ot);
  return kt - all - sg * fabs(db) - ot - dn - sg * (db < 0 ? -db : 0.0);
}

// Geometry of a whole-group tile of the materialized cost, precomputed at
// set-up so that a workgroup reaches its cost stream after a single load
// (instead of descriptor -> instance -> group tables -> data).
struct alignas(16) TileRec {
  long long c0;    // cost pool index of the tile's first entry (group row 0, block column 0)
  long long rp0;   // row-partial index of the group's first row in this column block
  long long pr0;   // pair index of the block's first column
  int a0;          // alpha index (internal order) of the group's first row
  int b0;          // beta index (internal order) of the block's first column
  int gn;          // rows of the group
  int ncol;        // valid columns of the block (1..TJ)
  int inst;        // instance
  float thr, gamma;
  int pad[3];
};
static_assert(sizeof(TileRec) == 64, "TileRec is one 64-byte record");

// threads of a per-group statistics workgroup (k_group_stats and the L-BFGS
// update that forms the same statistics; both kernels of a handle use the
// same size, hence the same fixed-order reduction): GS_LARGE for handles
// whose groups average more than GS_SMALL rows, else GS_SMALL
constexpr int GS_SMALL = 256, GS_LARGE = 1024;

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// The four statistics of a group over a GT-thread workgroup in a fixed
// order (wavefront trees, then the wavefronts in order); the totals are
// valid in thread 0.  sm: [4][GT / 64] of LDS.
template <int GT>
__device__ __forceinline__ void gs_reduce(double& up, double& dn, double& am, double& ams, double (*sm)[GT / 64]) {
  up = wave_sum_dd(up);
  dn = wave_sum_dd(dn);
  am = wave_max_d(am);
  ams = wave_max_d(ams);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[0][w] = up;
    sm[1][w] = dn;
    sm[2][w] = am;
    sm[3][w] = ams;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    up = dn = am = ams = 0.0;
    for (int i = 0; i < GT / 64; ++i) {
      up += sm[0][i];
      dn += sm[1][i];
      am = fmax(am, sm[2][i]);
      ams = fmax(ams, sm[3][i]);
    }
  }
}

// Per-group statistics of the change since the snapshot, in float64.
struct GroupStats {
  double up;        // || [alpha - alpha~]_+ ||  over the group
  double dn;        // || [alpha - alpha~]_- ||
  double all;       // || alpha - alpha~ ||
  double amax;      // max |alpha_i| over the group (current point)
  double amax_s;    // max |alpha~_i| over the group (snapshot)
  double sg;        // sqrt(g_l)
  double fa, fb;    // rounding factors of the safe upper bound (see screen.hip)
};

// Device-side counters (int64, integer atomics only).
enum Counter {
  CNT_EVALS = 0, CNT_PAIRS_TOTAL, CNT_PAIRS_N, CNT_PAIRS_CHECKED, CNT_PAIRS_UNSKIPPED,
  CNT_REFRESH, CNT_TILES_TOTAL, CNT_TILES_COMPUTED, CNT_NUM
};

// per-instance evaluation mode, read on the device
enum EvalMode { EM_DENSE = 0, EM_SCREEN = 1, EM_SNAPSHOT = 2, EM_SKIP = 3 };

// pair state written by the screen / extraction kernels
enum PairFlag : uint8_t { PAIR_SKIP = 0, PAIR_CHECK = 1, PAIR_IN_N = 2 };

// position of internal cost entry (row r of the group starting at gs with gn
// rows, padded column c) in the tile-major pool
__host__ __device__ inline size_t c_index(const InstDev& I, int gs, int gn, int r, int c) {
  return (size_t)I.c_off + (size_t)gs * I.nt_pad + (size_t)(c / TJ) * gn * TJ +
         (size_t)(r - gs) * TJ + (size_t)(c % TJ);
}

// loads per lane (per virtual wavefront) of row bucket b: 2, then the
// multiples of RSTEP up to RMAX, then of RSTEP_BIG up to RBIG
__host__ __device__ constexpr int bucket_R(int b) {
  return b == 0 ? 2 : b <= RMAX / RSTEP ? RSTEP * b : RMAX + RSTEP_BIG * (b - RMAX / RSTEP);
}

// row bucket of a whole-group tile: the smallest bucket_R(b) with
// 2 NW R >= rows (two rows per load)
__host__ __device__ inline int row_bucket(int rows) {
  const int r = (rows + 2 * NW - 1) / (2 * NW);
  if (r <= 2) return 0;
  if (r <= RMAX) return (r + RSTEP - 1) / RSTEP;
  return RMAX / RSTEP + (r - RMAX + RSTEP_BIG - 1) / RSTEP_BIG;
}

// registers per lane holding the alpha values of a wavefront's 2 R K rows
__host__ __device__ constexpr int av_regs(int R, int K) { return (2 * R * K + WAVE - 1) / WAVE; }

// teams of a row bucket: K tiles per workgroup, NW / K wavefronts each
// (R K <= 16 keeps two workgroups per compute unit; a team keeps at least
// two wavefronts)
__host__ __device__ constexpr int bucket_K(int b) {
  return bucket_R(b) <= 16 && 16 % bucket_R(b) == 0 ? 16 / bucket_R(b) : 1;
}
static_assert(bucket_K(0) <= NW / 2, "teams of at least two wavefronts");

// on-the-fly tiles: bucket b < 5 holds whole groups of up to 32 << b rows,
// one per team of 1 << b wavefronts with one 32-row block each; bucket 5
// groups of up to 1024 rows, teams of 16 wavefronts with two blocks each
constexpr int OTF_NBUCKET = 6;
__host__ __device__ inline int otf_bucket(int rows) {
  int b = 0;
  while (b < 5 && rows > (32 << b)) ++b;
  return b;
}

}  // namespace otgs
