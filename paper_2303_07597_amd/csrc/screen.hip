// Safe screening (Sec. 3.2, Algorithm 2) and the extraction of the set N
// (Sec. 3.3, Algorithm 1) on the (group, target) blocks.
//
// Upper bound (Def. 1, Eq. 6): z_lj <= z~_lj + ||[alpha - alpha~]_+||_[l] +
// sqrt(g_l) [beta_j - beta~_j]_+ holds in exact arithmetic.  The gradient
// kernel however decides "zero block" on its float32 value of z, so a block
// is skipped only when a rigorous upper bound on that *computed* value is at
// most the float32 threshold fl(mu gamma).  With u = 2^-24, n_op the number
// of roundings on any path of the sum of squares, gam = n_op u / (1 - n_op u)
// and delta = 2.01 u (max_l |alpha| + |beta_j| + max C) the error bound of one
// computed f = (alpha + beta) - c:
//   zhat <= (1+2u) sqrt(1+gam) (z + sqrt(g) delta)                       (a)
//   z~   <= zhat~ / ((1-2u) sqrt(1-gam)) + sqrt(g) delta~                 (b)
// and with Eq. 6 in between,
//   UB = (1+2u) sqrt(1+gam) [zhat~/((1-2u) sqrt(1-gam)) + sqrt(g)(delta~ +
//        delta) + ||[dalpha_[l]]_+|| + sqrt(g)[dbeta_j]_+] (1 + 1e-9),
// evaluated in float64; skip iff UB <= fl(mu gamma).  A skipped block is then
// exactly zero in the dense evaluation too, which makes screened results
// bit-identical to dense ones.
//
// Lower bound (Def. 2, Eq. 7), used only to build N (blocks evaluated
// without a check, Lemma 5): z_low = k~ - ||dalpha_[l]|| - sqrt(g)|dbeta_j| -
// o~ - ||[dalpha_[l]]_-|| - sqrt(g)|[dbeta_j]_-| with k~ = sqrt(z~^2 + o~^2).
// Membership in N never changes a result (N blocks are always evaluated), so
// this bound needs no rounding margin.
#include "otgs_internal.h"

namespace otgs {

struct ScreenArgs {
  const InstDev* inst;
  const int* g_start;
  const int* g_size;
  const int* grp_inst;       // global group index -> instance
  const TileDesc* tiles_all; // every group tile; aux = row class, or -nchunks
  int n_tiles_all;
  const float* alpha;        // current point, internal order
  const float* beta;
  const float* alpha_s;      // snapshot
  const float* beta_s;
  const float* zsnap;
  const float* osnap;
  GroupStats* gstats;
  uint8_t* inN;              // per pair
  uint8_t* tile_on;          // per group tile
  TileDesc* list_main;
  TileDesc* list_sg;         // split group tiles (combine)
  TileDesc* list_sc;         // split chunk tiles
  int* counts;               // [3]: main, split groups, split chunks
  long long* counters;
  const int* inst_mode;      // EvalMode per instance
  int use_lower;             // build N at snapshot refreshes
};

// Per-group float64 statistics of alpha - alpha~ (and max |alpha|, |alpha~|);
// one block per nonempty group of every instance.  Block 0 also resets the
// work-list counts of the screen that follows.
__global__ void __launch_bounds__(256) k_group_stats(ScreenArgs A) {
  __shared__ double sm[5][256];
  const int gidx = blockIdx.x;
  const int k = A.grp_inst[gidx];
  const InstDev I = A.inst[k];
  const int ge = gidx - I.grp_off;
  const int r0 = A.g_start[gidx], n = A.g_size[gidx];
  double up = 0, dn = 0, am = 0, ams = 0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const int r = I.row_off + r0 + q;
    const double a = A.alpha[r], as = A.alpha_s[r];
    const double d = a - as;
    if (d > 0) up += d * d; else dn += d * d;
    am = fmax(am, fabs(a));
    ams = fmax(ams, fabs(as));
  }
  sm[0][threadIdx.x] = up; sm[1][threadIdx.x] = dn;
  sm[2][threadIdx.x] = am; sm[3][threadIdx.x] = ams;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + o];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + o];
      sm[2][threadIdx.x] = fmax(sm[2][threadIdx.x], sm[2][threadIdx.x + o]);
      sm[3][threadIdx.x] = fmax(sm[3][threadIdx.x], sm[3][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    GroupStats s;
    s.up = sqrt(sm[0][0]);
    s.dn = sqrt(sm[1][0]);
    s.all = sqrt(sm[0][0] + sm[1][0]);
    s.amax = sm[2][0];
    s.amax_s = sm[3][0];
    s.pad[0] = s.pad[1] = s.pad[2] = 0;
    A.gstats[gidx] = s;
    if (ge == 0) {
      const int m = A.inst_mode[k];
      if (m != EM_SKIP) atomicAdd((unsigned long long*)&A.counters[CNT_EVALS], 1ull);
      if (m == EM_SNAPSHOT) atomicAdd((unsigned long long*)&A.counters[CNT_REFRESH], 1ull);
    }
    if (gidx == 0) {
      A.counts[0] = 0;
      A.counts[1] = 0;
      A.counts[2] = 0;
    }
  }
}

__device__ __forceinline__ long long wave_popc(bool b) { return __popcll(__ballot(b)); }

// One wavefront per group tile (4 per block), one lane per target column.
// mode 1 (screen): classify every pair (in N / bound tested / skipped), mark
// the tile when any pair must be evaluated and append it to the work lists.
// mode 2 (extract): rebuild N from the lower bound; no lists.
__global__ void __launch_bounds__(256) k_screen_pairs(ScreenArgs A) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= A.n_tiles_all) return;
  const TileDesc d = A.tiles_all[t];
  const InstDev I = A.inst[d.inst];
  const int gidx = I.grp_off + d.grp;
  const GroupStats S = A.gstats[gidx];
  const int g = A.g_size[gidx];
  const int col = d.jb * TJ + lane;
  const bool valid = col < I.nt;
  const size_t pr = (size_t)I.pair_off + (size_t)d.grp * I.nt_pad + col;
  const double b = A.beta[I.col_off + col], bs = A.beta_s[I.col_off + col];
  const double db = b - bs;
  const double sg = sqrt((double)g);
  const double thr = (double)I.thr;

  const int mode = A.inst_mode[d.inst];
  if (mode == EM_SKIP) {
    if (lane == 0) A.tile_on[(size_t)I.tile_off + (size_t)d.grp * I.njb + d.jb] = 0;
    return;
  }
  if (mode == EM_SNAPSHOT && valid) {
    // Algorithm 1: rebuild N from the lower bound against the old snapshot
    uint8_t f = PAIR_SKIP;
    if (A.use_lower) {
      const double zt = A.zsnap[pr], ot = A.osnap[pr];
      const double kt = sqrt(zt * zt + ot * ot);
      const double zlow = kt - S.all - sg * fabs(db) - ot - S.dn - sg * (db < 0 ? -db : 0.0);
      if (zlow > thr) f = PAIR_IN_N;
    }
    A.inN[pr] = f;
  }
  const double u = 5.9604644775390625e-08;
  const int nch = (g + CHUNK - 1) / CHUNK;
  const double nop = (double)g + 17.0 * nch + 16.0;
  const double gam = nop * u / (1.0 - nop * u);
  const double cm = (double)I.cmax;
  const double del_s = 2.01 * u * (S.amax_s + fabs(bs) + cm);
  const double del_c = 2.01 * u * (S.amax + fabs(b) + cm);
  bool inN = false, checked = false, compute = false;
  if (valid) {
    if (mode != EM_SCREEN) {
      compute = true;               // dense evaluation (also at a snapshot)
    } else if (A.inN[pr] == PAIR_IN_N) {
      inN = true;
      compute = true;
    } else {
      checked = true;
      const double zt = A.zsnap[pr];
      const double ub = (1.0 + 2.0 * u) * sqrt(1.0 + gam) *
                        (zt / ((1.0 - 2.0 * u) * sqrt(1.0 - gam)) + sg * (del_s + del_c) + S.up +
                         sg * (db > 0 ? db : 0.0)) *
                        (1.0 + 1e-9);
      compute = !(ub <= thr);
    }
  }
  const unsigned long long on = __ballot(compute);
  const long long c_valid = wave_popc(valid), c_in = wave_popc(inN), c_chk = wave_popc(checked),
                  c_uns = wave_popc(checked && compute);
  if (lane == 0) {
    const size_t tix = (size_t)I.tile_off + (size_t)d.grp * I.njb + d.jb;
    A.tile_on[tix] = on ? 1 : 0;
    atomicAdd((unsigned long long*)&A.counters[CNT_PAIRS_TOTAL], (unsigned long long)c_valid);
    if (c_in) atomicAdd((unsigned long long*)&A.counters[CNT_PAIRS_N], (unsigned long long)c_in);
    if (c_chk)
      atomicAdd((unsigned long long*)&A.counters[CNT_PAIRS_CHECKED], (unsigned long long)c_chk);
    if (c_uns)
      atomicAdd((unsigned long long*)&A.counters[CNT_PAIRS_UNSKIPPED], (unsigned long long)c_uns);
    atomicAdd((unsigned long long*)&A.counters[CNT_TILES_TOTAL], 1ull);
    if (on) {
      atomicAdd((unsigned long long*)&A.counters[CNT_TILES_COMPUTED], 1ull);
      if (d.aux >= 0) {
        const int pos = atomicAdd(&A.counts[0], 1);
        A.list_main[pos] = d;
      } else {
        const int pos = atomicAdd(&A.counts[1], 1);
        TileDesc e = d;
        e.aux = 0;
        A.list_sg[pos] = e;
        const int n = -d.aux;
        const int pc = atomicAdd(&A.counts[2], n);
        for (int c = 0; c < n; ++c) {
          e.aux = c;
          A.list_sc[pc + c] = e;
        }
      }
    }
  }
}

// alpha~ <- alpha, beta~ <- beta for the instances evaluated at a snapshot;
// grid (blocks, count)
__global__ void k_snapshot_copy(const InstDev* __restrict__ inst, const int* __restrict__ inst_mode,
                                const float* __restrict__ a, float* __restrict__ as,
                                const float* __restrict__ b, float* __restrict__ bs) {
  const int k = blockIdx.y;
  if (inst_mode[k] != EM_SNAPSHOT) return;
  const InstDev I = inst[k];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < I.ns + I.nt_pad; e += gridDim.x * blockDim.x) {
    if (e < I.ns) as[I.row_off + e] = a[I.row_off + e];
    else bs[I.col_off + e - I.ns] = b[I.col_off + e - I.ns];
  }
}

// every instance gets the same evaluation mode
__global__ void k_fill_mode(int* inst_mode, int count, int mode) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x)
    inst_mode[k] = mode;
}

// integer counter update from the device (no host round trip)
__global__ void k_count_add(long long* counters, int which, long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    atomicAdd((unsigned long long*)&counters[which], (unsigned long long)v);
}

}  // namespace otgs
