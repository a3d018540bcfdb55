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
  TileDesc* list_main;       // whole-group tiles, bucket b at main_off[b]
  const TileRec* rec_all;    // records of every tile (materialized cost; else null)
  TileRec* rec_dyn;          // records of list_main's entries
  TileDesc* list_sg;         // split group tiles (combine)
  TileDesc* list_sc;         // split chunk tiles
  int* counts;               // [NBUCKET + 2]: per bucket, split groups, split chunks
  int main_off[NBUCKET];
  long long* counters;
  long long* block_counters; // [screen blocks][CNT_NUM]
  const int* inst_mode;      // EvalMode per instance
  int use_lower;             // build N at snapshot refreshes
};

// Per-group float64 statistics of alpha - alpha~ (and max |alpha|, |alpha~|);
// one block per nonempty group of every instance.  Block 0 also resets the
// work-list counts of the screen that follows.
template <int GT>
__global__ void __launch_bounds__(GT) k_group_stats(ScreenArgs A) {
  __shared__ double sm[4][GT / 64];
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
  gs_reduce<GT>(up, dn, am, ams, sm);
  if (threadIdx.x == 0) {
    GroupStats s;
    s.up = sqrt(up);
    s.dn = sqrt(dn);
    s.all = sqrt(up + dn);
    s.amax = am;
    s.amax_s = ams;
    // per-group constants of the rounding-safe upper bound
    screen_group_consts(n, s.sg, s.fa, s.fb);
    A.gstats[gidx] = s;
    if (ge == 0) {
      const int m = A.inst_mode[k];
      if (m != EM_SKIP) atomicAdd((unsigned long long*)&A.counters[CNT_EVALS], 1ull);
      if (m == EM_SNAPSHOT) atomicAdd((unsigned long long*)&A.counters[CNT_REFRESH], 1ull);
    }
    if (gidx == 0)
      for (int q = 0; q < NBUCKET + 2; ++q) A.counts[q] = 0;
  }
}

constexpr int SCREEN_TILES = 16;   // group tiles (wavefronts) per screen block


constexpr int SCREEN_TPB = 2 * SCREEN_TILES;   // group tiles per screen block
static_assert(SCREEN_TPB <= WAVE && NBUCKET + 2 <= WAVE, "the block tally uses one lane per slot");

// One half wavefront per group tile (SCREEN_TPB per block: only 32 lanes of
// a tile have a column), one lane per target column.  SCREEN: classify
// every pair (in N / bound tested / skipped), mark the tile when any pair
// must be evaluated.  SNAPSHOT: rebuild N from the lower bound, then
// evaluate densely.  DENSE: every tile.  SKIP: nothing.  Active tiles are
// appended to the work lists; counters and list positions are aggregated
// per block so each block issues one atomic per quantity.
__global__ void __launch_bounds__(SCREEN_TILES * 64) k_screen_pairs(ScreenArgs A) {
  __shared__ int s_cnt[SCREEN_TPB][8];   // valid, inN, checked, unskipped, main, split,
                                         // chunks of an active split tile, tile counted
  __shared__ int s_bkt[SCREEN_TPB];
  __shared__ int s_base[NBUCKET + 2];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x >> 6;
  const int half = lane >> 5, c = lane & (TJ - 1);
  const int slot = 2 * wv + half;   // the tile's slot in the block
  const int t = blockIdx.x * SCREEN_TPB + slot;
  const bool tile_ok = t < A.n_tiles_all;
  TileDesc d{0, 0, 0, 0};
  if (tile_ok) d = A.tiles_all[t];
  // the tile's 64-byte record, 16 bytes per lane on lanes 0..3 of the half,
  // fetched now so that the list write below waits on no further load
  int4 rq{0, 0, 0, 0};
  const bool rec_lane = A.rec_all != nullptr && tile_ok && c < 4;
  if (rec_lane) rq = reinterpret_cast<const int4*>(A.rec_all + t)[c];
  int mode = EM_SKIP, tile_off = 0, njb = 0;
  bool valid = false, inN = false, checked = false, compute = false;
  if (tile_ok) {
    const InstDev* Ip = A.inst + d.inst;
    const int grp_off = Ip->grp_off, nt = Ip->nt, pair_off = Ip->pair_off;
    const int nt_pad = Ip->nt_pad, col_off = Ip->col_off;
    const float ithr = Ip->thr, cmax = Ip->cmax;
    tile_off = Ip->tile_off;
    njb = Ip->njb;
    mode = A.inst_mode[d.inst];
    const int gidx = grp_off + d.grp;
    const int col = d.jb * TJ + c;
    valid = col < nt && mode != EM_SKIP;
    const size_t pr = (size_t)pair_off + (size_t)d.grp * nt_pad + col;
    if (valid) {
      const GroupStats* Sp = A.gstats + gidx;
      const double b = A.beta[col_off + col], bs = A.beta_s[col_off + col];
      const double sg = Sp->sg;
      const double thr = (double)ithr;
      if (mode == EM_SNAPSHOT) {
        // Algorithm 1: rebuild N from the lower bound against the old snapshot
        uint8_t f = PAIR_SKIP;
        if (A.use_lower && screen_lower(A.zsnap[pr], A.osnap[pr], b, bs, Sp->all, Sp->dn, sg) > thr)
          f = PAIR_IN_N;
        A.inN[pr] = f;
        compute = true;
      } else if (mode == EM_DENSE) {
        compute = true;
      } else {
        // flag and snapshot norm loaded together (one round trip)
        const uint8_t f = A.inN[pr];
        const float zs = A.zsnap[pr];
        if (f == PAIR_IN_N) {
          inN = true;
          compute = true;
        } else {
          checked = true;
          const double ub = screen_upper(zs, b, bs, Sp->up, Sp->amax, Sp->amax_s, sg, Sp->fa, Sp->fb,
                                         (double)cmax);
          compute = !(ub <= thr);
        }
      }
    }
  }
  // per-half tallies
  const int sh = 32 * half;
  auto halfcount = [&](bool x) { return __popcll((__ballot(x) >> sh) & 0xffffffffull); };
  const int c_valid = halfcount(valid), c_in = halfcount(inN), c_chk = halfcount(checked);
  const int c_uns = halfcount(checked && compute);
  const bool on = tile_ok && halfcount(compute) != 0;
  if (c == 0) {
    if (tile_ok) A.tile_on[(size_t)tile_off + (size_t)d.grp * njb + d.jb] = on ? 1 : 0;
    s_cnt[slot][0] = c_valid;
    s_cnt[slot][1] = c_in;
    s_cnt[slot][2] = c_chk;
    s_cnt[slot][3] = c_uns;
    s_cnt[slot][4] = (on && d.aux >= 0) ? 1 : 0;
    s_cnt[slot][5] = (on && d.aux < 0) ? 1 : 0;
    s_cnt[slot][6] = (on && d.aux < 0) ? -d.aux : 0;
    s_cnt[slot][7] = (tile_ok && mode != EM_SKIP) ? 1 : 0;
    s_bkt[slot] = d.aux >= 0 ? d.aux : 0;
  }
  __syncthreads();
  // Block tally by wavefront 0, lane l standing for slot l: per-bucket
  // counts and each slot's rank by ballots, split offsets by wavefront
  // sums, one atomic per quantity (issued by different lanes together)
  if (wv == 0) {
    const bool has = lane < SCREEN_TPB;
    const int m4 = has ? s_cnt[lane][4] : 0, m5 = has ? s_cnt[lane][5] : 0;
    const int m6 = has ? s_cnt[lane][6] : 0, bk = has ? s_bkt[lane] : 0;
    const unsigned long long below = (1ull << lane) - 1ull;
    int rank = 0, nb_mine = 0;   // lane q < NBUCKET: tiles of bucket q in the block
#pragma unroll
    for (int q = 0; q < NBUCKET; ++q) {
      const unsigned long long bq = __ballot(m4 && bk == q);
      if (bk == q) rank = __popcll(bq & below);
      if (lane == q) nb_mine = __popcll(bq);
    }
    // exclusive prefixes of split tiles and chunks over the slots
    int ps = m5, pc = m6;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int ys = __shfl_up(ps, o), yc = __shfl_up(pc, o);
      if (lane >= o) {
        ps += ys;
        pc += yc;
      }
    }
    const int nsg = __shfl(ps, WAVE - 1), nsc = __shfl(pc, WAVE - 1);
    ps -= m5;
    pc -= m6;
    // list bases: lane q < NBUCKET for bucket q, NBUCKET split groups,
    // NBUCKET + 1 split chunks
    int base = 0;
    if (lane < NBUCKET && nb_mine) base = atomicAdd(&A.counts[lane], nb_mine);
    if (lane == NBUCKET && nsg) base = atomicAdd(&A.counts[NBUCKET], nsg);
    if (lane == NBUCKET + 1 && nsc) base = atomicAdd(&A.counts[NBUCKET + 1], nsc);
    if (lane < NBUCKET + 2) s_base[lane] = base;
    if (has) {
      s_cnt[lane][4] = rank;   // reused: position within the block's bucket
      s_cnt[lane][5] = ps;     // split group position within the block
      s_cnt[lane][6] = pc;     // split chunk position within the block
    }
    // counters: every block owns a slot (evaluations are ordered on the
    // stream, so a plain update suffices); slots are summed on request
    long long tq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      long long v = has ? s_cnt[lane][q] : 0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      tq[q] = v;
    }
    int nt_ = has ? s_cnt[lane][7] : 0, non = m4 + m5;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      nt_ += __shfl_xor(nt_, o);
      non += __shfl_xor(non, o);
    }
    if (lane == 0) {
      long long* C = A.block_counters + (size_t)blockIdx.x * CNT_NUM;
      C[CNT_PAIRS_TOTAL] += tq[0];
      C[CNT_PAIRS_N] += tq[1];
      C[CNT_PAIRS_CHECKED] += tq[2];
      C[CNT_PAIRS_UNSKIPPED] += tq[3];
      C[CNT_TILES_TOTAL] += nt_;
      C[CNT_TILES_COMPUTED] += non;
    }
  }
  __syncthreads();
  // list entries in tile order within the block
  if (on && d.aux >= 0 && (c == 0 || rec_lane)) {
    // the bucket's list offset (unrolled select: a kernel-argument array
    // indexed at run time would be copied to private memory)
    int moff = 0;
#pragma unroll
    for (int q = 0; q < NBUCKET; ++q)
      if (q == d.aux) moff = A.main_off[q];
    const int pm = s_base[d.aux] + s_cnt[slot][4];
    if (c == 0) A.list_main[moff + pm] = d;
    if (rec_lane) reinterpret_cast<int4*>(A.rec_dyn + moff + pm)[c] = rq;
  }
  if (c == 0 && on) {
    if (d.aux < 0) {
      const int ps = s_base[NBUCKET] + s_cnt[slot][5], pc = s_base[NBUCKET + 1] + s_cnt[slot][6];
      TileDesc e = d;
      e.aux = 0;
      A.list_sg[ps] = e;
      for (int q = 0; q < -d.aux; ++q) {
        e.aux = q;
        A.list_sc[pc + q] = e;
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
