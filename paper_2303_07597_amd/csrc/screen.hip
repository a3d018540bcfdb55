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
  const float* cmax_w;       // per instance max |c| of a re-centred cost (NULL: InstDev cmax)
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

constexpr int SCREEN_TILES = 16;   // wavefronts per screen block
constexpr int SCREEN_TPB = 2 * SCREEN_TILES;   // group tiles per pass of a screen block
static_assert(SCREEN_TPB <= WAVE && NBUCKET + 2 <= WAVE, "the block tally uses one lane per slot");
constexpr int SCREEN_WIDE_BLOCKS = 1024;  // single-pass grids above this many blocks take two passes

// One half wavefront per group tile (SCREEN_TPB tiles per pass, TPH passes
// per block: only 32 lanes of a tile have a column), one lane per target
// column.  SCREEN: classify every pair (in N / bound tested / skipped), mark
// the tile when any pair must be evaluated.  SNAPSHOT: rebuild N from the
// lower bound, then evaluate densely.  DENSE: every tile.  SKIP: nothing.
// Active tiles are appended to the work lists; counters and list positions
// are aggregated per block so each block issues one atomic per quantity.
// More passes per block amortise the block's fixed latency (descriptor
// fetch, list atomics, barriers, list writes) over more tiles and put fewer
// atomics on the shared list counts; a single pass keeps small grids wide.
template <int TPH>
__global__ void __launch_bounds__(SCREEN_TILES * 64) k_screen_pairs(ScreenArgs A) {
  constexpr int NE = SCREEN_TPB * TPH;        // tiles of the block; entry i * SCREEN_TPB + slot
  constexpr int NP = (NE + WAVE - 1) / WAVE;  // tally passes of wavefront 0
  __shared__ int s_cnt[NE][8];   // valid, inN, checked, unskipped, main, split,
                                 // chunks of an active split tile, tile counted
  __shared__ int s_bkt[NE];
  __shared__ int s_base[NBUCKET + 2];
  __shared__ int4 s_rec[TPH > 1 ? NE : 1][4];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x >> 6;
  const int half = lane >> 5, c = lane & (TJ - 1);
  const int slot = 2 * wv + half;   // the tile's slot in a pass
  const int tb = blockIdx.x * NE + slot;
  // descriptors of every pass, and each tile's 64-byte record (16 bytes per
  // lane on lanes 0..3 of the half), fetched first so that neither the
  // passes nor the list write below wait on them
  TileDesc dd[TPH];
  int4 rq[TPH];
  const bool rec_lane = A.rec_all != nullptr && c < 4;
#pragma unroll
  for (int i = 0; i < TPH; ++i) {
    const int t = tb + i * SCREEN_TPB;
    dd[i] = TileDesc{0, 0, 0, 0};
    rq[i] = int4{0, 0, 0, 0};
    if (t < A.n_tiles_all) {
      dd[i] = A.tiles_all[t];
      if (rec_lane) rq[i] = reinterpret_cast<const int4*>(A.rec_all + t)[c];
    }
  }
  // with several passes the records wait in LDS (registers stay free)
  if (TPH > 1 && rec_lane) {
#pragma unroll
    for (int i = 0; i < TPH; ++i) s_rec[i * SCREEN_TPB + slot][c] = rq[i];
  }
  bool onv[TPH];
  const int sh = 32 * half;
  auto halfcount = [&](bool x) { return __popcll((__ballot(x) >> sh) & 0xffffffffull); };
#pragma unroll
  for (int i = 0; i < TPH; ++i) {
    const int t = tb + i * SCREEN_TPB;
    const bool tile_ok = t < A.n_tiles_all;
    const TileDesc d = dd[i];
    int mode = EM_SKIP, tile_off = 0, njb = 0;
    bool valid = false, inN = false, checked = false, compute = false;
    if (tile_ok) {
      const InstDev* Ip = A.inst + d.inst;
      const int grp_off = Ip->grp_off, nt = Ip->nt, pair_off = Ip->pair_off;
      const int nt_pad = Ip->nt_pad, col_off = Ip->col_off;
      const float ithr = Ip->thr, cmax = A.cmax_w ? A.cmax_w[d.inst] : Ip->cmax;
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
    const int c_valid = halfcount(valid), c_in = halfcount(inN), c_chk = halfcount(checked);
    const int c_uns = halfcount(checked && compute);
    const bool on = tile_ok && halfcount(compute) != 0;
    onv[i] = on;
    if (c == 0) {
      if (tile_ok) A.tile_on[(size_t)tile_off + (size_t)d.grp * njb + d.jb] = on ? 1 : 0;
      int* sc = s_cnt[i * SCREEN_TPB + slot];
      sc[0] = c_valid;
      sc[1] = c_in;
      sc[2] = c_chk;
      sc[3] = c_uns;
      sc[4] = (on && d.aux >= 0) ? 1 : 0;
      sc[5] = (on && d.aux < 0) ? 1 : 0;
      sc[6] = (on && d.aux < 0) ? -d.aux : 0;
      sc[7] = (tile_ok && mode != EM_SKIP) ? 1 : 0;
      s_bkt[i * SCREEN_TPB + slot] = d.aux >= 0 ? d.aux : 0;
    }
  }
  __syncthreads();
  // Block tally by wavefront 0, lane l standing for entries l, l + 64, ...:
  // per-bucket counts and each entry's rank by ballots, split offsets by
  // wavefront sums, one atomic per quantity (issued by different lanes
  // together)
  if (wv == 0) {
    const unsigned long long below = (1ull << lane) - 1ull;
    int cntq[NBUCKET];   // wavefront-uniform running count per bucket
#pragma unroll
    for (int q = 0; q < NBUCKET; ++q) cntq[q] = 0;
    int nsg = 0, nsc = 0, nt_ = 0, non = 0;
    long long tq[4] = {0, 0, 0, 0};
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int e = p * WAVE + lane;
      const bool has = e < NE;
      const int m4 = has ? s_cnt[e][4] : 0, m5 = has ? s_cnt[e][5] : 0;
      const int m6 = has ? s_cnt[e][6] : 0, bk = has ? s_bkt[e] : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) tq[q] += has ? s_cnt[e][q] : 0;
      nt_ += has ? s_cnt[e][7] : 0;
      non += m4 + m5;
      int rank = 0;
#pragma unroll
      for (int q = 0; q < NBUCKET; ++q) {
        const unsigned long long bq = __ballot(m4 && bk == q);
        if (bk == q) rank = cntq[q] + __popcll(bq & below);
        cntq[q] += __popcll(bq);
      }
      // exclusive prefixes of split tiles and chunks over the entries
      int ps = m5, pc = m6;
#pragma unroll
      for (int o = 1; o < WAVE; o <<= 1) {
        const int ys = __shfl_up(ps, o), yc = __shfl_up(pc, o);
        if (lane >= o) {
          ps += ys;
          pc += yc;
        }
      }
      const int ts = __shfl(ps, WAVE - 1), tc = __shfl(pc, WAVE - 1);
      if (has) {
        s_cnt[e][4] = rank;            // reused: position within the block's bucket
        s_cnt[e][5] = nsg + ps - m5;   // split group position within the block
        s_cnt[e][6] = nsc + pc - m6;   // split chunk position within the block
      }
      nsg += ts;
      nsc += tc;
    }
    int nb_mine = 0;   // lane q < NBUCKET: tiles of bucket q in the block
#pragma unroll
    for (int q = 0; q < NBUCKET; ++q)
      if (lane == q) nb_mine = cntq[q];
    // list bases: lane q < NBUCKET for bucket q, NBUCKET split groups,
    // NBUCKET + 1 split chunks
    int base = 0;
    if (lane < NBUCKET && nb_mine) base = atomicAdd(&A.counts[lane], nb_mine);
    if (lane == NBUCKET && nsg) base = atomicAdd(&A.counts[NBUCKET], nsg);
    if (lane == NBUCKET + 1 && nsc) base = atomicAdd(&A.counts[NBUCKET + 1], nsc);
    if (lane < NBUCKET + 2) s_base[lane] = base;
    // counters: every block owns a slot (evaluations are ordered on the
    // stream, so a plain update suffices); slots are summed on request
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
      for (int q = 0; q < 4; ++q) tq[q] += __shfl_xor(tq[q], o);
      nt_ += __shfl_xor(nt_, o);
      non += __shfl_xor(non, o);
    }
    // (nothing to add, e.g. every tile of an instance whose solve has ended:
    // no read-modify-write)
    if (lane == 0 && (tq[0] | tq[1] | tq[2] | tq[3] | (long long)nt_ | (long long)non) != 0) {
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
  // list entries in entry order within the block
#pragma unroll
  for (int i = 0; i < TPH; ++i) {
    const TileDesc d = dd[i];
    const int e = i * SCREEN_TPB + slot;
    if (!onv[i]) continue;
    if (d.aux >= 0) {
      if (c == 0 || rec_lane) {
        // the bucket's list offset (unrolled select: a kernel-argument array
        // indexed at run time would be copied to private memory)
        int moff = 0;
#pragma unroll
        for (int q = 0; q < NBUCKET; ++q)
          if (q == d.aux) moff = A.main_off[q];
        const int pm = s_base[d.aux] + s_cnt[e][4];
        if (c == 0) A.list_main[moff + pm] = d;
        if (rec_lane) reinterpret_cast<int4*>(A.rec_dyn + moff + pm)[c] = TPH > 1 ? s_rec[e][c] : rq[0];
      }
    } else if (c == 0) {
      const int ps = s_base[NBUCKET] + s_cnt[e][5], pc = s_base[NBUCKET + 1] + s_cnt[e][6];
      TileDesc f = d;
      f.aux = 0;
      A.list_sg[ps] = f;
      for (int q = 0; q < -d.aux; ++q) {
        f.aux = q;
        A.list_sc[pc + q] = f;
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
