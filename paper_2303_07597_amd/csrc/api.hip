// Host side of libotgs: the handle, its device layout, and the C ABI of
// include/otgs.h.  All device work is enqueued on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "otgs_internal.h"
#include "../../include/otgs.h"

namespace otgs {

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess)                                                           \
      return fail(OT_GS_EDEVICE, "%s failed: %s (%s:%d)", #x, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                              \
  } while (0)

#define LAUNCHCHK()                                                                 \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess)                                                           \
      return fail(OT_GS_EDEVICE, "kernel launch failed: %s (%s:%d)",               \
                  hipGetErrorString(e_), __FILE__, __LINE__);                       \
  } while (0)

static inline long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

struct InstHost {
  InstDev d;
  int cost_mode;
  std::vector<int> g_size, g_start, g_chunk0, g_xblk, g_label;
  int n_chunk_rows;
};

// kernel ids of the timing facility
enum { KT_GRAD = 0, KT_SCREEN, KT_REDUCE, KT_LBFGS, KT_NUM };

struct Timing {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[KT_NUM];
  double ms[KT_NUM] = {0, 0, 0, 0};
  long long n[KT_NUM] = {0, 0, 0, 0};
};

}  // namespace otgs

using namespace otgs;

struct ot_gs_handle {
  int count = 0;
  std::vector<InstHost> inst;
  std::vector<void*> allocs;
  // totals
  long long tot_rows = 0, tot_cols = 0, tot_cols_pad = 0, tot_groups = 0, tot_pairs = 0,
            tot_tiles = 0, tot_c = 0, tot_r = 0, tot_chunk = 0, tot_x = 0, tot_y = 0;
  int n_main = 0, n_sg = 0, n_sc = 0;
  int n_bucket[NBUCKET] = {};
  int main_off[NBUCKET] = {};
  int dev = 0, n_cu = 256;
  // device arrays
  InstDev* d_inst = nullptr;
  int *perm_row = nullptr, *row_grp = nullptr, *perm_col = nullptr;
  int *row_map = nullptr, *col_map = nullptr;   // caller-order index of each internal row / column
  int* mode_dense = nullptr;                     // [count] EM_DENSE (dense evaluations of caller-order duals)
  int *g_start = nullptr, *g_size = nullptr, *g_chunk0 = nullptr, *grp_inst = nullptr;
  float* C = nullptr;
  // the pool the evaluations read and the cost bound of the screen margins:
  // C and InstDev cmax, or during a re-centred solve the reduced pool Cw and
  // its per-instance bounds cmax_w
  const float* C_eval = nullptr;
  const float* cmax_eval = nullptr;
  float* Cw = nullptr;
  float* cmax_w = nullptr;
  long long c_pool = 0;   // floats of the pool, padding rows included
  char* csr_scratch = nullptr;   // plan_csr's scratch, reserved in a workspace
  // on-the-fly cost: packed features and squared norms, per-group block offsets
  bool onthefly = false;
  int otf_dpmax = 16;   // largest padded feature count of the instances
  float *Xp = nullptr, *Yp = nullptr, *xn = nullptr, *yn = nullptr;
  int* g_xblk = nullptr;
  int* g_label = nullptr;          // label of each nonempty group
  long long* lab_pair_off = nullptr;   // [count] offsets of the caller-layout pair arrays
  long long tot_lab_pairs = 0;     // sum of n_groups * n_tgt
  // verification buffers (allocated by the first verified evaluation)
  struct Verify {
    float *ga = nullptr, *gb = nullptr;
    double* obj = nullptr;
    long long* cnt = nullptr;
    int* modes = nullptr;
    unsigned long long* diff = nullptr;
    double* objp = nullptr;   // assembly partials of D (verified solves)
  } ver;
  float *a_int = nullptr, *b_int = nullptr;
  float *a_cal = nullptr, *b_cal = nullptr;   // the marginals in the caller's order
  // dense ot_gs_dual_grad of a materialised cost: 1 the tiles read the
  // caller's duals through the index maps (no gather launch), 0 a gather
  // then the internal order; -1 by size (the maps' index loads cost more
  // than the gather saves once the cost pool is large); the autotuner sets it
  // from measurement
  int dense_direct = -1;
  // the caller's duals of the ot_gs_dual_grad call in progress (NULL outside one)
  const float *cal_alpha = nullptr, *cal_beta = nullptr;
  int *a_uniform = nullptr, *b_uniform = nullptr;
  std::vector<int> w_unit_h;   // per instance: every variable scale is 1 (uniform a, b and n_src = n_tgt)
  float *alpha = nullptr, *beta = nullptr, *ga = nullptr, *gb = nullptr;
  float *alpha_s = nullptr, *beta_s = nullptr, *zsnap = nullptr, *osnap = nullptr;
  float *rowpart = nullptr, *colsum = nullptr, *part = nullptr, *kappa = nullptr;
  float* excess = nullptr;
  double* obj = nullptr;
  GroupStats* gstats = nullptr;
  uint8_t *inN = nullptr, *tile_on = nullptr;
  TileDesc *tiles_all = nullptr, *list_main = nullptr, *list_sg = nullptr, *list_sc = nullptr;
  TileDesc *dyn_main = nullptr, *dyn_sg = nullptr, *dyn_sc = nullptr;
  // records of the whole-group materialized tiles: every tile (tiles_all
  // order), the static main list and the dynamic main list (screen output)
  TileRec *rec_all = nullptr, *rec_main = nullptr, *rec_dyn = nullptr;
  // screened solves: the update kernel forms the next evaluation's group
  // statistics (every group at most CHUNK rows)
  bool upd_stats = false;
  int max_le = 1;                // most nonempty groups of an instance
  bool gs_large = false;         // group-statistics workgroups of GS_LARGE threads
  int* counts_static = nullptr;  // [NBUCKET + 2]
  int* counts_dyn = nullptr;     // [NBUCKET + 2]
  long long* counters = nullptr;
  long long* block_counters = nullptr;  // [screen blocks][CNT_NUM]
  int n_screen_blocks = 0;
  int* err = nullptr;
  long long* t_off = nullptr;    // plan offsets
  int* inst_mode = nullptr;      // EvalMode per instance (device)
  long long tot_pairs_valid = 0; // sum of Le * nt
  int max_ns = 1, max_ntp = 64;
  int n_asm = 1;                 // assembly blocks per instance
  double* obj_part = nullptr;    // [count][n_asm]
  unsigned int* asm_done = nullptr;   // [count] assembly blocks finished (finalising evaluations)
  // solver buffers (allocated by the first solve)
  struct Solver {
    int hist = 0, maxb = 0, ndot = 0, cap_hist = 0;
    long long vtot = 0;
    long long* voff = nullptr;
    float *X = nullptr, *G = nullptr, *Dv = nullptr, *S = nullptr, *Y = nullptr, *W = nullptr;
    int* w_unit = nullptr;   // [count]: every scale of the instance is 1 (loads of W skipped)
    LbState* st = nullptr;
    AgdState* agd_st = nullptr;   // accelerated-ascent solves
    double* gram = nullptr;
    double* part = nullptr;
    int* n_active = nullptr;  // [2]: instances still running (or waiting), re-centrings asked for
    int* h_active = nullptr;  // pinned host [2]
    double* xref = nullptr;   // re-centring reference, actual variables
    double* obj_const = nullptr;
    // the buffers hold the state an L-BFGS solve left (a resumable state);
    // the working cost copy holds that state's re-centred cost; some
    // instance of the state was re-centred (xref != 0)
    bool lb_valid = false, cw_valid = false, xref_used = false;
    std::vector<void*> mem;
  } sol;
  Timing timing;
  bool has_snapshot = false;
  hipStream_t cap_stream = nullptr;   // stream that records solver steps into a graph
  // tile configuration (autotuned or set): per bucket of the tile lists the
  // team-shape variant (on-the-fly) and the grid multiplier (workgroups per
  // resident slot); index NBUCKET: the split-group passes
  int tile_var[NBUCKET + 1] = {};
  int tile_gm[NBUCKET + 1] = {};   // set to 2 at create

  // Device memory.  Without a caller workspace every buffer is a hipMalloc;
  // with one (ot_gs_create_ws) buffers are carved from it: those kept by the
  // handle from the bottom, set-up temporaries from the top (released at the
  // end of create).  The ledger counts the aligned bytes either way, which is
  // what ot_gs_workspace_size reports.
  char* ws_base = nullptr;
  size_t ws_size = 0, ws_lo = 0, ws_hi = 0;
  size_t led_persist = 0, led_temp = 0, led_temp_peak = 0;
  static size_t aligned(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~(size_t)255; }
  int dev_alloc(void** p, size_t bytes, bool temp) {
    const size_t a = aligned(bytes);
    if (temp) {
      led_temp += a;
      led_temp_peak = std::max(led_temp_peak, led_temp);
    } else {
      led_persist += a;
    }
    if (ws_base) {
      if (ws_hi - ws_lo < a)
        return fail(OT_GS_ENOMEM, "the workspace (%zu bytes) is too small; ot_gs_workspace_size gives the size",
                    ws_size);
      if (temp) {
        ws_hi -= a;
        *p = ws_base + ws_hi;
      } else {
        *p = ws_base + ws_lo;
        ws_lo += a;
      }
      return OT_GS_OK;
    }
    const hipError_t e = hipMalloc(p, a);
    if (e != hipSuccess) return fail(OT_GS_ENOMEM, "hipMalloc(%zu) failed: %s", a, hipGetErrorString(e));
    if (!temp) allocs.push_back(*p);
    return OT_GS_OK;
  }
  template <class T>
  int alloc(T** p, size_t n) {
    return dev_alloc((void**)p, std::max<size_t>(n, 1) * sizeof(T), false);
  }
  template <class T>
  int alloc_temp(T** p, size_t n) {
    return dev_alloc((void**)p, std::max<size_t>(n, 1) * sizeof(T), true);
  }
  // set-up temporaries (LIFO): in a workspace the top region comes back
  void free_temp(void* p, size_t bytes) {
    led_temp -= aligned(bytes);
    if (ws_base) ws_hi += aligned(bytes);
    else (void)hipFree(p);
  }
  void free_solver() {
    if (!ws_base)
      for (void* p : sol.mem) (void)hipFree(p);
    if (sol.h_active) (void)hipHostFree(sol.h_active);
    sol = Solver();
  }
  ~ot_gs_handle() {
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    free_solver();
    for (void* p : allocs) (void)hipFree(p);
    for (auto& v : timing.ev)
      for (auto& e : v) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  }
};

#define TRY(x)                 \
  do {                         \
    int rc_ = (x);             \
    if (rc_ != OT_GS_OK) return rc_; \
  } while (0)

// ------------------------------------------------------------ timing helpers

static int tbegin(ot_gs_handle* h, int which, hipStream_t s, hipEvent_t* ev) {
  if (!h->timing.on) return OT_GS_OK;
  HIPCHK(hipEventCreate(ev));
  HIPCHK(hipEventRecord(*ev, s));
  (void)which;
  return OT_GS_OK;
}
static int tend(ot_gs_handle* h, int which, hipStream_t s, hipEvent_t ev0) {
  if (!h->timing.on) return OT_GS_OK;
  hipEvent_t ev1;
  HIPCHK(hipEventCreate(&ev1));
  HIPCHK(hipEventRecord(ev1, s));
  h->timing.ev[which].push_back({ev0, ev1});
  return OT_GS_OK;
}

// ------------------------------------------------------------ create

static int sync_err(ot_gs_handle* h, hipStream_t s, int* out) {
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(out, h->err, sizeof(int), hipMemcpyDeviceToHost));
  return OT_GS_OK;
}

// error flag bits raised by kernels after set-up
constexpr int ERR_NONFINITE = 8;   // a NaN or Inf dual value met by the gather

static int clear_err(ot_gs_handle* h, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, h->err, 1LL, 0);
  LAUNCHCHK();
  return OT_GS_OK;
}

// buffers of checked and verified evaluations: two sets of caller-order
// gradients and objectives, saved counters and modes, a difference count
static int ensure_verify(ot_gs_handle* h) {
  auto& V = h->ver;
  if (V.ga) return OT_GS_OK;
  TRY(h->alloc(&V.ga, 2 * h->tot_rows));
  TRY(h->alloc(&V.gb, 2 * h->tot_cols_pad));
  TRY(h->alloc(&V.obj, 2 * (size_t)h->count));
  TRY(h->alloc(&V.cnt, CNT_NUM));
  TRY(h->alloc(&V.modes, h->count));
  TRY(h->alloc(&V.diff, 1));
  TRY(h->alloc(&V.objp, (size_t)h->count * h->n_asm));
  return OT_GS_OK;
}

// Synchronised report of a checked evaluation: ENUMERIC for a NaN or Inf
// input or objective, EVERIFY when the verified screened and dense
// evaluations differ.  Clears the error flags it reports.
static int check_report(ot_gs_handle* h, hipStream_t s, bool verify) {
  int herr = 0;
  std::vector<double> D(h->count);
  unsigned long long diff = 0;
  HIPCHK(hipMemcpyAsync(D.data(), h->ver.obj, sizeof(double) * h->count, hipMemcpyDeviceToHost, s));
  if (verify) HIPCHK(hipMemcpyAsync(&diff, h->ver.diff, sizeof diff, hipMemcpyDeviceToHost, s));
  TRY(sync_err(h, s, &herr));
  TRY(clear_err(h, s));
  HIPCHK(hipStreamSynchronize(s));
  if (herr & ERR_NONFINITE) return fail(OT_GS_ENUMERIC, "dual_grad: alpha or beta holds a NaN or Inf");
  for (int k = 0; k < h->count; ++k)
    if (!std::isfinite(D[k])) return fail(OT_GS_ENUMERIC, "dual_grad: the objective of instance %d is not finite", k);
  if (diff) return fail(OT_GS_EVERIFY, "dual_grad: %llu screened results differ from the dense ones", diff);
  return OT_GS_OK;
}

// Work lists over the (group, 32-target block) tiles: static lists for dense
// evaluations (whole groups by row bucket; split groups by chunk), and the
// dynamic lists the screen fills.  On-the-fly handles use a single bucket.
// A group runs in CHUNK-row chunks (two passes and a combine) when it has
// more rows than one tile holds: WHOLE_MAX for the materialised cost, CHUNK
// for the cost computed on the fly.
static bool group_split(bool onthefly, int rows) { return rows > (onthefly ? CHUNK : WHOLE_MAX); }

static int build_work_lists(ot_gs_handle* h, hipStream_t s) {
  const int count = h->count;
  {
    // Materialised cost: a row bucket with few tiles joins the next larger
    // nonempty one (one launch less per evaluation; a tile evaluated with
    // more loads per lane than it needs gives the same bits, the extra loads
    // adding exact zeros)
    int remap[NBUCKET];
    for (int b = 0; b < NBUCKET; ++b) remap[b] = b;
    if (!h->onthefly) {
      long long cnt[NBUCKET] = {};
      for (int k = 0; k < count; ++k) {
        const InstHost& ih = h->inst[k];
        for (int g = 0; g < ih.d.Le; ++g)
          if (!group_split(false, ih.g_size[g])) cnt[row_bucket(ih.g_size[g])] += ih.d.njb;
      }
      const long long few = 2LL * h->n_cu;   // fewer tiles than two workgroups per compute unit
      for (int b = 0; b < NBUCKET; ++b) {
        if (cnt[b] == 0 || cnt[b] >= few) continue;
        int b2 = b + 1;
        while (b2 < NBUCKET && cnt[b2] == 0) ++b2;
        if (b2 == NBUCKET) break;
        cnt[b2] += cnt[b];
        cnt[b] = 0;
        for (int q = 0; q < NBUCKET; ++q)
          if (remap[q] == b) remap[q] = b2;
      }
    }
    std::vector<TileDesc> all, sg, sc;
    std::vector<TileDesc> bucket[NBUCKET];
    for (int k = 0; k < count; ++k) {
      const InstHost& ih = h->inst[k];
      for (int g = 0; g < ih.d.Le; ++g) {
        const int n = ih.g_size[g];
        const bool split = group_split(h->onthefly, n);
        const int nch = (int)ceil_div(n, CHUNK);
        for (int jb = 0; jb < ih.d.njb; ++jb) {
          TileDesc t{k, g, jb, split ? -nch : (h->onthefly ? otf_bucket(n) : remap[row_bucket(n)])};
          all.push_back(t);
          if (!split) {
            bucket[t.aux].push_back(t);
          } else {
            sg.push_back(TileDesc{k, g, jb, 0});
            for (int c = 0; c < nch; ++c) sc.push_back(TileDesc{k, g, jb, c});
          }
        }
      }
    }
    std::vector<TileDesc> mainl;
    for (int b = 0; b < NBUCKET; ++b) {
      h->main_off[b] = (int)mainl.size();
      h->n_bucket[b] = (int)bucket[b].size();
      mainl.insert(mainl.end(), bucket[b].begin(), bucket[b].end());
    }
    h->n_main = (int)mainl.size();
    h->n_sg = (int)sg.size();
    h->n_sc = (int)sc.size();
    h->upd_stats = h->n_sg == 0;
    h->max_le = 1;
    long long grp = 0;
    for (int k = 0; k < count; ++k) {
      h->max_le = std::max(h->max_le, h->inst[k].d.Le);
      grp += h->inst[k].d.Le;
    }
    h->gs_large = grp > 0 && h->tot_rows > (long long)GS_SMALL * grp;
    TRY(h->alloc(&h->tiles_all, all.size()));
    TRY(h->alloc(&h->list_main, mainl.size()));
    TRY(h->alloc(&h->list_sg, sg.size()));
    TRY(h->alloc(&h->list_sc, sc.size()));
    TRY(h->alloc(&h->dyn_main, mainl.size()));
    TRY(h->alloc(&h->dyn_sg, sg.size()));
    TRY(h->alloc(&h->dyn_sc, sc.size()));
    auto up = [&](TileDesc* dst, const std::vector<TileDesc>& v) -> int {
      if (!v.empty())
        HIPCHK(hipMemcpyAsync(dst, v.data(), sizeof(TileDesc) * v.size(), hipMemcpyHostToDevice, s));
      return OT_GS_OK;
    };
    TRY(up(h->tiles_all, all));
    TRY(up(h->list_main, mainl));
    TRY(up(h->list_sg, sg));
    TRY(up(h->list_sc, sc));
    if (!h->onthefly) {
      // tile records (split tiles keep a zero record: never read)
      auto rec = [&](const TileDesc& t) {
        TileRec r;
        std::memset(&r, 0, sizeof r);
        if (t.aux < 0) return r;
        const InstHost& ih = h->inst[t.inst];
        const InstDev& I = ih.d;
        const int gs = ih.g_start[t.grp], gn = ih.g_size[t.grp];
        r.c0 = (long long)c_index(I, gs, gn, gs, t.jb * TJ);
        r.rp0 = I.r_off + (long long)t.jb * I.ns + gs;
        r.pr0 = (long long)I.pair_off + (long long)t.grp * I.nt_pad + (long long)t.jb * TJ;
        r.a0 = I.row_off + gs;
        r.b0 = I.col_off + t.jb * TJ;
        r.gn = gn;
        r.ncol = std::min(TJ, I.nt - t.jb * TJ);
        r.inst = t.inst;
        r.thr = I.thr;
        r.gamma = I.gamma;
        return r;
      };
      std::vector<TileRec> ra, rm;
      ra.reserve(all.size());
      rm.reserve(mainl.size());
      for (const TileDesc& t : all) ra.push_back(rec(t));
      for (const TileDesc& t : mainl) rm.push_back(rec(t));
      TRY(h->alloc(&h->rec_all, ra.size()));
      TRY(h->alloc(&h->rec_main, rm.size()));
      TRY(h->alloc(&h->rec_dyn, rm.size()));
      if (!ra.empty())
        HIPCHK(hipMemcpyAsync(h->rec_all, ra.data(), sizeof(TileRec) * ra.size(), hipMemcpyHostToDevice, s));
      if (!rm.empty())
        HIPCHK(hipMemcpyAsync(h->rec_main, rm.data(), sizeof(TileRec) * rm.size(), hipMemcpyHostToDevice, s));
      // the host vectors are released when this scope ends: wait for the copies
      HIPCHK(hipStreamSynchronize(s));
    }
    TRY(h->alloc(&h->counts_static, NBUCKET + 2));
    TRY(h->alloc(&h->counts_dyn, NBUCKET + 2));
    int hc[NBUCKET + 2];
    for (int b = 0; b < NBUCKET; ++b) hc[b] = h->n_bucket[b];
    hc[NBUCKET] = h->n_sg;
    hc[NBUCKET + 1] = h->n_sc;
    HIPCHK(hipMemcpyAsync(h->counts_static, hc, sizeof hc, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(h->counts_dyn, 0, sizeof(int) * (NBUCKET + 2), s));
  }
  return OT_GS_OK;
}

static void cache_apply(ot_gs_handle* h);

// On-the-fly cost setup: pack the source features per group and the target
// features in natural order, one pass over every (group, 32-target) tile for
// the largest unscaled cost (normalisation) and each column's least cost per
// group (nearest-class key), then the scale and max C of every instance.
static int setup_onthefly(ot_gs_handle* h, const ot_gs_problem* probs, int* colkey,
                          std::vector<std::pair<float*, size_t>>& temps, hipStream_t s) {
  const int count = h->count;
  TRY(h->alloc(&h->Xp, h->tot_x));
  TRY(h->alloc(&h->xn, h->tot_rows));
  TRY(h->alloc(&h->Yp, h->tot_y));
  TRY(h->alloc(&h->yn, h->tot_cols_pad));
  HIPCHK(hipMemsetAsync(h->Xp, 0, sizeof(float) * std::max<long long>(h->tot_x, 1), s));
  float *ynat = nullptr, *ynnat = nullptr, *colmin = nullptr;
  TRY(h->alloc_temp(&ynat, std::max<long long>(h->tot_y, 1)));
  temps.push_back({ynat, sizeof(float) * std::max<long long>(h->tot_y, 1)});
  TRY(h->alloc_temp(&ynnat, h->tot_cols_pad));
  temps.push_back({ynnat, sizeof(float) * h->tot_cols_pad});
  TRY(h->alloc_temp(&colmin, std::max<long long>(h->tot_pairs, 1)));
  temps.push_back({colmin, sizeof(float) * std::max<long long>(h->tot_pairs, 1)});
  TRY(h->alloc(&h->d_inst, count));
  std::vector<InstDev> hd(count);
  for (int k = 0; k < count; ++k) hd[k] = h->inst[k].d;
  HIPCHK(hipMemcpyAsync(h->d_inst, hd.data(), sizeof(InstDev) * count, hipMemcpyHostToDevice, s));
  const float** dxs = nullptr;
  const float** dxt = nullptr;
  unsigned int* maxbits = nullptr;
  TRY(h->alloc(&dxs, count));
  TRY(h->alloc(&dxt, count));
  TRY(h->alloc(&maxbits, count));
  std::vector<const float*> hxs(count), hxt(count);
  int maxns = 1, maxntp = 64, maxnt = 1;
  for (int k = 0; k < count; ++k) {
    hxs[k] = probs[k].x_src;
    hxt[k] = probs[k].x_tgt;
    maxns = std::max(maxns, h->inst[k].d.ns);
    maxntp = std::max(maxntp, h->inst[k].d.nt_pad);
    maxnt = std::max(maxnt, h->inst[k].d.nt);
  }
  HIPCHK(hipMemcpyAsync(dxs, hxs.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dxt, hxt.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(maxbits, 0, sizeof(unsigned int) * count, s));
  hipLaunchKernelGGL(k_otf_pack_x, dim3((unsigned)std::min<long long>(ceil_div(maxns, 256), 1024), count),
                     dim3(256), 0, s, h->d_inst, dxs, (const int*)h->perm_row, (const int*)h->row_grp,
                     (const int*)h->g_start, (const int*)h->g_xblk, h->Xp, h->xn, h->err);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_otf_pack_y, dim3((unsigned)ceil_div(maxntp, 256), count), dim3(256), 0, s,
                     h->d_inst, dxt, (const int*)nullptr, ynat, ynnat, h->err);
  LAUNCHCHK();
  int herr = 0;
  TRY(sync_err(h, s, &herr));
  if (herr & 2) return fail(OT_GS_ENUMERIC, "a feature (or its squared norm) is NaN or Inf");
  if (h->tot_tiles > 0) {
    GradArgs A;
    std::memset(&A, 0, sizeof A);
    A.inst = h->d_inst;
    A.g_start = h->g_start;
    A.g_size = h->g_size;
    A.g_xblk = h->g_xblk;
    A.Xp = h->Xp;
    A.xn = h->xn;
    A.list = h->tiles_all;
    const int n = (int)h->tot_tiles;
    hipLaunchKernelGGL(k_otf_setup, dim3(std::max(1, std::min(n, 2 * h->n_cu))), dim3(BLOCK), 0, s, A, n,
                       (const float*)ynat, (const float*)ynnat, colmin, maxbits);
    LAUNCHCHK();
  }
  std::vector<unsigned int> hmax(count);
  HIPCHK(hipMemcpyAsync(hmax.data(), maxbits, sizeof(unsigned int) * count, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < count; ++k) {
    InstDev& d = h->inst[k].d;
    float umax;
    std::memcpy(&umax, &hmax[k], sizeof umax);
    float sc = probs[k].cost_scale;
    if (sc == 0.f) {
      if (!(umax > 0.f)) return fail(OT_GS_ENUMERIC, "instance %d: max C is 0, cannot normalise", k);
      sc = (float)(1.0 / (double)umax);
    }
    // C = max(sc u, 0) is monotone in u; the slack covers any difference in
    // the last bit between this pass and the gradient tiles
    const float cm = umax * sc * (1.f + 1.0f / 65536.f);
    if (!std::isfinite(cm)) return fail(OT_GS_ENUMERIC, "instance %d: scaled cost overflows", k);
    d.cscale = sc;
    d.cmax = cm;
    hd[k] = d;
  }
  HIPCHK(hipMemcpyAsync(h->d_inst, hd.data(), sizeof(InstDev) * count, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_otf_assign, dim3((unsigned)ceil_div(maxnt, 256), count), dim3(256), 0, s,
                     (const InstDev*)h->d_inst, (const float*)colmin, colkey);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  return OT_GS_OK;
}

static int create_impl(const ot_gs_problem* probs, int count, ot_gs_handle** out, hipStream_t s,
                       void* ws = nullptr, size_t ws_bytes = 0) {
  if (!probs || !out || count < 1) return fail(OT_GS_EINVAL, "create: bad arguments");
  for (int k = 0; k < count; ++k) {
    const ot_gs_problem& p = probs[k];
    if (p.n_src < 1 || p.n_tgt < 1) return fail(OT_GS_EINVAL, "instance %d: n_src and n_tgt must be >= 1", k);
    if (p.n_groups < 1 || p.n_groups > MAX_GROUPS)
      return fail(OT_GS_EINVAL, "instance %d: n_groups must lie in [1, %d]", k, MAX_GROUPS);
    if (!p.labels) return fail(OT_GS_EINVAL, "instance %d: labels is NULL", k);
    if (!(p.gamma > 0.0) || !std::isfinite(p.gamma) || !((float)p.gamma > 0.f) || !std::isfinite((float)p.gamma))
      return fail(OT_GS_EINVAL, "instance %d: gamma must be > 0 (and a normal float32)", k);
    if (!(p.mu >= 0.0) || !std::isfinite(p.mu) || !std::isfinite((float)(p.mu * p.gamma)))
      return fail(OT_GS_EINVAL, "instance %d: mu must be >= 0 with mu gamma finite in float32", k);
    if (!std::isfinite(p.cost_scale) || p.cost_scale < 0.f)
      return fail(OT_GS_ENUMERIC, "instance %d: cost_scale must be finite and >= 0", k);
    if (p.cost_mode == OT_GS_COST_GIVEN) {
      if (!p.cost) return fail(OT_GS_EINVAL, "instance %d: COST_GIVEN needs cost", k);
    } else if (p.cost_mode == OT_GS_COST_MATERIALIZE) {
      if (!p.x_src || !p.x_tgt || p.dim < 1)
        return fail(OT_GS_EINVAL, "instance %d: COST_MATERIALIZE needs x_src, x_tgt and dim >= 1", k);
    } else if (p.cost_mode == OT_GS_COST_ONTHEFLY) {
      if (!p.x_src || !p.x_tgt || p.dim < 1 || p.dim > DP_MAX)
        return fail(OT_GS_EINVAL, "instance %d: COST_ONTHEFLY needs x_src, x_tgt and 1 <= dim <= %d", k,
                    DP_MAX);
    } else {
      return fail(OT_GS_EINVAL, "instance %d: unknown cost_mode %d", k, p.cost_mode);
    }
  }
  const bool otf = probs[0].cost_mode == OT_GS_COST_ONTHEFLY;
  for (int k = 1; k < count; ++k)
    if ((probs[k].cost_mode == OT_GS_COST_ONTHEFLY) != otf)
      return fail(OT_GS_EINVAL, "instance %d: COST_ONTHEFLY cannot be mixed with materialized costs in one handle", k);
  auto* h = new ot_gs_handle();
  for (int b = 0; b <= NBUCKET; ++b) h->tile_gm[b] = 2;   // workgroups per resident slot
  std::unique_ptr<ot_gs_handle> guard(h);
  if (ws) {
    const uintptr_t p0 = (uintptr_t)ws, p1 = (p0 + 255) & ~(uintptr_t)255;
    if (ws_bytes < (p1 - p0) + 256) return fail(OT_GS_ENOMEM, "create: workspace too small");
    h->ws_base = (char*)p1;
    h->ws_size = ws_bytes - (p1 - p0);
    h->ws_lo = 0;
    h->ws_hi = h->ws_size;
  }
  h->onthefly = otf;
  h->count = count;
  h->inst.resize(count);
  HIPCHK(hipGetDevice(&h->dev));
  {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, h->dev));
    h->n_cu = prop.multiProcessorCount;
  }

  // ---- offsets independent of the group layout
  long long lab_tot = 0;
  std::vector<long long> lab_off(count);
  int maxL = 1;
  for (int k = 0; k < count; ++k) {
    const ot_gs_problem& p = probs[k];
    InstDev& d = h->inst[k].d;
    std::memset(&d, 0, sizeof d);
    d.ns = p.n_src;
    d.nt = p.n_tgt;
    d.nt_pad = (int)ceil_div(p.n_tgt, TJ) * TJ;
    d.njb = d.nt_pad / TJ;
    d.L = p.n_groups;
    d.row_off = (int)h->tot_rows;
    d.scol_off = (int)h->tot_cols;
    d.col_off = (int)h->tot_cols_pad;
    d.gamma = (float)p.gamma;
    d.mu = (float)p.mu;
    d.thr = (float)(p.mu * p.gamma);
    d.gamma64 = p.gamma;
    if (otf) {
      d.onthefly = 1;
      d.dim = p.dim;
      d.dp = (int)ceil_div(p.dim, 16) * 16;
      h->otf_dpmax = std::max(h->otf_dpmax, d.dp);
    }
    h->inst[k].cost_mode = p.cost_mode;
    lab_off[k] = lab_tot;
    lab_tot += p.n_groups;
    maxL = std::max(maxL, p.n_groups);
    h->tot_rows += p.n_src;
    h->tot_cols += p.n_tgt;
    h->tot_cols_pad += d.nt_pad;
    if (h->tot_rows > 2000000000LL || h->tot_cols_pad > 2000000000LL)
      return fail(OT_GS_EINVAL, "total sizes exceed the 32-bit index range");
  }
  TRY(h->alloc(&h->err, 1));
  HIPCHK(hipMemsetAsync(h->err, 0, sizeof(int), s));

  // ---- group layout of the rows: histogram, host prefix sums, stable scatter
  int *labels = nullptr, *cnt = nullptr, *start = nullptr, *keymap = nullptr;
  SegDesc* segs = nullptr;
  TRY(h->alloc(&labels, h->tot_rows));
  TRY(h->alloc(&cnt, lab_tot));
  TRY(h->alloc(&start, lab_tot));
  TRY(h->alloc(&keymap, lab_tot));
  TRY(h->alloc(&segs, count));
  TRY(h->alloc(&h->perm_row, h->tot_rows));
  TRY(h->alloc(&h->row_grp, h->tot_rows));
  std::vector<SegDesc> hseg(count);
  for (int k = 0; k < count; ++k) {
    const InstDev& d = h->inst[k].d;
    HIPCHK(hipMemcpyAsync(labels + d.row_off, probs[k].labels, sizeof(int) * d.ns,
                          hipMemcpyDeviceToDevice, s));
    hseg[k] = SegDesc{d.ns, d.L, d.row_off, (int)lab_off[k], d.row_off, 0, 0, 0};
  }
  HIPCHK(hipMemcpyAsync(segs, hseg.data(), sizeof(SegDesc) * count, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_histogram, dim3(count), dim3(256), sizeof(int) * maxL, s, segs, labels, cnt, h->err);
  LAUNCHCHK();
  int herr = 0;
  TRY(sync_err(h, s, &herr));
  if (herr & 1) return fail(OT_GS_EINVAL, "a label lies outside [0, n_groups)");
  std::vector<int> hcnt(lab_tot), hstart(lab_tot), hkey(lab_tot);
  HIPCHK(hipMemcpy(hcnt.data(), cnt, sizeof(int) * lab_tot, hipMemcpyDeviceToHost));
  for (int k = 0; k < count; ++k) {
    InstHost& ih = h->inst[k];
    int acc = 0, ge = 0;
    for (int l = 0; l < ih.d.L; ++l) {
      const int c = hcnt[lab_off[k] + l];
      hstart[lab_off[k] + l] = acc;
      hkey[lab_off[k] + l] = c > 0 ? ge : -1;
      if (c > 0) {
        ih.g_start.push_back(acc);
        ih.g_size.push_back(c);
        ih.g_label.push_back(l);
        ++ge;
      }
      acc += c;
    }
    ih.d.Le = ge;
  }
  HIPCHK(hipMemcpyAsync(start, hstart.data(), sizeof(int) * lab_tot, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(keymap, hkey.data(), sizeof(int) * lab_tot, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_stable_scatter, dim3(count), dim3(WAVE), sizeof(int) * maxL, s, segs, labels,
                     start, keymap, h->perm_row, h->row_grp);
  LAUNCHCHK();

  // ---- offsets that depend on the groups
  for (int k = 0; k < count; ++k) {
    InstHost& ih = h->inst[k];
    InstDev& d = ih.d;
    d.grp_off = (int)h->tot_groups;
    d.pair_off = (int)h->tot_pairs;
    d.tile_off = (int)h->tot_tiles;
    d.c_off = h->tot_c;
    d.r_off = h->tot_r;
    d.chunk_off = h->tot_chunk;
    ih.n_chunk_rows = 0;
    for (int g = 0; g < d.Le; ++g) {
      if (group_split(otf, ih.g_size[g])) {
        ih.g_chunk0.push_back(ih.n_chunk_rows);
        ih.n_chunk_rows += (int)ceil_div(ih.g_size[g], CHUNK);
      } else {
        ih.g_chunk0.push_back(-1);
      }
    }
    if (otf) {
      d.x_off = h->tot_x;
      d.y_off = h->tot_y;
      int xb = 0;
      for (int g = 0; g < d.Le; ++g) {
        ih.g_xblk.push_back(xb);
        xb += (int)ceil_div(ih.g_size[g], 32);
      }
      h->tot_x += (long long)xb * 32 * d.dp;
      h->tot_y += (long long)d.njb * 32 * d.dp;
    }
    h->tot_groups += d.Le;
    h->tot_pairs += (long long)d.Le * d.nt_pad;
    h->tot_tiles += (long long)d.Le * d.njb;
    h->tot_c += (long long)d.ns * d.nt_pad;
    h->tot_r += (long long)d.njb * d.ns;
    h->tot_chunk += (long long)ih.n_chunk_rows * d.nt_pad;
    if (h->tot_pairs > 2000000000LL || h->tot_tiles > 2000000000LL)
      return fail(OT_GS_EINVAL, "total pair count exceeds the 32-bit index range");
  }
  {
    std::vector<int> gs, gn, gc, gi, gx, gl;
    std::vector<long long> lpo(count);
    for (int k = 0; k < count; ++k) {
      const InstHost& ih = h->inst[k];
      lpo[k] = h->tot_lab_pairs;
      h->tot_lab_pairs += (long long)ih.d.L * ih.d.nt;
      gl.insert(gl.end(), ih.g_label.begin(), ih.g_label.end());
      gx.insert(gx.end(), ih.g_xblk.begin(), ih.g_xblk.end());
      gs.insert(gs.end(), ih.g_start.begin(), ih.g_start.end());
      gn.insert(gn.end(), ih.g_size.begin(), ih.g_size.end());
      gc.insert(gc.end(), ih.g_chunk0.begin(), ih.g_chunk0.end());
      gi.insert(gi.end(), ih.d.Le, k);
    }
    TRY(h->alloc(&h->g_start, gs.size()));
    TRY(h->alloc(&h->g_size, gs.size()));
    TRY(h->alloc(&h->g_chunk0, gs.size()));
    TRY(h->alloc(&h->grp_inst, gs.size()));
    TRY(h->alloc(&h->g_label, gs.size()));
    TRY(h->alloc(&h->lab_pair_off, count));
    HIPCHK(hipMemcpyAsync(h->g_label, gl.data(), sizeof(int) * gl.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->lab_pair_off, lpo.data(), sizeof(long long) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->g_start, gs.data(), sizeof(int) * gs.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->g_size, gn.data(), sizeof(int) * gs.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->g_chunk0, gc.data(), sizeof(int) * gs.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->grp_inst, gi.data(), sizeof(int) * gs.size(), hipMemcpyHostToDevice, s));
    if (otf) {
      TRY(h->alloc(&h->g_xblk, gs.size()));
      HIPCHK(hipMemcpyAsync(h->g_xblk, gx.data(), sizeof(int) * gs.size(), hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
  }
  TRY(build_work_lists(h, s));

  // ---- cost provider: a materialized pool, or packed features for the
  // on-the-fly cost; both give the scale, max C and the column clustering key
  int* colkey = nullptr;
  TRY(h->alloc(&colkey, h->tot_cols));
  std::vector<std::pair<float*, size_t>> temps;
  struct TempFree {
    ot_gs_handle* h;
    std::vector<std::pair<float*, size_t>>& v;
    ~TempFree() {
      for (size_t i = v.size(); i-- > 0;) h->free_temp(v[i].first, v[i].second);
    }
  } tfree{h, temps};
  const float** d_costs = nullptr;
  float* d_scale = nullptr;
  if (!otf) {
    // ---- cost in the caller's order (given or built from features)
    std::vector<const float*> hcost(count);
    for (int k = 0; k < count; ++k) {
      const ot_gs_problem& p = probs[k];
      if (p.cost_mode == OT_GS_COST_GIVEN) {
        hcost[k] = p.cost;
      } else {
        float* tmp = nullptr;
        TRY(h->alloc_temp(&tmp, (size_t)p.n_src * p.n_tgt));
        temps.push_back({tmp, sizeof(float) * (size_t)p.n_src * p.n_tgt});
        dim3 grid((unsigned)ceil_div(p.n_tgt, 64), (unsigned)ceil_div(p.n_src, 64));
        hipLaunchKernelGGL(k_cost_features, grid, dim3(256), 0, s, p.x_src, p.x_tgt, p.n_src, p.n_tgt,
                           p.dim, tmp);
        LAUNCHCHK();
        hcost[k] = tmp;
      }
    }
    long long* d_sizes = nullptr;
    unsigned int* d_max = nullptr;
    TRY(h->alloc(&d_costs, count));
    TRY(h->alloc(&d_sizes, count));
    TRY(h->alloc(&d_max, count));
    TRY(h->alloc(&d_scale, count));
    std::vector<long long> hsizes(count);
    long long maxsize = 1;
    for (int k = 0; k < count; ++k) {
      hsizes[k] = (long long)probs[k].n_src * probs[k].n_tgt;
      maxsize = std::max(maxsize, hsizes[k]);
    }
    HIPCHK(hipMemcpyAsync(d_costs, hcost.data(), sizeof(float*) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_sizes, hsizes.data(), sizeof(long long) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(d_max, 0, sizeof(unsigned int) * count, s));
    {
      dim3 grid((unsigned)std::min<long long>(ceil_div(maxsize, 256 * 8), 2048), count);
      hipLaunchKernelGGL(k_cost_max, grid, dim3(256), 0, s, d_costs, d_sizes, d_max, h->err);
      LAUNCHCHK();
    }
    TRY(sync_err(h, s, &herr));
    if (herr & 2) return fail(OT_GS_ENUMERIC, "the cost has a negative, NaN or Inf entry");
    std::vector<unsigned int> hmax(count);
    std::vector<float> hscale(count);
    HIPCHK(hipMemcpy(hmax.data(), d_max, sizeof(unsigned int) * count, hipMemcpyDeviceToHost));
    for (int k = 0; k < count; ++k) {
      float cmax;
      std::memcpy(&cmax, &hmax[k], sizeof cmax);
      float sc = probs[k].cost_scale;
      if (sc == 0.f) {
        if (!(cmax > 0.f)) return fail(OT_GS_ENUMERIC, "instance %d: max C is 0, cannot normalise", k);
        sc = (float)(1.0 / (double)cmax);
      }
      hscale[k] = sc;
      h->inst[k].d.cscale = sc;
      const float cm = cmax * sc;   // rounding is monotone: max of the scaled cost
      if (!std::isfinite(cm)) return fail(OT_GS_ENUMERIC, "instance %d: scaled cost overflows", k);
      h->inst[k].d.cmax = cm;
    }
    HIPCHK(hipMemcpyAsync(d_scale, hscale.data(), sizeof(float) * count, hipMemcpyHostToDevice, s));

    // ---- instance descriptors
    TRY(h->alloc(&h->d_inst, count));
    {
      std::vector<InstDev> hd(count);
      for (int k = 0; k < count; ++k) hd[k] = h->inst[k].d;
      HIPCHK(hipMemcpyAsync(h->d_inst, hd.data(), sizeof(InstDev) * count, hipMemcpyHostToDevice, s));
    }

    {
      int maxnt = 1;
      for (int k = 0; k < count; ++k) maxnt = std::max(maxnt, probs[k].n_tgt);
      hipLaunchKernelGGL(k_col_assign, dim3((unsigned)ceil_div(maxnt, 256), count), dim3(256), 0, s,
                         h->d_inst, d_costs, h->perm_row, h->row_grp, colkey);
      LAUNCHCHK();
    }
  } else {
    TRY(setup_onthefly(h, probs, colkey, temps, s));
  }
  // ---- column clustering: nearest source class, then a stable sort by it
  int *ccnt = nullptr, *cstart = nullptr;
  SegDesc* csegs = nullptr;
  TRY(h->alloc(&ccnt, std::max<long long>(h->tot_groups, 1)));
  TRY(h->alloc(&cstart, std::max<long long>(h->tot_groups, 1)));
  TRY(h->alloc(&csegs, count));
  TRY(h->alloc(&h->perm_col, h->tot_cols_pad));
  HIPCHK(hipMemsetAsync(h->perm_col, 0xff, sizeof(int) * h->tot_cols_pad, s));
  std::vector<SegDesc> cseg(count);
  int maxLe = 1;
  for (int k = 0; k < count; ++k) {
    const InstDev& d = h->inst[k].d;
    cseg[k] = SegDesc{d.nt, d.Le, d.scol_off, d.grp_off, d.col_off, 0, 0, 0};
    maxLe = std::max(maxLe, d.Le);
  }
  HIPCHK(hipMemcpyAsync(csegs, cseg.data(), sizeof(SegDesc) * count, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_histogram, dim3(count), dim3(256), sizeof(int) * maxLe, s, csegs, colkey, ccnt, h->err);
  LAUNCHCHK();
  TRY(sync_err(h, s, &herr));
  if (herr) return fail(OT_GS_EDEVICE, "column clustering produced an invalid key");
  {
    std::vector<int> hc(std::max<long long>(h->tot_groups, 1)), hs(hc.size());
    HIPCHK(hipMemcpy(hc.data(), ccnt, sizeof(int) * h->tot_groups, hipMemcpyDeviceToHost));
    for (int k = 0; k < count; ++k) {
      const InstDev& d = h->inst[k].d;
      int acc = 0;
      for (int g = 0; g < d.Le; ++g) {
        hs[d.grp_off + g] = acc;
        acc += hc[d.grp_off + g];
      }
    }
    HIPCHK(hipMemcpyAsync(cstart, hs.data(), sizeof(int) * h->tot_groups, hipMemcpyHostToDevice, s));
  }
  hipLaunchKernelGGL(k_stable_scatter, dim3(count), dim3(WAVE), sizeof(int) * maxLe, s, csegs, colkey,
                     cstart, (const int*)nullptr, h->perm_col, (int*)nullptr);
  LAUNCHCHK();

  if (otf) {
    // target features in the internal column order
    const float** dxt = nullptr;
    TRY(h->alloc(&dxt, count));
    std::vector<const float*> hx(count);
    int maxntp = 64;
    for (int k = 0; k < count; ++k) {
      hx[k] = probs[k].x_tgt;
      maxntp = std::max(maxntp, h->inst[k].d.nt_pad);
    }
    HIPCHK(hipMemcpyAsync(dxt, hx.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_otf_pack_y, dim3((unsigned)ceil_div(maxntp, 256), count), dim3(256), 0, s,
                       h->d_inst, dxt, (const int*)h->perm_col, h->Yp, h->yn, h->err);
    LAUNCHCHK();
  } else {
    // ---- internal cost
    // the gradient kernel may read up to CHUNK rows past a group (masked), so
    // the pool carries CHUNK zero rows of the widest instance at its end
    {
      long long maxntp = 64;
      for (int k = 0; k < count; ++k) maxntp = std::max<long long>(maxntp, h->inst[k].d.nt_pad);
      const long long pad = (long long)CHUNK * maxntp;
      h->c_pool = h->tot_c + pad;
      TRY(h->alloc(&h->C, h->c_pool));
      HIPCHK(hipMemsetAsync(h->C + h->tot_c, 0, sizeof(float) * pad, s));
    }
    {
      int maxns = 1, maxntp = 64;
      for (int k = 0; k < count; ++k) {
        maxns = std::max(maxns, h->inst[k].d.ns);
        maxntp = std::max(maxntp, h->inst[k].d.nt_pad);
      }
      dim3 grid((unsigned)std::min<long long>(ceil_div(maxntp, 256), 64), (unsigned)std::min(maxns, 65535), count);
      hipLaunchKernelGGL(k_relayout_cost, grid, dim3(256), 0, s, h->d_inst, d_costs, d_scale, h->perm_row,
                         h->perm_col, h->row_grp, h->g_start, h->g_size, h->C);
      LAUNCHCHK();
    }

  }

  // ---- marginals: given ones must be finite, nonnegative and carry the same
  // total mass (a plan with row sums a and column sums b exists only then);
  // uniform ones have mass 1
  for (int k = 0; k < count; ++k) {
    double mass[2] = {1.0, 1.0};
    const float* m[2] = {probs[k].a, probs[k].b};
    const int len[2] = {probs[k].n_src, probs[k].n_tgt};
    for (int q = 0; q < 2; ++q) {
      if (!m[q]) continue;
      std::vector<float> hm((size_t)len[q]);
      HIPCHK(hipMemcpyAsync(hm.data(), m[q], sizeof(float) * len[q], hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double acc = 0.0;
      for (float v : hm) {
        if (!std::isfinite(v)) return fail(OT_GS_ENUMERIC, "instance %d: marginal %c has a NaN or Inf", k, "ab"[q]);
        if (v < 0.f) return fail(OT_GS_EINVAL, "instance %d: marginal %c has a negative entry", k, "ab"[q]);
        acc += v;
      }
      mass[q] = acc;
    }
    if (!(std::fabs(mass[0] - mass[1]) <= 1e-6 * std::max(1.0, std::max(mass[0], mass[1]))))
      return fail(OT_GS_EINVAL, "instance %d: marginals differ in mass (sum a = %.9g, sum b = %.9g)", k, mass[0],
                  mass[1]);
  }
  TRY(h->alloc(&h->a_int, h->tot_rows));
  TRY(h->alloc(&h->a_cal, h->tot_rows));
  TRY(h->alloc(&h->b_cal, std::max<long long>(h->tot_cols, 1)));
  TRY(h->alloc(&h->b_int, h->tot_cols_pad));
  TRY(h->alloc(&h->a_uniform, count));
  TRY(h->alloc(&h->b_uniform, count));
  {
    const float** da = nullptr;
    const float** db = nullptr;
    TRY(h->alloc(&da, count));
    TRY(h->alloc(&db, count));
    std::vector<const float*> ha(count), hb(count);
    std::vector<int> ua(count), ub(count);
    int maxn = 1;
    for (int k = 0; k < count; ++k) {
      ha[k] = probs[k].a;
      hb[k] = probs[k].b;
      ua[k] = probs[k].a == nullptr;
      ub[k] = probs[k].b == nullptr;
      h->w_unit_h.push_back(ua[k] && ub[k] && h->inst[k].d.ns == h->inst[k].d.nt);
      maxn = std::max(maxn, std::max(h->inst[k].d.ns, h->inst[k].d.nt_pad));
    }
    HIPCHK(hipMemcpyAsync(da, ha.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(db, hb.data(), sizeof(void*) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->a_uniform, ua.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(h->b_uniform, ub.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_marginals, dim3((unsigned)std::min<long long>(ceil_div(maxn, 256), 1024), count),
                       dim3(256), 0, s, h->d_inst, da, db, h->perm_row, h->perm_col, h->a_int, h->b_int,
                       h->a_cal, h->b_cal);
    LAUNCHCHK();
  }

  TRY(h->alloc(&h->row_map, h->tot_rows));
  TRY(h->alloc(&h->col_map, h->tot_cols_pad));
  TRY(h->alloc(&h->mode_dense, count));
  HIPCHK(hipMemsetAsync(h->mode_dense, 0, sizeof(int) * count, s));   // EM_DENSE
  {
    int maxn = 1;
    for (int k = 0; k < count; ++k) maxn = std::max(maxn, std::max(h->inst[k].d.ns, h->inst[k].d.nt_pad));
    hipLaunchKernelGGL(k_build_maps, dim3((unsigned)std::min<long long>(ceil_div(maxn, 256), 1024), count),
                       dim3(256), 0, s, h->d_inst, (const int*)h->perm_row, (const int*)h->perm_col, h->row_map,
                       h->col_map);
    LAUNCHCHK();
  }

  // ---- evaluation state
  for (int k = 0; k < count; ++k) {
    h->max_ns = std::max(h->max_ns, h->inst[k].d.ns);
    h->max_ntp = std::max(h->max_ntp, h->inst[k].d.nt_pad);
    h->tot_pairs_valid += (long long)h->inst[k].d.Le * h->inst[k].d.nt;
  }
  h->n_asm = asm_row_blocks(h->max_ns) + asm_col_blocks(h->max_ntp);
  TRY(h->alloc(&h->obj_part, (size_t)count * h->n_asm));
  TRY(h->alloc(&h->asm_done, count));
  HIPCHK(hipMemsetAsync(h->asm_done, 0, sizeof(unsigned int) * count, s));
  TRY(h->alloc(&h->inst_mode, count));
  HIPCHK(hipMemsetAsync(h->inst_mode, 0, sizeof(int) * count, s));
  TRY(h->alloc(&h->alpha, h->tot_rows));
  TRY(h->alloc(&h->beta, h->tot_cols_pad));
  TRY(h->alloc(&h->ga, h->tot_rows));
  TRY(h->alloc(&h->gb, h->tot_cols_pad));
  TRY(h->alloc(&h->alpha_s, h->tot_rows));
  TRY(h->alloc(&h->beta_s, h->tot_cols_pad));
  TRY(h->alloc(&h->zsnap, h->tot_pairs));
  TRY(h->alloc(&h->osnap, h->tot_pairs));
  TRY(h->alloc(&h->colsum, h->tot_pairs));
  TRY(h->alloc(&h->kappa, h->tot_pairs));
  TRY(h->alloc(&h->inN, h->tot_pairs));
  TRY(h->alloc(&h->rowpart, h->tot_r));
  TRY(h->alloc(&h->excess, h->tot_pairs));
  TRY(h->alloc(&h->tile_on, h->tot_tiles));
  TRY(h->alloc(&h->part, 3 * std::max<long long>(h->tot_chunk, 1)));
  TRY(h->alloc(&h->gstats, std::max<long long>(h->tot_groups, 1)));
  TRY(h->alloc(&h->obj, count));
  TRY(h->alloc(&h->counters, CNT_NUM));
  h->n_screen_blocks = (int)ceil_div(h->tot_tiles, SCREEN_TILES);
  TRY(h->alloc(&h->block_counters, (size_t)h->n_screen_blocks * CNT_NUM));
  HIPCHK(hipMemsetAsync(h->block_counters, 0, sizeof(long long) * h->n_screen_blocks * CNT_NUM, s));
  TRY(h->alloc(&h->t_off, count));
  HIPCHK(hipMemsetAsync(h->alpha_s, 0, sizeof(float) * h->tot_rows, s));
  HIPCHK(hipMemsetAsync(h->beta_s, 0, sizeof(float) * h->tot_cols_pad, s));
  HIPCHK(hipMemsetAsync(h->zsnap, 0, sizeof(float) * h->tot_pairs, s));
  HIPCHK(hipMemsetAsync(h->osnap, 0, sizeof(float) * h->tot_pairs, s));
  HIPCHK(hipMemsetAsync(h->inN, 0, h->tot_pairs, s));
  HIPCHK(hipMemsetAsync(h->counters, 0, sizeof(long long) * CNT_NUM, s));
  {
    std::vector<long long> to(count);
    long long acc = 0;
    for (int k = 0; k < count; ++k) {
      to[k] = acc;
      acc += (long long)probs[k].n_src * probs[k].n_tgt;
    }
    HIPCHK(hipMemcpyAsync(h->t_off, to.data(), sizeof(long long) * count, hipMemcpyHostToDevice, s));
  }
  TRY(sync_err(h, s, &herr));
  if (herr) return fail(OT_GS_EDEVICE, "setup kernels reported error flags %d", herr);
  cache_apply(h);
  *out = guard.release();
  return OT_GS_OK;
}

// ------------------------------------------------------------ evaluation

static GradArgs grad_args(ot_gs_handle* h) {
  GradArgs A;
  std::memset(&A, 0, sizeof A);
  A.inst = h->d_inst;
  A.g_start = h->g_start;
  A.g_size = h->g_size;
  A.g_chunk0 = h->g_chunk0;
  A.C = h->C_eval ? h->C_eval : h->C;
  A.g_xblk = h->g_xblk;
  A.Xp = h->Xp;
  A.Yp = h->Yp;
  A.xn = h->xn;
  A.yn = h->yn;
  A.alpha = h->alpha;
  A.beta = h->beta;
  A.rowpart = h->rowpart;
  A.colsum = h->colsum;
  A.excess = h->excess;
  A.zsnap = h->zsnap;
  A.osnap = h->osnap;
  A.part = h->part;
  A.part_stride = std::max<long long>(h->tot_chunk, 1);
  A.kappa = h->kappa;
  A.inst_mode = h->inst_mode;
  A.single_inst = h->count == 1 ? 1 : 0;
  return A;
}

static ScreenArgs screen_args(ot_gs_handle* h, int use_lower) {
  ScreenArgs S;
  std::memset(&S, 0, sizeof S);
  S.inst = h->d_inst;
  S.g_start = h->g_start;
  S.g_size = h->g_size;
  S.grp_inst = h->grp_inst;
  S.tiles_all = h->tiles_all;
  S.n_tiles_all = (int)h->tot_tiles;
  S.alpha = h->alpha;
  S.beta = h->beta;
  S.alpha_s = h->alpha_s;
  S.beta_s = h->beta_s;
  S.zsnap = h->zsnap;
  S.osnap = h->osnap;
  S.gstats = h->gstats;
  S.inN = h->inN;
  S.tile_on = h->tile_on;
  S.list_main = h->dyn_main;
  S.rec_all = h->rec_all;
  S.rec_dyn = h->rec_dyn;
  S.list_sg = h->dyn_sg;
  S.list_sc = h->dyn_sc;
  S.counts = h->counts_dyn;
  for (int b = 0; b < NBUCKET; ++b) S.main_off[b] = h->main_off[b];
  S.counters = h->counters;
  S.block_counters = h->block_counters;
  S.inst_mode = h->inst_mode;
  S.use_lower = use_lower;
  S.cmax_w = h->cmax_eval;
  return S;
}

static int grid_for(ot_gs_handle* h, int n) {
  // enough workgroups to fill the chip twice, never more than the list
  return std::max(1, std::min(n, 2 * h->n_cu));
}

static ReduceArgs reduce_args(ot_gs_handle* h, bool dynamic, float* ga_out, float* gb_out) {
  ReduceArgs R;
  std::memset(&R, 0, sizeof R);
  R.inst = h->d_inst;
  R.row_grp = h->row_grp;
  R.perm_row = h->perm_row;
  R.perm_col = h->perm_col;
  R.rowpart = h->rowpart;
  R.colsum = h->colsum;
  R.excess = h->excess;
  R.tile_on = dynamic ? h->tile_on : nullptr;
  R.a_int = h->a_int;
  R.b_int = h->b_int;
  R.a_cal = h->a_cal;
  R.b_cal = h->b_cal;
  R.alpha_cal = h->cal_alpha;
  R.beta_cal = h->cal_beta;
  R.alpha = h->alpha;
  R.beta = h->beta;
  R.ga_int = h->ga;
  R.gb_int = h->gb;
  R.ga_out = ga_out;
  R.gb_out = gb_out;
  R.obj = h->obj;
  R.obj_part = h->obj_part;
  R.obj_stride = h->n_asm;
  R.max_ns = h->max_ns;
  R.a_uniform = h->a_uniform;
  R.b_uniform = h->b_uniform;
  R.err = h->err;
  R.inst_mode = h->inst_mode;
  R.done = h->asm_done;
  return R;
}

// On-the-fly team shapes: bucket b has variant 0 = (1 << b wavefronts, one
// row block each) for b < 5 and (16, 2) for b = 5; variant 1 halves the
// team and gives every wavefront two blocks (b = 1..4).  Same results for
// every variant (per-block partial sums in block order).
static int otf_variants(int b) { return (b >= 1 && b <= 4) ? 2 : 1; }

// variants of a bucket of this handle's tile lists
static int tile_variants(const ot_gs_handle* h, int b) {
  if (b >= NBUCKET) return 1;
  if (h->onthefly) return b < OTF_NBUCKET ? otf_variants(b) : 1;
  // R = 2: teams only; R <= 16: plain, next tile in flight, LDS copy; up to
  // RMAX: plain, next tile in flight; beyond: plain
  return bucket_R(b) <= 2 ? 1 : bucket_R(b) <= 16 ? 3 : bucket_R(b) <= RMAX ? 2 : 1;
}

static void otf_shape(int b, int var, int* WT, int* BPW) {
  if (b >= 5) {
    *WT = NW;
    *BPW = 2;
  } else if (var == 0) {
    *WT = 1 << b;
    *BPW = 1;
  } else {
    *WT = 1 << (b - 1);
    *BPW = 2;
  }
}

// resident workgroups per CU of a tile kernel shape (VGPR-bound occupancy)
static int otf_resident(int WT, int BPW) {
  const int nwv = std::max(WT, 4);
  return (BPW == 1 ? 32 : 16) / nwv;
}

static int launch_otf_bucket(ot_gs_handle* h, GradArgs A, int b, int n, bool snap_possible, hipStream_t s) {
  int WT, BPW;
  otf_shape(b, h->tile_var[b], &WT, &BPW);
  const int NWV = std::max(WT, 4), K = NWV / WT;
  const dim3 grid(std::max(1, std::min((n + K - 1) / K, h->tile_gm[b] * otf_resident(WT, BPW) * h->n_cu))),
      block(64 * NWV);
  // teams of 8 or more wavefronts stage the target block in LDS
  const size_t shm = WT >= 8 ? sizeof(float) * 32 * h->otf_dpmax : 0;
  for (int sp = 0; sp < (snap_possible ? 2 : 1); ++sp) {
#define OTGS_OTF(WW, BB)                                                                     \
  if (WT == WW && BPW == BB) {                                                              \
    if (sp) hipLaunchKernelGGL((k_grad_tiles_otf<WW, BB, 0, true>), grid, block, shm, s, A); \
    else hipLaunchKernelGGL((k_grad_tiles_otf<WW, BB, 0, false>), grid, block, shm, s, A);   \
  }
    OTGS_OTF(1, 1) OTGS_OTF(2, 1) OTGS_OTF(4, 1) OTGS_OTF(8, 1) OTGS_OTF(16, 1)
    OTGS_OTF(1, 2) OTGS_OTF(2, 2) OTGS_OTF(4, 2) OTGS_OTF(8, 2) OTGS_OTF(16, 2)
#undef OTGS_OTF
    LAUNCHCHK();
  }
  return OT_GS_OK;
}

// materialised buckets: variant 0 loads a tile when it starts, variant 1
// keeps the next tile's loads in flight in registers during the current
// tile, variant 2 (R <= 16) copies the next tile into LDS meanwhile (same bits)
// materialised buckets: variant 0 runs bucket_K(b) teams per workgroup
// (groups of up to 64, 128, 256 rows: 8, 4, 2 teams; same bits as one tile
// per workgroup), variant 1 keeps the next tile's loads in flight
// in registers during the current tile, variant 2 (R <= 16) copies the next
// tile into LDS meanwhile
template <int B>
static void launch_mat_b(GradArgs A, dim3 grid, dim3 tgrid, dim3 block, bool pf, bool dma, bool mixed, int sp,
                         hipStream_t s) {
  constexpr int RR = bucket_R(B), KK = bucket_K(B);
  if constexpr (RR >= 4 && RR <= RMAX) {
    if (dma) {
      if (sp) hipLaunchKernelGGL((k_grad_tiles_dma<(RR <= 16 ? RR : 16), true>), grid, block, 0, s, A);
      else hipLaunchKernelGGL((k_grad_tiles_dma<(RR <= 16 ? RR : 16), false>), grid, block, 0, s, A);
      return;
    }
    if (pf) {
      if (sp) hipLaunchKernelGGL((k_grad_tiles_pf<RR, true>), grid, block, 0, s, A);
      else hipLaunchKernelGGL((k_grad_tiles_pf<RR, false>), grid, block, 0, s, A);
      return;
    }
  }
  if constexpr (RR <= 16) {
    if (mixed) {
      hipLaunchKernelGGL((k_grad_tiles_mixed<RR, KK>), tgrid, block, 0, s, A);
      return;
    }
  }
  if (sp) hipLaunchKernelGGL((k_grad_tiles<RR, 0, true, KK>), tgrid, block, 0, s, A);
  else hipLaunchKernelGGL((k_grad_tiles<RR, 0, false, KK>), tgrid, block, 0, s, A);
}

static int launch_mat_bucket(ot_gs_handle* h, GradArgs A, int b, int n, bool snap_possible, hipStream_t s) {
  const dim3 grid(std::max(1, std::min(n, h->tile_gm[b] * h->n_cu))), block(BLOCK);
  const bool pf = h->tile_var[b] == 1 && bucket_R(b) >= 4 && bucket_R(b) <= RMAX;
  const bool dma = h->tile_var[b] == 2 && bucket_R(b) >= 4 && bucket_R(b) <= 16;
  // variant 0 with teams: the grid counts workgroups of K tiles
  const int K = (!pf && !dma) ? bucket_K(b) : 1;
  const dim3 tgrid(std::max(1, std::min((n + K - 1) / K, h->tile_gm[b] * h->n_cu)));
  // one launch takes the tiles of both modes when both bodies fit the
  // register budget of two workgroups per compute unit (R <= 16)
  const bool mixed = !pf && !dma && snap_possible && bucket_R(b) <= 16;
  for (int sp = 0; sp < ((snap_possible && !mixed) ? 2 : 1); ++sp) {
    switch (b) {
      case 0: launch_mat_b<0>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 1: launch_mat_b<1>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 2: launch_mat_b<2>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 3: launch_mat_b<3>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 4: launch_mat_b<4>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 5: launch_mat_b<5>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 6: launch_mat_b<6>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 7: launch_mat_b<7>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 8: launch_mat_b<8>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 9: launch_mat_b<9>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 10: launch_mat_b<10>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      case 11: launch_mat_b<11>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
      default: launch_mat_b<12>(A, grid, tgrid, block, pf, dma, mixed, sp, s); break;
    }
    LAUNCHCHK();
  }
  return OT_GS_OK;
}

// split groups: chunk column partials, combine, chunk row sums
static int launch_split(ot_gs_handle* h, GradArgs A, bool dynamic, bool snap_possible, hipStream_t s) {
  const int* cnt = dynamic ? h->counts_dyn : h->counts_static;
  const int gm = h->tile_gm[NBUCKET];
  A.list = dynamic ? h->dyn_sc : h->list_sc;
  A.count = cnt + NBUCKET + 1;
  const dim3 block(BLOCK);
  const dim3 g1(std::max(1, std::min(h->n_sc, gm * (h->onthefly ? 2 : 1) * h->n_cu)));
  const dim3 g2(std::max(1, std::min(h->n_sc, gm * h->n_cu)));
  for (int sp = 0; sp < (snap_possible ? 2 : 1); ++sp) {
    if (h->onthefly) {
      const size_t shm = sizeof(float) * 32 * h->otf_dpmax;
      if (sp) hipLaunchKernelGGL((k_grad_tiles_otf<NW, 2, 1, true>), g1, block, shm, s, A);
      else hipLaunchKernelGGL((k_grad_tiles_otf<NW, 2, 1, false>), g1, block, shm, s, A);
    } else {
      if (sp) hipLaunchKernelGGL((k_grad_tiles<RMAX, 1, true>), g1, block, 0, s, A);
      else hipLaunchKernelGGL((k_grad_tiles<RMAX, 1, false>), g1, block, 0, s, A);
    }
    LAUNCHCHK();
  }
  A.list = dynamic ? h->dyn_sg : h->list_sg;
  A.count = cnt + NBUCKET;
  hipLaunchKernelGGL(k_split_combine, dim3(grid_for(h, h->n_sg) * 4), dim3(WAVE), 0, s, A);
  LAUNCHCHK();
  A.list = dynamic ? h->dyn_sc : h->list_sc;
  A.count = cnt + NBUCKET + 1;
  if (h->onthefly) hipLaunchKernelGGL((k_grad_tiles_otf<NW, 2, 2, false>), g2, block, 0, s, A);
  else hipLaunchKernelGGL((k_grad_tiles<RMAX, 2, false>), g2, block, 0, s, A);
  LAUNCHCHK();
  return OT_GS_OK;
}

// Gradient-tile launches over the static (every tile) or dynamic (screen
// output) work lists: one kernel per bucket, plus the split-group passes.
static int launch_tiles(ot_gs_handle* h, GradArgs A, bool dynamic, bool snap_possible, hipStream_t s) {
  const int* cnt = dynamic ? h->counts_dyn : h->counts_static;
  TileDesc* mlist = dynamic ? h->dyn_main : h->list_main;
  const int nb = h->onthefly ? OTF_NBUCKET : NBUCKET;
  for (int b = 0; b < nb; ++b) {
    if (h->n_bucket[b] == 0) continue;
    A.list = mlist + h->main_off[b];
    A.count = cnt + b;
    A.rec = (dynamic ? h->rec_dyn : h->rec_main) + h->main_off[b];
    A.n_static = dynamic ? -1 : h->n_bucket[b];
    if (h->onthefly) TRY(launch_otf_bucket(h, A, b, h->n_bucket[b], snap_possible, s));
    else TRY(launch_mat_bucket(h, A, b, h->n_bucket[b], snap_possible, s));
  }
  if (h->n_sg > 0) TRY(launch_split(h, A, dynamic, snap_possible, s));
  return OT_GS_OK;
}

// Gradient tiles over the static (every tile) or dynamic (screen output)
// work lists, then the fixed-order assembly.
static int run_tiles_and_reduce(ot_gs_handle* h, bool dynamic, float* ga_out, float* gb_out,
                                hipStream_t s, bool write_kappa, bool finalize = true,
                                bool snap_possible = false, double* obj_out = nullptr) {
  hipEvent_t e0 = nullptr;
  TRY(tbegin(h, KT_GRAD, s, &e0));
  GradArgs A = grad_args(h);
  A.write_kappa = write_kappa ? 1 : 0;
  TRY(launch_tiles(h, A, dynamic, snap_possible, s));
  TRY(tend(h, KT_GRAD, s, e0));
  TRY(tbegin(h, KT_REDUCE, s, &e0));
  ReduceArgs R = reduce_args(h, dynamic, ga_out, gb_out);
  // finalising: the last assembly block of each instance forms D
  R.finalize = finalize ? 1 : 0;
  R.obj_out = obj_out;
  // inside a solver step (the only non-finalising evaluations) the control
  // step counts the live instances afresh
  R.zero_first = finalize ? nullptr : h->sol.n_active;
  hipLaunchKernelGGL(k_assemble, dim3(h->n_asm, h->count), dim3(ASM_BLOCK), 0, s, R);
  LAUNCHCHK();
  TRY(tend(h, KT_REDUCE, s, e0));
  return OT_GS_OK;
}

// Evaluation with the mode of every instance read on the device: screen
// (bounds, extraction at refreshes, work lists), tiles, assembly, snapshot.
// per-group statistics of every nonempty group (one workgroup each)
static int launch_group_stats(ot_gs_handle* h, const ScreenArgs& S, hipStream_t s) {
  if (h->gs_large)
    hipLaunchKernelGGL(k_group_stats<GS_LARGE>, dim3((unsigned)h->tot_groups), dim3(GS_LARGE), 0, s, S);
  else
    hipLaunchKernelGGL(k_group_stats<GS_SMALL>, dim3((unsigned)h->tot_groups), dim3(GS_SMALL), 0, s, S);
  LAUNCHCHK();
  return OT_GS_OK;
}

static int evaluate_dynamic(ot_gs_handle* h, hipStream_t s, int use_lower, float* ga_out,
                            float* gb_out, bool write_kappa = false, bool finalize = true,
                            bool snapshot_copy = true, bool group_stats = true,
                            bool snap_possible = true, double* obj_out = nullptr) {
  hipEvent_t e0 = nullptr;
  TRY(tbegin(h, KT_SCREEN, s, &e0));
  ScreenArgs S = screen_args(h, use_lower);
  if (h->tot_groups > 0) {
    if (group_stats) {
      TRY(launch_group_stats(h, S, s));
    }
    // two or four passes per block once one pass per block would take
    // several rounds of resident blocks
    const long long nb1 = ceil_div(h->tot_tiles, SCREEN_TPB);
    if (nb1 > 2 * SCREEN_WIDE_BLOCKS)
      hipLaunchKernelGGL(k_screen_pairs<4>, dim3((unsigned)ceil_div(h->tot_tiles, 4 * SCREEN_TPB)),
                         dim3(SCREEN_TILES * 64), 0, s, S);
    else if (nb1 > SCREEN_WIDE_BLOCKS)
      hipLaunchKernelGGL(k_screen_pairs<2>, dim3((unsigned)ceil_div(h->tot_tiles, 2 * SCREEN_TPB)),
                         dim3(SCREEN_TILES * 64), 0, s, S);
    else
      hipLaunchKernelGGL(k_screen_pairs<1>, dim3((unsigned)ceil_div(h->tot_tiles, SCREEN_TPB)),
                         dim3(SCREEN_TILES * 64), 0, s, S);
    LAUNCHCHK();
  }
  TRY(tend(h, KT_SCREEN, s, e0));
  TRY(run_tiles_and_reduce(h, true, ga_out, gb_out, s, write_kappa, finalize, snap_possible, obj_out));
  if (!snapshot_copy) return OT_GS_OK;
  hipLaunchKernelGGL(k_snapshot_copy, dim3((unsigned)std::min<long long>(ceil_div(h->max_ns + h->max_ntp, 256), 256), h->count),
                     dim3(256), 0, s, h->d_inst, h->inst_mode, h->alpha, h->alpha_s, h->beta, h->beta_s);
  LAUNCHCHK();
  return OT_GS_OK;
}

// Host-directed evaluation of every instance in one mode (OT_GS_DENSE uses the
// static work lists and needs no screen pass).
static Prologue prologue_args(ot_gs_handle* h, int mode) {
  return Prologue{h->inst_mode, h->count, mode, h->counters, h->tot_pairs_valid, h->tot_tiles};
}

// (prologue_done: the gather kernel already ran the prologue)
static int evaluate(ot_gs_handle* h, int mode, float* ga_out, float* gb_out, hipStream_t s,
                    bool write_kappa = false, bool prologue_done = false, double* obj_out = nullptr) {
  if (!prologue_done) {
    hipLaunchKernelGGL(k_prologue, dim3(1), dim3(256), 0, s, h->inst_mode, h->count, mode, h->counters,
                       h->tot_pairs_valid, h->tot_tiles);
    LAUNCHCHK();
  }
  if (mode != OT_GS_DENSE) {
    // (the snapshot copy acts only on instances evaluated at a snapshot)
    TRY(evaluate_dynamic(h, s, 1, ga_out, gb_out, write_kappa, true, mode == OT_GS_SNAPSHOT, true,
                         mode == OT_GS_SNAPSHOT, obj_out));
    if (mode == OT_GS_SNAPSHOT) h->has_snapshot = true;
    return OT_GS_OK;
  }
  return run_tiles_and_reduce(h, false, ga_out, gb_out, s, write_kappa, true, false, obj_out);
}

// caller-order duals into the internal order; with mode >= 0 the same launch
// runs the evaluation prologue for that mode
static int gather(ot_gs_handle* h, const float* alpha, const float* beta, hipStream_t s, int mode = -1) {
  const long long maxn = std::max<long long>(h->max_ns, h->max_ntp);
  hipLaunchKernelGGL(k_gather_duals, dim3((unsigned)std::min<long long>(ceil_div(maxn, 256), 1024), h->count),
                     dim3(256), 0, s, h->d_inst, h->perm_row, h->perm_col, alpha, beta, h->alpha, h->beta,
                     h->err, prologue_args(h, mode < 0 ? 0 : mode), mode >= 0 ? 1 : 0);
  LAUNCHCHK();
  return OT_GS_OK;
}

// ------------------------------------------------------------ autotuning

// Cache of tuned tile configurations: a text file named by the environment
// variable OTGS_AUTOTUNE_CACHE, one "key variant grid_mult" line per entry.
// The key names the kernel family, the bucket, the feature padding and the
// size class (power of two of the tile count) and the device.
static std::string tune_key(ot_gs_handle* h, int b, int n) {
  hipDeviceProp_t prop;
  std::string arch = "gfx";
  if (hipGetDeviceProperties(&prop, h->dev) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ') c = '_';
  int lg = 0;
  while ((1 << (lg + 1)) <= std::max(n, 1)) ++lg;
  char buf[256];
  snprintf(buf, sizeof buf, "%s|%s|b%d|dp%d|n%d|cu%d", arch.c_str(), h->onthefly ? "otf" : "mat", b,
           h->onthefly ? h->inst[0].d.dp : 0, lg, h->n_cu);
  return buf;
}

static std::vector<std::pair<std::string, std::pair<int, int>>> cache_read() {
  std::vector<std::pair<std::string, std::pair<int, int>>> v;
  const char* path = std::getenv("OTGS_AUTOTUNE_CACHE");
  if (!path || !*path) return v;
  FILE* f = std::fopen(path, "r");
  if (!f) return v;
  char key[256];
  int a, b;
  while (std::fscanf(f, "%255s %d %d", key, &a, &b) == 3) v.push_back({key, {a, b}});
  std::fclose(f);
  return v;
}

static void cache_write(const std::vector<std::pair<std::string, std::pair<int, int>>>& v) {
  const char* path = std::getenv("OTGS_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (auto& e : v) std::fprintf(f, "%s %d %d\n", e.first.c_str(), e.second.first, e.second.second);
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

static int bucket_tiles(ot_gs_handle* h, int b) { return b < NBUCKET ? h->n_bucket[b] : h->n_sc; }

// apply cached configurations that match this handle
static void cache_apply(ot_gs_handle* h) {
  const auto v = cache_read();
  if (v.empty()) return;
  for (int b = 0; b <= NBUCKET; ++b) {
    const int n = bucket_tiles(h, b);
    if (n == 0) continue;
    const std::string k = tune_key(h, b, n);
    for (auto& e : v)
      if (e.first == k) {
        const int nvar = tile_variants(h, b);
        if (e.second.first >= 0 && e.second.first < nvar && e.second.second >= 1 && e.second.second <= 16) {
          h->tile_var[b] = e.second.first;
          h->tile_gm[b] = e.second.second;
        }
      }
  }
}

// time `repeats` dense launches of one bucket's tile kernel (or the split
// passes, b = NBUCKET) under the handle's current configuration
// (cal_a, cal_b: the current point in the caller's order; the tiles then
// read it as a dense ot_gs_dual_grad does)
static int time_bucket(ot_gs_handle* h, int b, int repeats, hipStream_t s, float* ms, const float* cal_a = nullptr,
                       const float* cal_b = nullptr) {
  GradArgs A = grad_args(h);
  if (cal_a) {
    A.alpha = cal_a;
    A.beta = cal_b;
    A.row_map = h->row_map;
    A.col_map = h->col_map;
    A.inst_mode = h->mode_dense;
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto run = [&]() -> int {
    if (b == NBUCKET) return launch_split(h, A, false, false, s);
    A.list = h->list_main + h->main_off[b];
    A.count = h->counts_static + b;
    A.rec = h->rec_main ? h->rec_main + h->main_off[b] : nullptr;
    A.n_static = h->n_bucket[b];
    return h->onthefly ? launch_otf_bucket(h, A, b, h->n_bucket[b], false, s)
                       : launch_mat_bucket(h, A, b, h->n_bucket[b], false, s);
  };
  int rc = run();   // warm-up
  if (rc == OT_GS_OK) {
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < repeats && rc == OT_GS_OK; ++i) rc = run();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(ms, e0, e1);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

static int dense_caller_order(ot_gs_handle* h, const float* alpha, const float* beta, float* ga_out,
                              float* gb_out, double* obj, hipStream_t s);

static int autotune_impl(ot_gs_handle* h, int repeats, hipStream_t s) {
  const bool was_on = h->timing.on;
  h->timing.on = false;
  // dense mode for every instance: every listed tile is computed
  hipLaunchKernelGGL(k_prologue, dim3(1), dim3(256), 0, s, h->inst_mode, h->count, (int)OT_GS_DENSE,
                     h->counters, 0LL, 0LL);
  LAUNCHCHK();
  auto cache = cache_read();
  // materialised handles are timed on the read path of dense
  // ot_gs_dual_grad calls (caller-order duals through the index maps), with
  // the current point scattered into caller order; a handle in a caller's
  // workspace, which allocates nothing more, is timed on the internal order
  float* cal = nullptr;
  if (!h->onthefly && !h->ws_base) {
    const size_t nr = (size_t)h->tot_rows, nc = (size_t)std::max<long long>(h->tot_cols, 1);
    if (hipMalloc(&cal, sizeof(float) * (nr + nc)) == hipSuccess) {
      const long long maxv = std::max<long long>(h->max_ns, h->max_ntp);
      hipLaunchKernelGGL(k_scatter_duals, dim3((unsigned)std::min<long long>(ceil_div(maxv, 256), 1024), h->count),
                         dim3(256), 0, s, h->d_inst, h->perm_row, h->perm_col, (const float*)h->alpha,
                         (const float*)h->beta, cal, cal + nr);
      LAUNCHCHK();
    } else {
      (void)hipGetLastError();
      cal = nullptr;
    }
  }
  struct CalFree {
    float*& p;
    ~CalFree() {
      if (p) (void)hipFree(p);
    }
  } cal_free{cal};
  const float* cal_b = cal ? cal + h->tot_rows : nullptr;
  if (cal) {
    // the read path of dense ot_gs_dual_grad calls: whole evaluations each
    // way at the current point, the faster kept; the tile shapes are then
    // tuned on that path
    float* out = nullptr;
    const size_t nr = (size_t)h->tot_rows, nc = (size_t)std::max<long long>(h->tot_cols, 1);
    if (hipMalloc(&out, sizeof(float) * (nr + nc) + sizeof(double) * h->count) == hipSuccess) {
      struct OutFree {
        float* p;
        ~OutFree() { (void)hipFree(p); }
      } out_free{out};
      double* obj = (double*)(out + nr + nc);
      float best[2] = {INFINITY, INFINITY};
      for (int direct = 0; direct < 2; ++direct) {
        auto eval = [&]() -> int {
          if (direct) return dense_caller_order(h, cal, cal_b, out, out + nr, obj, s);
          TRY(gather(h, cal, cal_b, s, OT_GS_DENSE));
          return evaluate(h, OT_GS_DENSE, out, out + nr, s, false, true, obj);
        };
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        int rc = eval();
        if (rc == OT_GS_OK) {
          (void)hipEventRecord(e0, s);
          for (int i = 0; i < repeats && rc == OT_GS_OK; ++i) rc = eval();
          (void)hipEventRecord(e1, s);
          (void)hipEventSynchronize(e1);
          (void)hipEventElapsedTime(&best[direct], e0, e1);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != OT_GS_OK) {
          h->timing.on = was_on;
          return rc;
        }
      }
      h->dense_direct = best[1] <= best[0] ? 1 : 0;
    } else {
      (void)hipGetLastError();
    }
    if (h->dense_direct == 0) cal_b = nullptr;
  }
  const float* cal_a = cal_b ? cal : nullptr;
  static const int gms[] = {1, 2, 4};
  for (int b = 0; b <= NBUCKET; ++b) {
    const int n = bucket_tiles(h, b);
    if (n == 0 || (h->onthefly && b >= OTF_NBUCKET && b < NBUCKET)) continue;
    const int nvar = tile_variants(h, b);
    float best = INFINITY;
    int bv = h->tile_var[b], bg = h->tile_gm[b];
    for (int var = 0; var < nvar; ++var)
      for (int gm : gms) {
        h->tile_var[b] = var;
        h->tile_gm[b] = gm;
        float ms = 0.f;
        const int rc = time_bucket(h, b, repeats, s, &ms, cal_a, cal_b);
        if (rc != OT_GS_OK) {
          h->timing.on = was_on;
          return rc;
        }
        if (ms < best) {
          best = ms;
          bv = var;
          bg = gm;
        }
      }
    h->tile_var[b] = bv;
    h->tile_gm[b] = bg;
    const std::string k = tune_key(h, b, n);
    bool found = false;
    for (auto& e : cache)
      if (e.first == k) {
        e.second = {bv, bg};
        found = true;
      }
    if (!found) cache.push_back({k, {bv, bg}});
  }
  cache_write(cache);
  h->timing.on = was_on;
  return OT_GS_OK;
}

// ------------------------------------------------------------ C ABI

// one pass of the sparse plan over every tile (count or fill)
template <int MODE>
static int csr_pass(ot_gs_handle* h, const CsrSink& K, hipStream_t s) {
  const int n = (int)h->tot_tiles;
  if (n == 0) return OT_GS_OK;
  if (h->onthefly) {
    GradArgs A = grad_args(h);
    A.list = h->tiles_all;
    hipLaunchKernelGGL(k_otf_emit<MODE>, dim3(grid_for(h, n)), dim3(BLOCK), 0, s, A, n, (const int*)h->perm_row,
                       (const int*)h->perm_col, (const long long*)h->t_off, (float*)nullptr, K);
  } else {
    hipLaunchKernelGGL(k_plan_csr<MODE>, dim3((unsigned)std::min(n, 8 * h->n_cu)), dim3(256), 0, s, h->d_inst,
                       (const TileDesc*)h->tiles_all, n, (const int*)h->perm_row, (const int*)h->perm_col,
                       (const int*)h->g_start, (const int*)h->g_size, (const float*)h->C, (const float*)h->alpha,
                       (const float*)h->beta, (const float*)h->kappa, K);
  }
  LAUNCHCHK();
  return OT_GS_OK;
}

static int ensure_solver(ot_gs_handle* h, int hist, hipStream_t s);

// Everything a handle can later need on the device, allocated now: the
// solver buffers for up to max_hist pairs, the checked-evaluation buffers,
// the re-centring copy of a materialised cost and plan_csr's scratch.
static int reserve_all(ot_gs_handle* h, int max_hist, hipStream_t s) {
  TRY(ensure_solver(h, max_hist, s));
  TRY(ensure_verify(h));
  if (!h->onthefly) {
    TRY(h->alloc(&h->Cw, h->c_pool));
    TRY(h->alloc(&h->cmax_w, h->count));
  }
  long long cstride = 1;
  for (int k = 0; k < h->count; ++k) cstride = std::max<long long>(cstride, h->inst[k].d.njb);
  const size_t rows = (size_t)h->tot_rows;
  const size_t bytes = ot_gs_handle::aligned(sizeof(int) * rows * cstride) +
                       ot_gs_handle::aligned(sizeof(long long) * rows * cstride);
  TRY(h->alloc(&h->csr_scratch, bytes));
  HIPCHK(hipStreamSynchronize(s));
  return OT_GS_OK;
}

template <class Step>
static int capture_n(ot_gs_handle* h, int n, hipGraphExec_t* exec, Step&& step);

extern "C" {

int ot_gs_workspace_size(const ot_gs_problem* probs, int count, int max_hist, size_t* bytes, void* stream) {
  if (!bytes || max_hist < 1 || max_hist > HMAX)
    return fail(OT_GS_EINVAL, "workspace_size: bytes NULL or max_hist outside [1, %d]", HMAX);
  ot_gs_handle* h = nullptr;
  try {
    TRY(create_impl(probs, count, &h, (hipStream_t)stream));
  } catch (...) {
    return fail(OT_GS_ENOMEM, "workspace_size: host allocation failed");
  }
  std::unique_ptr<ot_gs_handle> guard(h);
  TRY(reserve_all(h, max_hist, (hipStream_t)stream));
  *bytes = h->led_persist + h->led_temp_peak + 256;
  return OT_GS_OK;
}

int ot_gs_create_ws(const ot_gs_problem* probs, int count, int max_hist, void* workspace, size_t ws_bytes,
                    ot_gs_handle** out, void* stream) {
  if (!workspace || !out || max_hist < 1 || max_hist > HMAX)
    return fail(OT_GS_EINVAL, "create_ws: NULL workspace or out, or max_hist outside [1, %d]", HMAX);
  ot_gs_handle* h = nullptr;
  try {
    TRY(create_impl(probs, count, &h, (hipStream_t)stream, workspace, ws_bytes));
  } catch (...) {
    return fail(OT_GS_ENOMEM, "create_ws: host allocation failed");
  }
  std::unique_ptr<ot_gs_handle> guard(h);
  TRY(reserve_all(h, max_hist, (hipStream_t)stream));
  *out = guard.release();
  return OT_GS_OK;
}

int ot_gs_create(const ot_gs_problem* probs, int count, ot_gs_handle** out, void* stream) {
  try {
    return create_impl(probs, count, out, (hipStream_t)stream);
  } catch (...) {
    return fail(OT_GS_ENOMEM, "create: host allocation failed");
  }
}

void ot_gs_destroy(ot_gs_handle* h) { delete h; }

static bool use_dense_direct(const ot_gs_handle* h) {
  if (h->onthefly) return false;
  if (h->dense_direct >= 0) return h->dense_direct != 0;
  return h->c_pool <= (64ll << 20);   // up to 8192^2 entries
}

// Dense evaluation of caller-order duals in two launches: the tiles read
// alpha and beta through the caller-order maps (every instance's mode read
// as dense), the assembly reads them through the permutations, flags
// non-finite values and runs the evaluation prologue; the internal copies
// of alpha and beta are not written.
static int dense_caller_order(ot_gs_handle* h, const float* alpha, const float* beta, float* ga_out,
                              float* gb_out, double* obj, hipStream_t s) {
  hipEvent_t e0 = nullptr;
  TRY(tbegin(h, KT_GRAD, s, &e0));
  GradArgs A = grad_args(h);
  A.alpha = alpha;
  A.beta = beta;
  A.row_map = h->row_map;
  A.col_map = h->col_map;
  A.inst_mode = h->mode_dense;
  TRY(launch_tiles(h, A, false, false, s));
  TRY(tend(h, KT_GRAD, s, e0));
  TRY(tbegin(h, KT_REDUCE, s, &e0));
  ReduceArgs R = reduce_args(h, false, ga_out, gb_out);
  R.alpha = alpha;
  R.beta = beta;
  R.alpha_cal = alpha;
  R.beta_cal = beta;
  R.caller_order = 1;
  R.pro = prologue_args(h, OT_GS_DENSE);
  R.finalize = 1;
  R.obj_out = obj;
  hipLaunchKernelGGL(k_assemble, dim3(h->n_asm, h->count), dim3(ASM_BLOCK), 0, s, R);
  LAUNCHCHK();
  TRY(tend(h, KT_REDUCE, s, e0));
  return OT_GS_OK;
}

int ot_gs_dual_grad(ot_gs_handle* h, const float* alpha, const float* beta, float* grad_alpha,
                    float* grad_beta, double* obj, int mode, void* stream) {
  if (!h || !alpha || !beta) return fail(OT_GS_EINVAL, "dual_grad: NULL argument");
  const int base = mode & 0xff, flags = mode & ~0xff;
  if (base != OT_GS_DENSE && base != OT_GS_SCREENED && base != OT_GS_SNAPSHOT)
    return fail(OT_GS_EINVAL, "dual_grad: unknown mode %d", base);
  if (flags & ~(OT_GS_CHECK | OT_GS_VERIFY)) return fail(OT_GS_EINVAL, "dual_grad: unknown mode flags 0x%x", flags);
  hipStream_t s = (hipStream_t)stream;
  if (!flags && base == OT_GS_DENSE && use_dense_direct(h))
    return dense_caller_order(h, alpha, beta, grad_alpha, grad_beta, obj, s);
  // the assembly forms D from the caller's arrays, as the path above does
  struct CallerDuals {
    ot_gs_handle* h;
    ~CallerDuals() { h->cal_alpha = h->cal_beta = nullptr; }
  } caller_duals{h};
  h->cal_alpha = alpha;
  h->cal_beta = beta;
  if (!flags) {
    TRY(gather(h, alpha, beta, s, base));
    TRY(evaluate(h, base, grad_alpha, grad_beta, s, false, true, obj));
    return OT_GS_OK;
  }
  // checked call: this call's inputs only, then a synchronised report
  TRY(clear_err(h, s));
  TRY(gather(h, alpha, beta, s, base));
  if (!(flags & OT_GS_VERIFY) || base == OT_GS_DENSE) {
    TRY(ensure_verify(h));
    TRY(evaluate(h, base, grad_alpha, grad_beta, s, false, true, h->ver.obj));
    if (obj) HIPCHK(hipMemcpyAsync(obj, h->ver.obj, sizeof(double) * h->count, hipMemcpyDeviceToDevice, s));
    return check_report(h, s, false);
  }
  // verified call: the screened evaluation, then a dense one at the same
  // point (its counts taken back), compared bit for bit
  TRY(ensure_verify(h));
  auto& V = h->ver;
  float* ga2 = V.ga + h->tot_rows;
  float* gb2 = V.gb + h->tot_cols;
  double* o2 = V.obj + h->count;
  TRY(evaluate(h, base, V.ga, V.gb, s, false, true, V.obj));
  HIPCHK(hipMemcpyAsync(V.cnt, h->counters, sizeof(long long) * CNT_NUM, hipMemcpyDeviceToDevice, s));
  TRY(evaluate(h, OT_GS_DENSE, ga2, gb2, s, false, false, o2));
  HIPCHK(hipMemcpyAsync(h->counters, V.cnt, sizeof(long long) * CNT_NUM, hipMemcpyDeviceToDevice, s));
  const long long maxn = std::max<long long>(std::max<long long>(h->max_ns, h->max_ntp), 1);
  hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, V.diff, 1LL, 0ull);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_bits_differ, dim3((unsigned)std::min<long long>(ceil_div(maxn, 256), 256), h->count), dim3(256),
                     0, s, h->d_inst, (const int*)nullptr, 1, V.ga, ga2, V.gb, gb2, V.obj, o2, 1LL, V.diff);
  LAUNCHCHK();
  if (grad_alpha)
    HIPCHK(hipMemcpyAsync(grad_alpha, V.ga, sizeof(float) * h->tot_rows, hipMemcpyDeviceToDevice, s));
  if (grad_beta)
    HIPCHK(hipMemcpyAsync(grad_beta, V.gb, sizeof(float) * h->tot_cols, hipMemcpyDeviceToDevice, s));
  if (obj) HIPCHK(hipMemcpyAsync(obj, V.obj, sizeof(double) * h->count, hipMemcpyDeviceToDevice, s));
  return check_report(h, s, true);
}

int ot_gs_check(ot_gs_handle* h, void* stream) {
  if (!h) return fail(OT_GS_EINVAL, "check: NULL handle");
  hipStream_t s = (hipStream_t)stream;
  int herr = 0;
  TRY(sync_err(h, s, &herr));
  TRY(clear_err(h, s));
  HIPCHK(hipStreamSynchronize(s));
  if (herr & ERR_NONFINITE) return fail(OT_GS_ENUMERIC, "a NaN or Inf dual value was passed since the last check");
  return OT_GS_OK;
}

int ot_gs_screen_state(ot_gs_handle* h, float* alpha_s, float* beta_s, float* z_snap, float* o_snap,
                       uint8_t* in_N, void* stream) {
  if (!h) return fail(OT_GS_EINVAL, "screen_state: NULL handle");
  hipStream_t s = (hipStream_t)stream;
  const long long np = h->tot_lab_pairs;
  const unsigned fb = (unsigned)std::min<long long>(std::max<long long>(ceil_div(np, 256), 1), 4096);
  if (z_snap) hipLaunchKernelGGL(k_fill<float>, dim3(fb), dim3(256), 0, s, z_snap, np, 0.f);
  if (o_snap) hipLaunchKernelGGL(k_fill<float>, dim3(fb), dim3(256), 0, s, o_snap, np, 0.f);
  if (in_N) hipLaunchKernelGGL(k_fill<uint8_t>, dim3(fb), dim3(256), 0, s, in_N, np, (uint8_t)0);
  LAUNCHCHK();
  long long maxp = 1;
  for (int k = 0; k < h->count; ++k)
    maxp = std::max<long long>(maxp, std::max<long long>((long long)h->inst[k].d.Le * h->inst[k].d.nt,
                                                         h->inst[k].d.ns + h->inst[k].d.nt));
  hipLaunchKernelGGL(k_export_screen, dim3((unsigned)std::min<long long>(ceil_div(maxp, 256), 1024), h->count),
                     dim3(256), 0, s, h->d_inst, (const int*)h->perm_row, (const int*)h->perm_col,
                     (const int*)h->g_label, (const long long*)h->lab_pair_off, (const float*)h->alpha_s,
                     (const float*)h->beta_s, (const float*)h->zsnap, (const float*)h->osnap,
                     (const uint8_t*)h->inN, alpha_s, beta_s, z_snap, o_snap, in_N);
  LAUNCHCHK();
  return OT_GS_OK;
}

int ot_gs_plan(ot_gs_handle* h, const float* alpha, const float* beta, float* T, void* stream) {
  if (!h || !alpha || !beta || !T) return fail(OT_GS_EINVAL, "plan: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  TRY(gather(h, alpha, beta, s));
  TRY(evaluate(h, OT_GS_DENSE, nullptr, nullptr, s, true));
  if (h->onthefly) {
    GradArgs A = grad_args(h);
    A.list = h->tiles_all;
    const int n = (int)h->tot_tiles;
    if (n > 0) {
      hipLaunchKernelGGL(k_otf_emit<PLAN_DENSE>, dim3(grid_for(h, n)), dim3(BLOCK), 0, s, A, n,
                         (const int*)h->perm_row, (const int*)h->perm_col, (const long long*)h->t_off, T, CsrSink{});
      LAUNCHCHK();
    }
    return OT_GS_OK;
  }
  dim3 grid((unsigned)std::min<long long>(ceil_div(h->max_ntp, 256), 16), (unsigned)std::min(h->max_ns, 4096), h->count);
  hipLaunchKernelGGL(k_plan_dense, grid, dim3(256), 0, s, h->d_inst, h->perm_row, h->perm_col, h->row_grp,
                     h->g_start, h->g_size, h->C, h->alpha, h->beta, h->kappa, h->t_off, T);
  LAUNCHCHK();
  return OT_GS_OK;
}

int ot_gs_plan_csr(ot_gs_handle* h, const float* alpha, const float* beta, long long* row_ptr, int* col_idx,
                   float* val, long long* nnz, void* stream) {
  if (!h || !alpha || !beta || !row_ptr) return fail(OT_GS_EINVAL, "plan_csr: NULL argument");
  if (col_idx ? !val : !nnz) return fail(OT_GS_EINVAL, "plan_csr: count needs nnz, fill needs col_idx and val");
  hipStream_t s = (hipStream_t)stream;
  TRY(gather(h, alpha, beta, s));
  TRY(evaluate(h, OT_GS_DENSE, nullptr, nullptr, s, true));
  long long cstride = 1;
  for (int k = 0; k < h->count; ++k) cstride = std::max<long long>(cstride, h->inst[k].d.njb);
  const long long rows = h->tot_rows;
  // temporary device memory of this call: segment counts, then row totals
  // (count) or segment offsets (fill)
  std::vector<void*> tmp;
  struct Free {
    std::vector<void*>& v;
    ~Free() {
      for (void* p : v) (void)hipFree(p);
    }
  } free_tmp{tmp};
  size_t used = 0;   // of the workspace's reserved scratch
  auto al = [&](void** p, size_t bytes) -> int {
    if (h->csr_scratch) {
      *p = h->csr_scratch + used;
      used += ot_gs_handle::aligned(bytes);
      return OT_GS_OK;
    }
    const hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 8));
    if (e != hipSuccess) return fail(OT_GS_ENOMEM, "plan_csr: hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    tmp.push_back(*p);
    return OT_GS_OK;
  };
  int* cnt = nullptr;
  TRY(al((void**)&cnt, sizeof(int) * (size_t)rows * cstride));
  CsrSink K{cnt, nullptr, cstride, nullptr, nullptr};
  TRY(csr_pass<CSR_COUNT>(h, K, s));
  const dim3 rgrid((unsigned)std::min<long long>(ceil_div(h->max_ns, 256), 1024), h->count);
  if (!col_idx) {
    long long* tot = nullptr;
    TRY(al((void**)&tot, sizeof(long long) * (size_t)rows));
    hipLaunchKernelGGL(k_csr_rowsum, rgrid, dim3(256), 0, s, h->d_inst, (const int*)cnt, cstride, tot);
    LAUNCHCHK();
    std::vector<long long> ht((size_t)rows), rp((size_t)rows + 1);
    HIPCHK(hipMemcpyAsync(ht.data(), tot, sizeof(long long) * (size_t)rows, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    rp[0] = 0;
    for (long long i = 0; i < rows; ++i) rp[(size_t)i + 1] = rp[(size_t)i] + ht[(size_t)i];
    HIPCHK(hipMemcpyAsync(row_ptr, rp.data(), sizeof(long long) * ((size_t)rows + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    *nnz = rp[(size_t)rows];
    return OT_GS_OK;
  }
  long long* seg = nullptr;
  TRY(al((void**)&seg, sizeof(long long) * (size_t)rows * cstride));
  HIPCHK(hipMemsetAsync(h->err, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_csr_segoff, rgrid, dim3(256), 0, s, h->d_inst, (const int*)cnt, cstride,
                     (const long long*)row_ptr, seg, h->err);
  LAUNCHCHK();
  K.seg = seg;
  K.col = col_idx;
  K.val = val;
  TRY(csr_pass<CSR_FILL>(h, K, s));
  int herr = 0;
  TRY(sync_err(h, s, &herr));
  if (herr & 16) return fail(OT_GS_EINVAL, "plan_csr: row counts differ from row_ptr (a point other than the count call's)");
  return OT_GS_OK;
}

int ot_gs_cost(ot_gs_handle* h, float* C_out, void* stream) {
  if (!h || !C_out) return fail(OT_GS_EINVAL, "cost: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if (h->onthefly) {
    GradArgs A = grad_args(h);
    A.list = h->tiles_all;
    const int n = (int)h->tot_tiles;
    if (n > 0) {
      hipLaunchKernelGGL(k_otf_emit<0>, dim3(grid_for(h, n)), dim3(BLOCK), 0, s, A, n,
                         (const int*)h->perm_row, (const int*)h->perm_col, (const long long*)h->t_off, C_out,
                         CsrSink{});
      LAUNCHCHK();
    }
    return OT_GS_OK;
  }
  dim3 grid((unsigned)std::min<long long>(ceil_div(h->max_ntp, 256), 16), (unsigned)std::min(h->max_ns, 4096), h->count);
  hipLaunchKernelGGL(k_cost_dump, grid, dim3(256), 0, s, h->d_inst, h->perm_row, h->perm_col, h->row_grp,
                     h->g_start, h->g_size, h->C, h->t_off, C_out);
  LAUNCHCHK();
  return OT_GS_OK;
}

int ot_gs_rho_to_mu(double gamma, double rho, double* gamma_out, double* mu_out) {
  if (!(gamma > 0) || !(rho >= 0 && rho < 1)) return fail(OT_GS_EINVAL, "rho must lie in [0,1), gamma > 0");
  if (gamma_out) *gamma_out = gamma * (1 - rho);
  if (mu_out) *mu_out = rho / (1 - rho);
  return OT_GS_OK;
}

int ot_gs_get_stats(ot_gs_handle* h, ot_gs_stats* out, int reset, void* stream) {
  if (!h || !out) return fail(OT_GS_EINVAL, "get_stats: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  long long c[CNT_NUM];
  std::vector<long long> bc((size_t)h->n_screen_blocks * CNT_NUM);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(c, h->counters, sizeof c, hipMemcpyDeviceToHost));
  if (!bc.empty())
    HIPCHK(hipMemcpy(bc.data(), h->block_counters, sizeof(long long) * bc.size(), hipMemcpyDeviceToHost));
  for (size_t b = 0; b < (size_t)h->n_screen_blocks; ++b)
    for (int q = 0; q < CNT_NUM; ++q) c[q] += bc[b * CNT_NUM + q];
  out->evals = c[CNT_EVALS];
  out->pairs_total = c[CNT_PAIRS_TOTAL];
  out->pairs_in_N = c[CNT_PAIRS_N];
  out->pairs_checked = c[CNT_PAIRS_CHECKED];
  out->pairs_unskipped = c[CNT_PAIRS_UNSKIPPED];
  out->refreshes = c[CNT_REFRESH];
  out->tiles_total = c[CNT_TILES_TOTAL];
  out->tiles_computed = c[CNT_TILES_COMPUTED];
  if (reset) {
    HIPCHK(hipMemset(h->counters, 0, sizeof c));
    if (!bc.empty()) HIPCHK(hipMemset(h->block_counters, 0, sizeof(long long) * bc.size()));
  }
  return OT_GS_OK;
}

int ot_gs_profile_tiles(ot_gs_handle* h, const float* alpha, const float* beta, int repeats, double* us_per_launch,
                        void* stream) {
  if (!h || repeats < 1 || !us_per_launch) return fail(OT_GS_EINVAL, "profile_tiles: bad arguments");
  if (!alpha != !beta) return fail(OT_GS_EINVAL, "profile_tiles: alpha and beta go together");
  if (alpha && h->onthefly) return fail(OT_GS_EINVAL, "profile_tiles: caller-order duals need a materialised cost");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_prologue, dim3(1), dim3(256), 0, s, h->inst_mode, h->count, (int)OT_GS_DENSE,
                     h->counters, 0LL, 0LL);
  LAUNCHCHK();
  const bool was_on = h->timing.on;
  h->timing.on = false;
  GradArgs A = grad_args(h);
  if (alpha && use_dense_direct(h)) {
    A.alpha = alpha;
    A.beta = beta;
    A.row_map = h->row_map;
    A.col_map = h->col_map;
    A.inst_mode = h->mode_dense;
  } else if (alpha) {
    // the handle's dense evaluations gather first: so does this
    TRY(gather(h, alpha, beta, s));
  }
  // the launches recorded into a graph and replayed (once to warm up), so
  // that the time between two events is the launches' own, with the short
  // in-graph gaps between them
  hipGraphExec_t exec = nullptr;
  TRY(capture_n(h, repeats, &exec, [&](hipStream_t cs) { return launch_tiles(h, A, false, false, cs); }));
  struct ExecFree {
    hipGraphExec_t e;
    ~ExecFree() { (void)hipGraphExecDestroy(e); }
  } exec_free{exec};
  HIPCHK(hipGraphLaunch(exec, s));
  HIPCHK(hipEventRecord(e0, s));
  HIPCHK(hipGraphLaunch(exec, s));
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  h->timing.on = was_on;
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *us_per_launch = 1e3 * (double)ms / repeats;
  return OT_GS_OK;
}

int ot_gs_tile_config(ot_gs_handle* h, int bucket, int variant, int grid_mult) {
  if (!h || bucket < 0 || bucket > NBUCKET) return fail(OT_GS_EINVAL, "tile_config: bad bucket");
  const int nvar = tile_variants(h, bucket);
  if (variant < 0 || variant >= nvar) return fail(OT_GS_EINVAL, "tile_config: bucket %d has %d variants", bucket, nvar);
  if (grid_mult < 1 || grid_mult > 16) return fail(OT_GS_EINVAL, "tile_config: grid_mult must lie in [1, 16]");
  h->tile_var[bucket] = variant;
  h->tile_gm[bucket] = grid_mult;
  return OT_GS_OK;
}

int ot_gs_get_tile_config(ot_gs_handle* h, int bucket, int* variant, int* grid_mult, int* n_tiles) {
  if (!h || bucket < 0 || bucket > NBUCKET) return fail(OT_GS_EINVAL, "get_tile_config: bad bucket");
  if (variant) *variant = h->tile_var[bucket];
  if (grid_mult) *grid_mult = h->tile_gm[bucket];
  if (n_tiles) *n_tiles = bucket < NBUCKET ? h->n_bucket[bucket] : h->n_sc;
  return OT_GS_OK;
}

int ot_gs_autotune(ot_gs_handle* h, int repeats, void* stream) {
  if (!h || repeats < 1) return fail(OT_GS_EINVAL, "autotune: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  return autotune_impl(h, repeats, s);
}

int ot_gs_kernel_timing(ot_gs_handle* h, int enable) {
  if (!h) return fail(OT_GS_EINVAL, "kernel_timing: NULL handle");
  h->timing.on = enable != 0;
  return OT_GS_OK;
}

int ot_gs_kernel_time(ot_gs_handle* h, int which, double* ms, long long* launches) {
  if (!h || which < 0 || which >= KT_NUM) return fail(OT_GS_EINVAL, "kernel_time: bad arguments");
  auto& v = h->timing.ev[which];
  for (auto& e : v) {
    HIPCHK(hipEventSynchronize(e.second));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e.first, e.second));
    h->timing.ms[which] += t;
    h->timing.n[which] += 1;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  v.clear();
  if (ms) *ms = h->timing.ms[which];
  if (launches) *launches = h->timing.n[which];
  h->timing.ms[which] = 0;
  h->timing.n[which] = 0;
  return OT_GS_OK;
}

int ot_gs_layout_info(ot_gs_handle* h, int k, int* n_groups_nonempty, int* n_tgt_padded, int* n_tiles) {
  if (!h || k < 0 || k >= h->count) return fail(OT_GS_EINVAL, "layout_info: bad arguments");
  const InstDev& d = h->inst[k].d;
  if (n_groups_nonempty) *n_groups_nonempty = d.Le;
  if (n_tgt_padded) *n_tgt_padded = d.nt_pad;
  if (n_tiles) *n_tiles = d.Le * d.njb;
  return OT_GS_OK;
}

const char* ot_gs_last_error(void) { return g_err.c_str(); }

const char* ot_gs_version(void) { return "otgs 0.1 (gfx950)"; }

}  // extern "C"

extern "C" {

void ot_gs_default_options(ot_gs_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->max_iter = 200;
  o->hist = 10;
  o->refresh = 10;
  o->use_screen = 1;
  o->use_lower = 1;
  o->max_ls = 40;
  o->init_user = 0;
  o->c1 = 1e-4;
  o->c2 = 0.9;
  o->gtol = 0.0;
  o->obj_trace = nullptr;
  o->time_trace = nullptr;
  o->use_graph = 1;
  o->verify = 0;
  o->recenter = 1;
  o->recenter_tol = 1e-9;
}

}  // extern "C"

// ------------------------------------------------------------ solver

// Solver buffers for a history of `hist` pairs.  Without a workspace they are
// allocated by the first solve (again when the history grows); in a
// workspace they were reserved at create for the largest history the
// caller named, and a solve with a shorter history uses a prefix of them.
static int ensure_solver(ot_gs_handle* h, int hist, hipStream_t s) {
  auto& V = h->sol;
  if (V.hist == hist && V.X) return OT_GS_OK;
  V.lb_valid = V.cw_valid = V.xref_used = false;
  if (V.X && h->ws_base) {
    if (hist > V.cap_hist)
      return fail(OT_GS_EINVAL, "solve: hist %d above the %d the workspace was sized for", hist, V.cap_hist);
    HIPCHK(hipStreamSynchronize(s));
    V.hist = hist;
    V.ndot = 5 + 3 * hist;
    HIPCHK(hipMemsetAsync(V.st, 0, sizeof(LbState) * h->count, s));
    HIPCHK(hipMemsetAsync(V.S, 0, sizeof(float) * V.vtot * hist, s));
    HIPCHK(hipMemsetAsync(V.Y, 0, sizeof(float) * V.vtot * hist, s));
    return OT_GS_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  h->free_solver();
  std::vector<long long> voff(h->count);
  long long acc = 0;
  int maxb = 1;
  for (int k = 0; k < h->count; ++k) {
    voff[k] = acc;
    const long long n = (long long)h->inst[k].d.ns + h->inst[k].d.nt_pad;
    acc += n;
    maxb = std::max<int>(maxb, (int)ceil_div(n, LB_VB));
  }
  V.hist = hist;
  V.vtot = acc;
  V.maxb = maxb;
  V.ndot = 5 + 3 * hist;
  V.cap_hist = hist;
  auto al = [&](void** p, size_t bytes) -> int {
    if (h->ws_base) return h->dev_alloc(p, bytes, false);
    h->led_persist += ot_gs_handle::aligned(bytes);
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 8));
    if (e != hipSuccess) return fail(OT_GS_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    V.mem.push_back(*p);
    return OT_GS_OK;
  };
  TRY(al((void**)&V.voff, sizeof(long long) * h->count));
  TRY(al((void**)&V.X, sizeof(float) * acc));
  TRY(al((void**)&V.W, sizeof(float) * acc));
  TRY(al((void**)&V.w_unit, sizeof(int) * h->count));
  TRY(al((void**)&V.G, sizeof(float) * acc));
  TRY(al((void**)&V.Dv, sizeof(float) * acc));
  TRY(al((void**)&V.S, sizeof(float) * acc * hist));
  TRY(al((void**)&V.Y, sizeof(float) * acc * hist));
  TRY(al((void**)&V.st, sizeof(LbState) * h->count));
  TRY(al((void**)&V.agd_st, sizeof(AgdState) * h->count));
  TRY(al((void**)&V.gram, sizeof(double) * 2 * hist * hist * h->count));
  TRY(al((void**)&V.part, sizeof(double) * (size_t)h->count * maxb * V.ndot));
  TRY(al((void**)&V.n_active, 2 * sizeof(int)));
  TRY(al((void**)&V.xref, sizeof(double) * acc));
  TRY(al((void**)&V.obj_const, sizeof(double) * h->count));
  HIPCHK(hipHostMalloc((void**)&V.h_active, 2 * sizeof(int), hipHostMallocDefault));
  HIPCHK(hipMemsetAsync(V.n_active, 0, 2 * sizeof(int), s));
  HIPCHK(hipMemcpyAsync(V.voff, voff.data(), sizeof(long long) * h->count, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(V.w_unit, h->w_unit_h.data(), sizeof(int) * h->count, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(V.st, 0, sizeof(LbState) * h->count, s));
  HIPCHK(hipMemsetAsync(V.S, 0, sizeof(float) * acc * hist, s));
  HIPCHK(hipMemsetAsync(V.Y, 0, sizeof(float) * acc * hist, s));
  {
    const long long maxv = h->max_ns + h->max_ntp;
    hipLaunchKernelGGL(k_lbfgs_weights, dim3((unsigned)std::min<long long>(ceil_div(maxv, 256), 256), h->count),
                       dim3(256), 0, s, h->d_inst, (const long long*)V.voff, (const float*)h->a_int,
                       (const float*)h->b_int, (const int*)h->a_uniform, (const int*)h->b_uniform, V.W);
    LAUNCHCHK();
  }
  return OT_GS_OK;
}

static LbArgs lb_args(ot_gs_handle* h, const LbParams& P) {
  LbArgs A;
  std::memset(&A, 0, sizeof A);
  auto& V = h->sol;
  A.inst = h->d_inst;
  A.P = P;
  A.st = V.st;
  A.inst_mode = h->inst_mode;
  A.n_active = V.n_active;
  A.voff = V.voff;
  A.X = V.X;
  A.G = V.G;
  A.Dv = V.Dv;
  A.S = V.S;
  A.Y = V.Y;
  A.vtot = V.vtot;
  A.alpha = h->alpha;
  A.beta = h->beta;
  A.ga = h->ga;
  A.gb = h->gb;
  A.obj = h->obj;
  A.part = V.part;
  A.maxb = V.maxb;
  A.ndot = V.ndot;
  A.obj_part = h->obj_part;
  A.obj_stride = h->n_asm;
  A.obj_out = h->obj;
  A.gram = V.gram;
  A.alpha_s = h->alpha_s;
  A.beta_s = h->beta_s;
  A.counters = h->counters;
  A.gstats = h->gstats;
  A.g_start = h->g_start;
  A.g_size = h->g_size;
  A.counts = h->counts_dyn;
  A.max_le = h->max_le;
  A.batched = h->count > 1;
  A.W = V.W;
  A.w_unit = V.w_unit;
  A.block_counters = h->block_counters;
  A.n_screen_blocks = h->n_screen_blocks;
  A.n_recenter = V.n_active + 1;
  if (P.recenter) {
    A.xref = V.xref;
    A.obj_const = V.obj_const;
  }
  return A;
}

// The L-BFGS vector update of every instance (with the next evaluation's
// group statistics when `upd`).
static int launch_lbfgs_update(ot_gs_handle* h, const LbArgs& A, bool upd, hipStream_t s) {
  const long long maxv = h->max_ns + h->max_ntp;
  if (upd)
  {
    if (h->gs_large)
      hipLaunchKernelGGL(k_lbfgs_update_gs<GS_LARGE>, dim3((unsigned)(h->max_le + ceil_div(h->max_ntp, GS_LARGE)), h->count),
                         dim3(GS_LARGE), 0, s, A);
    else
      hipLaunchKernelGGL(k_lbfgs_update_gs<GS_SMALL>, dim3((unsigned)(h->max_le + ceil_div(h->max_ntp, GS_SMALL)), h->count),
                         dim3(GS_SMALL), 0, s, A);
  }
  else
    hipLaunchKernelGGL(k_lbfgs_update, dim3((unsigned)std::min<long long>(ceil_div(maxv, 256), 256), h->count),
                       dim3(256), 0, s, A);
  LAUNCHCHK();
  return OT_GS_OK;
}

// One function evaluation of every live instance and one step of its solver.
static int solver_step(ot_gs_handle* h, const LbArgs& A, int use_lower, int use_screen,
                       int init_user, hipStream_t s, bool verify = false) {
  // the control kernel finalises D and the update kernel records snapshots;
  // unscreened solves run every tile of the live instances from the static
  // lists, with no screen pass
  // (with upd_stats the previous step's update formed the group statistics)
  const bool upd = use_screen && h->upd_stats;
  if (use_screen)
    TRY(evaluate_dynamic(h, s, use_lower, nullptr, nullptr, false, false, false, !upd, true));
  else
    TRY(run_tiles_and_reduce(h, false, nullptr, nullptr, s, false, false, false, nullptr));
  if (verify && use_screen) {
    // Lemma 2 checked at every evaluation: the live instances evaluated
    // again densely at the same trial point must give the same bits; the
    // modes go back before the control kernel reads them
    auto& V = h->ver;
    HIPCHK(hipMemcpyAsync(V.ga, h->ga, sizeof(float) * h->tot_rows, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(V.gb, h->gb, sizeof(float) * h->tot_cols_pad, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(V.objp, h->obj_part, sizeof(double) * h->count * h->n_asm, hipMemcpyDeviceToDevice, s));
    const unsigned mb = (unsigned)std::min<long long>(ceil_div(h->count, 256), 64);
    hipLaunchKernelGGL(k_verify_modes, dim3(mb), dim3(256), 0, s, h->inst_mode, V.modes, h->count, 0);
    LAUNCHCHK();
    TRY(run_tiles_and_reduce(h, false, nullptr, nullptr, s, false, false, false, nullptr));
    const long long maxn = std::max<long long>(h->max_ns, h->max_ntp);
    hipLaunchKernelGGL(k_bits_differ, dim3((unsigned)std::min<long long>(ceil_div(maxn, 256), 256), h->count),
                       dim3(256), 0, s, h->d_inst, (const int*)V.modes, 0, V.ga, (const float*)h->ga, V.gb,
                       (const float*)h->gb, V.objp, (const double*)h->obj_part, (long long)h->n_asm, V.diff);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_verify_modes, dim3(mb), dim3(256), 0, s, h->inst_mode, V.modes, h->count, 1);
    LAUNCHCHK();
  }
  hipEvent_t e0 = nullptr;
  TRY(tbegin(h, KT_LBFGS, s, &e0));
  // batches with long vectors: LB_SEQ_SPLIT wavefronts per vector block
  // loop over the history slots (g~ and d read LB_SEQ_SPLIT times instead of
  // once per slot); otherwise one wavefront per (block, slot)
  if (h->count > 1 && h->sol.vtot >= LB_SEQ_MIN_VTOT)
    hipLaunchKernelGGL(k_lbfgs_dots_seq, dim3(h->sol.maxb, h->count, LB_SEQ_SPLIT), dim3(LB_BLOCK), 0, s, A);
  else
    hipLaunchKernelGGL(k_lbfgs_dots, dim3(h->sol.maxb, h->count, 1 + h->sol.hist), dim3(LB_BLOCK), 0, s, A);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_lbfgs_ctrl, dim3(h->count), dim3(64), 0, s, A);
  LAUNCHCHK();
  TRY(launch_lbfgs_update(h, A, upd, s));
  TRY(tend(h, KT_LBFGS, s, e0));
  return OT_GS_OK;
}

// Records `n` calls of step(stream) on the handle's capture stream into an
// executable graph.
template <class Step>
static int capture_n(ot_gs_handle* h, int n, hipGraphExec_t* exec, Step&& step) {
  if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = OT_GS_OK;
  for (int i = 0; i < n && rc == OT_GS_OK; ++i) rc = step(h->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (rc != OT_GS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(OT_GS_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) {
    *exec = nullptr;
    return fail(OT_GS_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e2));
  }
  return OT_GS_OK;
}

// `n` L-BFGS solver steps into an executable graph
static int capture_steps(ot_gs_handle* h, const LbArgs& A, const LbParams& P, int init_user, int n,
                         hipGraphExec_t* exec) {
  return capture_n(h, n, exec, [&](hipStream_t cs) {
    return solver_step(h, A, P.use_lower, P.use_screen, init_user, cs);
  });
}

// One accelerated-ascent step: the evaluation at the current point (screened
// or dense, as for L-BFGS), then dots, control and update.
static int agd_step(ot_gs_handle* h, const AgdArgs& G, int use_lower, int use_screen, hipStream_t s) {
  if (use_screen)
    TRY(evaluate_dynamic(h, s, use_lower, nullptr, nullptr, false, false, true, true, true));
  else
    TRY(run_tiles_and_reduce(h, false, nullptr, nullptr, s, false, false, false, nullptr));
  hipEvent_t e0 = nullptr;
  TRY(tbegin(h, KT_LBFGS, s, &e0));
  const long long maxv = h->max_ns + h->max_ntp;
  hipLaunchKernelGGL(k_agd_dots, dim3(h->sol.maxb, h->count), dim3(LB_BLOCK), 0, s, G);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_agd_ctrl, dim3(h->count), dim3(64), 0, s, G);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_agd_update, dim3((unsigned)std::min<long long>(ceil_div(maxv, 256), 256), h->count),
                     dim3(256), 0, s, G);
  LAUNCHCHK();
  TRY(tend(h, KT_LBFGS, s, e0));
  return OT_GS_OK;
}

// ot_gs_solve with OT_GS_SOLVER_AGD
static int solve_agd(ot_gs_handle* h, const ot_gs_options& o, float* alpha_io, float* beta_io, ot_gs_info* info,
                     hipStream_t s) {
  if (o.verify) return fail(OT_GS_EINVAL, "solve: verify is for L-BFGS solves only");
  TRY(ensure_solver(h, std::max(o.hist, 1), s));
  LbParams P;
  std::memset(&P, 0, sizeof P);
  P.hist = std::max(o.hist, 1);
  P.max_iter = o.max_iter;
  P.max_ls = o.max_ls;
  P.refresh = o.refresh;
  P.use_screen = o.use_screen ? 1 : 0;
  P.use_lower = o.use_lower ? 1 : 0;
  P.c1 = o.c1;
  P.c2 = o.c2;
  P.gtol = o.gtol;
  P.obj_trace = o.obj_trace;
  P.time_trace = o.time_trace;
  P.stats_trace = o.stats_trace;
  P.gnorm_trace = o.gnorm_trace;
  h->sol.lb_valid = h->sol.cw_valid = h->sol.xref_used = false;   // the buffers now hold this solve's vectors
  AgdArgs G;
  std::memset(&G, 0, sizeof G);
  G.A = lb_args(h, P);
  G.st = h->sol.agd_st;
  G.max_bt = o.max_ls;
  G.momentum = 1;
  G.shrink = 0.8;
  TRY(clear_err(h, s));
  if (o.init_user) TRY(gather(h, alpha_io, beta_io, s));
  const long long maxv = h->max_ns + h->max_ntp;
  const dim3 vgrid((unsigned)std::min<long long>(ceil_div(maxv, 256), 256), h->count);
  hipLaunchKernelGGL(k_lbfgs_init, vgrid, dim3(256), 0, s, G.A, o.init_user ? 1 : 0, h->alpha_s, h->beta_s,
                     h->zsnap, h->osnap, h->inN, P.use_screen);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_agd_init, vgrid, dim3(256), 0, s, G);
  LAUNCHCHK();
  h->has_snapshot = P.use_screen != 0;
  // at most 1 + max_ls evaluations per accepted step, plus one at v
  const long long max_steps = 1 + (long long)o.max_iter * (o.max_ls + 2);
  const int check_every = 16;
  hipGraphExec_t exec = nullptr;
  if (o.use_graph && !h->timing.on)
    TRY(capture_n(h, check_every, &exec, [&](hipStream_t cs) { return agd_step(h, G, P.use_lower, P.use_screen, cs); }));
  struct ExecFree {
    hipGraphExec_t& e;
    ~ExecFree() {
      if (e) (void)hipGraphExecDestroy(e);
    }
  } exec_free{exec};
  for (long long step = 0; step < max_steps;) {
    if (exec && step + check_every <= max_steps) {
      HIPCHK(hipGraphLaunch(exec, s));
      step += check_every;
    } else {
      TRY(agd_step(h, G, P.use_lower, P.use_screen, s));
      ++step;
      if (step % check_every != 0 && step != max_steps) continue;
    }
    HIPCHK(hipMemcpyAsync(h->sol.h_active, h->sol.n_active, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h->sol.h_active[0] == 0) break;
  }
  // final points: u_k of every instance (X), back in the caller's order
  hipLaunchKernelGGL(k_lbfgs_export, vgrid, dim3(256), 0, s, G.A);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_scatter_duals, dim3((unsigned)std::min<long long>(ceil_div(maxv, 256), 1024), h->count),
                     dim3(256), 0, s, h->d_inst, h->perm_row, h->perm_col, h->alpha, h->beta, alpha_io, beta_io);
  LAUNCHCHK();
  std::vector<AgdState> hs(h->count);
  HIPCHK(hipMemcpyAsync(hs.data(), h->sol.agd_st, sizeof(AgdState) * h->count, hipMemcpyDeviceToHost, s));
  int herr = 0;
  TRY(sync_err(h, s, &herr));
  int worst = OT_GS_OK;
  for (int k = 0; k < h->count; ++k) {
    int st = OT_GS_NOT_CONVERGED;
    if (hs[k].status == LB_CONVERGED) st = OT_GS_OK;
    else if (hs[k].status == LB_LSFAIL) st = OT_GS_LINESEARCH;
    worst = std::max(worst, st);
    if (info) {
      info[k].iters = hs[k].iter;
      info[k].evals = hs[k].evals;
      info[k].status = st;
      info[k].obj = hs[k].Dk;
      info[k].gnorm_inf = hs[k].gmax;
    }
  }
  if (herr & ERR_NONFINITE) {
    TRY(clear_err(h, s));
    return fail(OT_GS_ENUMERIC, "solve: the starting point holds a NaN or Inf");
  }
  for (int k = 0; k < h->count; ++k)
    if (!std::isfinite(hs[k].Dk)) return fail(OT_GS_ENUMERIC, "solve: the objective of instance %d is not finite", k);
  return worst;
}

extern "C" int ot_gs_solve(ot_gs_handle* h, const ot_gs_options* opts, float* alpha_io,
                           float* beta_io, ot_gs_info* info, void* stream) {
  if (!h || !opts || !alpha_io || !beta_io) return fail(OT_GS_EINVAL, "solve: NULL argument");
  const ot_gs_options& o = *opts;
  if (o.hist < 1 || o.hist > HMAX) return fail(OT_GS_EINVAL, "solve: hist must lie in [1, %d]", HMAX);
  if (o.max_iter < 0 || o.refresh < 1 || o.max_ls < 1)
    return fail(OT_GS_EINVAL, "solve: max_iter >= 0, refresh >= 1, max_ls >= 1 required");
  if (!(o.c1 > 0 && o.c1 < o.c2 && o.c2 < 1)) return fail(OT_GS_EINVAL, "solve: need 0 < c1 < c2 < 1");
  if (o.solver != OT_GS_SOLVER_LBFGS && o.solver != OT_GS_SOLVER_AGD)
    return fail(OT_GS_EINVAL, "solve: unknown solver %d", o.solver);
  if (!(o.recenter_tol >= 0.0)) return fail(OT_GS_EINVAL, "solve: recenter_tol must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  const bool resume = o.resume != 0;
  if (resume && o.solver != OT_GS_SOLVER_LBFGS) return fail(OT_GS_EINVAL, "solve: resume is for L-BFGS solves");
  if (o.solver == OT_GS_SOLVER_AGD) return solve_agd(h, o, alpha_io, beta_io, info, s);
  if (resume) {
    if (!h->sol.lb_valid)
      return fail(OT_GS_EINVAL, "solve: resume needs the state of an L-BFGS solve on the handle "
                                "(a finished solve, or ot_gs_solver_load)");
    if (h->sol.hist != o.hist)
      return fail(OT_GS_EINVAL, "solve: resume needs the state's history size %d (got %d)", h->sol.hist, o.hist);
    if (h->sol.xref_used && !(o.recenter && !h->onthefly))
      return fail(OT_GS_EINVAL, "solve: the state was re-centred; resume it with recenter = 1");
  }
  TRY(ensure_solver(h, o.hist, s));
  LbParams P;
  std::memset(&P, 0, sizeof P);
  P.hist = o.hist;
  P.max_iter = o.max_iter;
  P.max_ls = o.max_ls;
  P.refresh = o.refresh;
  P.use_screen = o.use_screen ? 1 : 0;
  P.use_lower = o.use_lower ? 1 : 0;
  P.c1 = o.c1;
  P.c2 = o.c2;
  P.gtol = o.gtol;
  P.obj_trace = o.obj_trace;
  P.time_trace = o.time_trace;
  P.stats_trace = o.stats_trace;
  P.gnorm_trace = o.gnorm_trace;
  P.recenter = (o.recenter && !h->onthefly) ? 1 : 0;
  P.recenter_tol = o.recenter_tol;
  if (P.recenter) {
    // the evaluations of this solve read a working copy of the pool, which
    // re-centrings rewrite; its cost bounds start as max C
    if (!h->Cw) {
      TRY(h->alloc(&h->Cw, h->c_pool));
      TRY(h->alloc(&h->cmax_w, h->count));
    }
    if (!(resume && h->sol.cw_valid)) {
      HIPCHK(hipMemcpyAsync(h->Cw, h->C, sizeof(float) * h->c_pool, hipMemcpyDeviceToDevice, s));
      std::vector<float> cm(h->count);
      for (int k = 0; k < h->count; ++k) cm[k] = h->inst[k].d.cmax;
      HIPCHK(hipMemcpyAsync(h->cmax_w, cm.data(), sizeof(float) * h->count, hipMemcpyHostToDevice, s));
      if (resume && h->sol.xref_used) {
        // a restored state: its working cost from the reference
        // (fl32(c - xref_i - xref_j), the re-centring's own arithmetic)
        hipLaunchKernelGGL(k_fill<float>, dim3(1), dim3(64), 0, s, h->cmax_w, (long long)h->count, 0.f);
        LAUNCHCHK();
        LbParams P0 = P;
        const LbArgs A0 = lb_args(h, P0);
        const dim3 cg((unsigned)std::min<long long>(ceil_div(h->max_ntp, 256), 8),
                      (unsigned)std::min(h->max_ns, 256), h->count);
        hipLaunchKernelGGL(k_recenter_cost, cg, dim3(256), 0, s, A0, (const float*)h->C, h->Cw,
                           (const int*)h->row_grp, (const int*)h->g_start, (const int*)h->g_size, h->cmax_w, 1);
        LAUNCHCHK();
      }
      HIPCHK(hipStreamSynchronize(s));
    }
    h->C_eval = h->Cw;
    h->cmax_eval = h->cmax_w;
  }
  struct EvalPoolReset {
    ot_gs_handle* h;
    ~EvalPoolReset() {
      h->C_eval = nullptr;
      h->cmax_eval = nullptr;
    }
  } pool_reset{h};
  bool recentered = false;
  LbArgs A = lb_args(h, P);
  const bool verify = o.verify && P.use_screen;
  if (verify) {
    TRY(ensure_verify(h));
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, h->ver.diff, 1LL, 0ull);
    LAUNCHCHK();
  }
  TRY(clear_err(h, s));
  const long long maxv = h->max_ns + h->max_ntp;
  if (resume) {
    // go on from the state: the step the iteration limit cut short, then
    // the update forms the trial point (and the group statistics)
    hipLaunchKernelGGL(k_lbfgs_resume, dim3(h->count), dim3(64), 0, s, A);
    LAUNCHCHK();
    TRY(launch_lbfgs_update(h, A, P.use_screen && h->upd_stats, s));
    h->has_snapshot = P.use_screen != 0;
  } else {
    if (o.init_user) TRY(gather(h, alpha_io, beta_io, s));
    hipLaunchKernelGGL(k_lbfgs_init, dim3((unsigned)std::min<long long>(ceil_div(maxv, 256), 256), h->count),
                       dim3(256), 0, s, A, o.init_user ? 1 : 0, h->alpha_s, h->beta_s, h->zsnap, h->osnap,
                       h->inN, P.use_screen);
    LAUNCHCHK();
    h->has_snapshot = P.use_screen != 0;
    if (P.use_screen && h->upd_stats && h->tot_groups > 0) {
      // statistics of the first evaluation (later ones come from the update)
      ScreenArgs S = screen_args(h, P.use_lower);
      TRY(launch_group_stats(h, S, s));
    }
    h->sol.xref_used = false;
  }
  h->sol.lb_valid = false;   // valid again once this solve has ended
  // upper bound on evaluations: the first one plus max_ls per iteration
  const long long max_steps = 1 + (long long)o.max_iter * o.max_ls;
  const int check_every = 16;
  // the steps between two checks, recorded once into a graph and replayed
  // (every argument is a device pointer or a constant of this solve); not
  // while kernel timing records events
  hipGraphExec_t exec = nullptr;
  if (o.use_graph && !h->timing.on && !verify) TRY(capture_steps(h, A, P, o.init_user, check_every, &exec));
  struct ExecFree {
    hipGraphExec_t& e;
    ~ExecFree() {
      if (e) (void)hipGraphExecDestroy(e);
    }
  } exec_free{exec};
  for (long long step = 0; step < max_steps;) {
    if (exec && step + check_every <= max_steps) {
      HIPCHK(hipGraphLaunch(exec, s));
      step += check_every;
    } else {
      TRY(solver_step(h, A, P.use_lower, P.use_screen, o.init_user, s, verify));
      ++step;
      if (step % check_every != 0 && step != max_steps) continue;
    }
    HIPCHK(hipMemcpyAsync(h->sol.h_active, h->sol.n_active, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h->sol.h_active[1] > 0) {
      // instances whose searches ran out of float32 resolution: re-centre
      // them at their points and let them go on
      recentered = true;
      hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, h->sol.n_active + 1, 1LL, 0);
      LAUNCHCHK();
      hipLaunchKernelGGL(k_recenter_vec, dim3(h->count), dim3(1024), 0, s, A, (const float*)h->a_int,
                         (const float*)h->b_int, (const int*)h->a_uniform, (const int*)h->b_uniform, h->zsnap,
                         h->osnap, h->inN, h->cmax_w);
      LAUNCHCHK();
      // (batches: fewer row workgroups per instance; the instances not being
      // re-centred leave at once, and a grid of 2048 workgroups per instance
      // over 256 instances costs more to dispatch than the re-centred
      // instance's cost takes to rewrite)
      const dim3 cg((unsigned)std::min<long long>(ceil_div(h->max_ntp, 256), 8),
                    (unsigned)std::min(h->max_ns, std::max(16, 256 / h->count)), h->count);
      hipLaunchKernelGGL(k_recenter_cost, cg, dim3(256), 0, s, A, (const float*)h->C, h->Cw, (const int*)h->row_grp,
                         (const int*)h->g_start, (const int*)h->g_size, h->cmax_w, 0);
      LAUNCHCHK();
      hipLaunchKernelGGL(k_recenter_resume, dim3((unsigned)ceil_div(h->count, 256)), dim3(256), 0, s, A, h->count);
      LAUNCHCHK();
      continue;
    }
    if (h->sol.h_active[0] == 0) break;
  }
  // final points: X of every instance, back in the caller's order
  hipLaunchKernelGGL(k_lbfgs_export, dim3((unsigned)std::min<long long>(ceil_div(maxv, 256), 256), h->count),
                     dim3(256), 0, s, A);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_scatter_duals, dim3((unsigned)std::min<long long>(ceil_div(maxv, 256), 1024), h->count),
                     dim3(256), 0, s, h->d_inst, h->perm_row, h->perm_col, h->alpha, h->beta, alpha_io, beta_io);
  LAUNCHCHK();
  h->sol.xref_used = h->sol.xref_used || recentered;
  if (recentered || (resume && h->sol.xref_used)) {
    // the snapshot and N refer to re-centred points and the reduced cost:
    // back to the zero snapshot, exact for the handle's own cost (C >= 0)
    const unsigned fb = (unsigned)std::min<long long>(ceil_div(std::max(h->tot_pairs, h->tot_cols_pad), 256), 4096);
    hipLaunchKernelGGL(k_fill<float>, dim3(fb), dim3(256), 0, s, h->zsnap, h->tot_pairs, 0.f);
    hipLaunchKernelGGL(k_fill<float>, dim3(fb), dim3(256), 0, s, h->osnap, h->tot_pairs, 0.f);
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3(fb), dim3(256), 0, s, h->inN, h->tot_pairs, (uint8_t)0);
    hipLaunchKernelGGL(k_fill<float>, dim3(fb), dim3(256), 0, s, h->alpha_s, h->tot_rows, 0.f);
    hipLaunchKernelGGL(k_fill<float>, dim3(fb), dim3(256), 0, s, h->beta_s, h->tot_cols_pad, 0.f);
    LAUNCHCHK();
  }
  std::vector<LbState> hs(h->count);
  HIPCHK(hipMemcpyAsync(hs.data(), h->sol.st, sizeof(LbState) * h->count, hipMemcpyDeviceToHost, s));
  h->sol.lb_valid = true;
  h->sol.cw_valid = P.recenter != 0;
  unsigned long long diff = 0;
  if (verify) HIPCHK(hipMemcpyAsync(&diff, h->ver.diff, sizeof diff, hipMemcpyDeviceToHost, s));
  int herr = 0;
  TRY(sync_err(h, s, &herr));
  int worst = OT_GS_OK;
  for (int k = 0; k < h->count; ++k) {
    int st = OT_GS_NOT_CONVERGED;
    if (hs[k].status == LB_CONVERGED) st = OT_GS_OK;
    else if (hs[k].status == LB_LSFAIL) st = OT_GS_LINESEARCH;
    worst = std::max(worst, st);
    if (info) {
      info[k].iters = hs[k].iter;
      info[k].evals = hs[k].evals;
      info[k].status = st;
      info[k].obj = -hs[k].f;
      info[k].gnorm_inf = hs[k].gmax;
    }
  }
  if (herr & ERR_NONFINITE) {
    TRY(clear_err(h, s));
    return fail(OT_GS_ENUMERIC, "solve: the starting point holds a NaN or Inf");
  }
  for (int k = 0; k < h->count; ++k)
    if (!std::isfinite(hs[k].f)) return fail(OT_GS_ENUMERIC, "solve: the objective of instance %d is not finite", k);
  if (diff) return fail(OT_GS_EVERIFY, "solve: %llu screened results differed from dense ones", diff);
  return worst;
}
