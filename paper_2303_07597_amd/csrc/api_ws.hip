// Host side of the learned warm start: the network handle, its training and
// inference calls, the feature builder, and the warm-start entry point of
// include/otgs.h.  Every computation is one of the kernels of mlp.hip.

struct ot_gs_mlp {
  int din = 0, w = 0, max_rows = 0, np = 0;
  long long step = 0;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *dZ1 = nullptr, *dZ2 = nullptr;
  float *out = nullptr, *dout = nullptr, *parts = nullptr;
  double *loss_part = nullptr, *loss = nullptr;
  std::vector<void*> allocs;
  // flat parameter layout: W1 [din, w], b1 [w], W2 [w, w], b2 [w], w3 [w], b3
  long long oW1() const { return 0; }
  long long ob1() const { return (long long)din * w; }
  long long oW2() const { return ob1() + w; }
  long long ob2() const { return oW2() + (long long)w * w; }
  long long ow3() const { return ob2() + w; }
  long long ob3() const { return ow3() + w; }
  template <class T>
  int alloc(T** q, size_t n) {
    void* x = nullptr;
    hipError_t e = hipMalloc(&x, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) return fail(OT_GS_ENOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
    allocs.push_back(x);
    *q = (T*)x;
    return OT_GS_OK;
  }
  ~ot_gs_mlp() {
    for (void* x : allocs) (void)hipFree(x);
  }
};

namespace otgs {

// rows per split-K partial of the weight gradients and per partial of the
// column sums: a 4096-row batch gives 16 x 16 workgroups for a 256 x 256
// weight gradient and 256 x (width / 256) for a column sum, whose partials
// are then added 16 threads per column (one workgroup per partial of 4096
// rows would leave the chip nearly idle)
constexpr int WS_KCHUNK = 256;
constexpr int WS_COLROWS = 16;

static int ws_parts_needed(const ot_gs_mlp* M) {
  const long long nk = ceil_div(M->max_rows, WS_KCHUNK), nc = ceil_div(M->max_rows, WS_COLROWS);
  return (int)std::max(nk * (long long)std::max(M->din, M->w) * M->w, nc * (long long)M->w);
}

static GemmArgs gemm(int Mr, int Nc, int K, const float* A, long long a_rs, long long a_cs, const float* B,
                     long long b_rs, long long b_cs, float* C, long long ldc) {
  GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.M = Mr;
  g.N = Nc;
  g.K = K;
  g.kchunk = K;
  g.A = A;
  g.a_rs = a_rs;
  g.a_cs = a_cs;
  g.B = B;
  g.b_rs = b_rs;
  g.b_cs = b_cs;
  g.C = C;
  g.ldc = ldc;
  return g;
}

static dim3 gemm_grid(const GemmArgs& g, int zparts) {
  return dim3((unsigned)ceil_div(g.N, 64), (unsigned)ceil_div(g.M, 64), (unsigned)zparts);
}

// deep stages for grids of a few hundred workgroups, shallow ones where
// thousands of workgroups hide the latency
template <int EPI>
static int launch_gemm(const GemmArgs& g, dim3 grid, hipStream_t s) {
  if ((long long)grid.x * grid.y * grid.z >= 2048)
    hipLaunchKernelGGL((k_gemm_bf16<EPI, 32>), grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((k_gemm_bf16<EPI, 128>), grid, dim3(256), 0, s, g);
  LAUNCHCHK();
  return OT_GS_OK;
}

// forward of rows [0, n) of F (n <= max_rows): Z1, H1, Z2, H2, out; with y
// also dout and the loss partials (mean over n rows)
static int ws_forward(ot_gs_mlp* M, const float* F, int n, const float* y, float* out, hipStream_t s) {
  const int w = M->w, din = M->din;
  GemmArgs g1 = gemm(n, w, din, F, din, 1, M->p + M->oW1(), w, 1, M->H1, w);
  g1.bias = M->p + M->ob1();
  g1.Z = M->Z1;
  TRY(launch_gemm<EPI_BIAS_GELU>(g1, gemm_grid(g1, 1), s));
  LAUNCHCHK();
  GemmArgs g2 = gemm(n, w, w, M->H1, w, 1, M->p + M->oW2(), w, 1, M->H2, w);
  g2.bias = M->p + M->ob2();
  g2.Z = M->Z2;
  TRY(launch_gemm<EPI_BIAS_GELU>(g2, gemm_grid(g2, 1), s));
  LAUNCHCHK();
  hipLaunchKernelGGL(k_mlp_head, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, (const float*)M->H2,
                     (const float*)(M->p + M->ow3()), (const float*)(M->p + M->ob3()), n, w, out, y,
                     1.0f / (float)n, M->dout, y ? M->loss_part : (double*)nullptr);
  LAUNCHCHK();
  return OT_GS_OK;
}

// column sums of A [n x w] (times wt per row if given) into dst[w]
static int ws_colsum(ot_gs_mlp* M, const float* A, const float* wt, int n, float* dst, hipStream_t s) {
  const int nc = (int)ceil_div(n, WS_COLROWS);
  hipLaunchKernelGGL(k_colsum_parts, dim3((unsigned)ceil_div(M->w, 256), nc), dim3(256), 0, s, A, wt, n, M->w,
                     WS_COLROWS, M->parts);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_sum_parts_wide, dim3((unsigned)ceil_div(M->w, 64)), dim3(1024), 0, s, (const float*)M->parts,
                     nc, (long long)M->w, (long long)M->w, dst);
  LAUNCHCHK();
  return OT_GS_OK;
}

// split-K product into dst (fixed-order sum of the partials)
static int ws_gemm_splitk(ot_gs_mlp* M, GemmArgs g, float* dst, hipStream_t s) {
  const int nz = (int)ceil_div(g.K, WS_KCHUNK);
  g.kchunk = WS_KCHUNK;
  g.C = M->parts;
  g.part_stride = (long long)g.M * g.ldc;
  TRY(launch_gemm<EPI_STORE>(g, gemm_grid(g, nz), s));
  LAUNCHCHK();
  const long long cnt = (long long)g.M * g.ldc;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)std::min<long long>(ceil_div(cnt, 256), 4096)), dim3(256), 0, s,
                     (const float*)M->parts, nz, cnt, cnt, dst);
  LAUNCHCHK();
  return OT_GS_OK;
}

// loss (mean squared error, into M->loss) and its gradient into M->g
static int ws_loss_grad(ot_gs_mlp* M, const float* F, const float* y, int n, hipStream_t s) {
  const int w = M->w, din = M->din;
  TRY(ws_forward(M, F, n, y, M->out, s));
  hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, s, (const double*)M->loss_part, (int)ceil_div(n, 4),
                     1.0 / (double)n, M->loss);
  LAUNCHCHK();
  // output layer
  TRY(ws_colsum(M, M->H2, M->dout, n, M->g + M->ow3(), s));
  hipLaunchKernelGGL(k_sum_vec, dim3(1), dim3(256), 0, s, (const float*)M->dout, n, M->g + M->ob3());
  LAUNCHCHK();
  hipLaunchKernelGGL(k_mlp_dz2, dim3((unsigned)std::min<long long>(ceil_div((long long)n * w, 256), 8192)),
                     dim3(256), 0, s, (const float*)M->dout, (const float*)(M->p + M->ow3()), (const float*)M->Z2,
                     n, w, M->dZ2);
  LAUNCHCHK();
  // second layer: dW2 = H1^T dZ2, db2, dZ1 = (dZ2 W2^T) GELU'(Z1)
  TRY(ws_colsum(M, M->dZ2, nullptr, n, M->g + M->ob2(), s));
  TRY(ws_gemm_splitk(M, gemm(w, w, n, M->H1, 1, w, M->dZ2, w, 1, nullptr, w), M->g + M->oW2(), s));
  GemmArgs gd = gemm(n, w, w, M->dZ2, w, 1, M->p + M->oW2(), 1, w, M->dZ1, w);
  gd.Zin = M->Z1;
  TRY(launch_gemm<EPI_GELU_GRAD>(gd, gemm_grid(gd, 1), s));
  LAUNCHCHK();
  // first layer: dW1 = F^T dZ1, db1
  TRY(ws_colsum(M, M->dZ1, nullptr, n, M->g + M->ob1(), s));
  TRY(ws_gemm_splitk(M, gemm(din, w, n, F, 1, din, M->dZ1, w, 1, nullptr, w), M->g + M->oW1(), s));
  return OT_GS_OK;
}

static int ws_adam(ot_gs_mlp* M, float lr, hipStream_t s) {
  M->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)M->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)M->step)));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)ceil_div(M->np, 256)), dim3(256), 0, s, M->p, M->m, M->v,
                     (const float*)M->g, M->np, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
  LAUNCHCHK();
  return OT_GS_OK;
}

// features of `count` instances into F ([sum n_src + sum n_tgt] x (dim + 8),
// sources of every instance first, then targets)
static int ws_features(const ot_gs_problem* probs, int count, const float* scales, float* F, hipStream_t s) {
  if (!probs || count < 1 || !scales || !F) return fail(OT_GS_EINVAL, "features: bad arguments");
  const int d = probs[0].dim;
  if (d < 1) return fail(OT_GS_EINVAL, "features: dim must be >= 1");
  std::vector<FeatDesc> fd(count);
  long long tot_n = 0, tot_m = 0, tot_c = 0, tot_L = 0;
  int maxL = 1, maxnm = 1;
  for (int k = 0; k < count; ++k) {
    const ot_gs_problem& p = probs[k];
    if (p.dim != d) return fail(OT_GS_EINVAL, "features: instance %d has dim %d, expected %d", k, p.dim, d);
    if (!p.x_src || !p.x_tgt || !p.labels) return fail(OT_GS_EINVAL, "features: instance %d lacks features", k);
    if (p.n_src < 1 || p.n_tgt < 1 || p.n_groups < 1 || p.n_groups > MAX_GROUPS)
      return fail(OT_GS_EINVAL, "features: instance %d has bad sizes", k);
    if (!(scales[k] > 0.f) || !(p.gamma > 0.0) || !(p.mu >= 0.0))
      return fail(OT_GS_EINVAL, "features: instance %d needs scale > 0, gamma > 0, mu >= 0", k);
    tot_n += p.n_src;
    tot_m += p.n_tgt;
  }
  long long tr = tot_n;
  long long sr = 0;
  for (int k = 0; k < count; ++k) {
    const ot_gs_problem& p = probs[k];
    FeatDesc& D = fd[k];
    std::memset(&D, 0, sizeof D);
    D.n = p.n_src;
    D.m = p.n_tgt;
    D.L = p.n_groups;
    D.xs = p.x_src;
    D.xt = p.x_tgt;
    D.labels = p.labels;
    D.src_row = sr;
    D.tgt_row = tr;
    D.cent_off = tot_c;
    D.cls_off = tot_L;
    D.scale = scales[k];
    D.lg = (float)std::log(p.gamma);
    D.lm = (float)std::log(std::max(p.mu, 1e-8));
    sr += p.n_src;
    tr += p.n_tgt;
    tot_c += (long long)p.n_groups * d;
    tot_L += p.n_groups;
    maxL = std::max(maxL, p.n_groups);
    maxnm = std::max(maxnm, p.n_src + p.n_tgt);
  }
  struct Tmp {
    std::vector<void*> v;
    ~Tmp() {
      for (void* x : v) (void)hipFree(x);
    }
  } tmp;
  auto talloc = [&](void** q, size_t bytes) -> int {
    hipError_t e = hipMalloc(q, std::max<size_t>(bytes, 4));
    if (e != hipSuccess) return fail(OT_GS_ENOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
    tmp.v.push_back(*q);
    return OT_GS_OK;
  };
  FeatDesc* dfd;
  float *cs, *ct, *dmin;
  int *cc, *tc, *pseudo;
  TRY(talloc((void**)&dfd, sizeof(FeatDesc) * count));
  TRY(talloc((void**)&cs, sizeof(float) * tot_c));
  TRY(talloc((void**)&ct, sizeof(float) * tot_c));
  TRY(talloc((void**)&cc, sizeof(int) * tot_L));
  TRY(talloc((void**)&tc, sizeof(int) * tot_L));
  TRY(talloc((void**)&pseudo, sizeof(int) * (tot_n + tot_m)));
  TRY(talloc((void**)&dmin, sizeof(float) * (tot_n + tot_m)));
  HIPCHK(hipMemcpyAsync(dfd, fd.data(), sizeof(FeatDesc) * count, hipMemcpyHostToDevice, s));
  const int bd = std::min(256, ((d + 63) / 64) * 64);
  hipLaunchKernelGGL(k_ws_src_centroid, dim3(maxL, count), dim3(bd), 0, s, (const FeatDesc*)dfd, d, cs, cc);
  LAUNCHCHK();
  int maxm = 1;
  for (int k = 0; k < count; ++k) maxm = std::max(maxm, probs[k].n_tgt);
  hipLaunchKernelGGL(k_ws_tgt_assign, dim3((unsigned)ceil_div(maxm, 256), count), dim3(256), 0, s,
                     (const FeatDesc*)dfd, d, (const float*)cs, (const int*)cc, pseudo, dmin);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_ws_tgt_centroid, dim3(maxL, count), dim3(bd), 0, s, (const FeatDesc*)dfd, d,
                     (const int*)pseudo, ct, tc);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_ws_features, dim3((unsigned)ceil_div(maxnm, 256), count), dim3(256), 0, s,
                     (const FeatDesc*)dfd, d, (const float*)cs, (const int*)cc, (const float*)ct, (const int*)tc,
                     (const int*)pseudo, (const float*)dmin, F);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  return OT_GS_OK;
}

static int ws_infer(ot_gs_mlp* M, const float* F, long long n, float* out, hipStream_t s) {
  for (long long r0 = 0; r0 < n; r0 += M->max_rows) {
    const int nb = (int)std::min<long long>(M->max_rows, n - r0);
    TRY(ws_forward(M, F + r0 * M->din, nb, nullptr, out + r0, s));
  }
  return OT_GS_OK;
}

}  // namespace otgs

extern "C" {

int ot_gs_mlp_create(int d_in, int width, int max_rows, ot_gs_mlp** out) {
  if (!out || d_in < 1 || width < 1 || width > 4096 || max_rows < 1)
    return fail(OT_GS_EINVAL, "mlp_create: bad arguments");
  try {
    auto* M = new ot_gs_mlp();
    std::unique_ptr<ot_gs_mlp> guard(M);
    M->din = d_in;
    M->w = width;
    M->max_rows = max_rows;
    M->np = (int)(M->ob3() + 1);
    const size_t act = (size_t)max_rows * width;
    TRY(M->alloc(&M->p, M->np));
    TRY(M->alloc(&M->m, M->np));
    TRY(M->alloc(&M->v, M->np));
    TRY(M->alloc(&M->g, M->np));
    TRY(M->alloc(&M->Z1, act));
    TRY(M->alloc(&M->H1, act));
    TRY(M->alloc(&M->Z2, act));
    TRY(M->alloc(&M->H2, act));
    TRY(M->alloc(&M->dZ1, act));
    TRY(M->alloc(&M->dZ2, act));
    TRY(M->alloc(&M->out, max_rows));
    TRY(M->alloc(&M->dout, max_rows));
    TRY(M->alloc(&M->parts, ws_parts_needed(M)));
    TRY(M->alloc(&M->loss_part, ceil_div(max_rows, 4)));
    TRY(M->alloc(&M->loss, 1));
    HIPCHK(hipMemset(M->p, 0, sizeof(float) * M->np));
    HIPCHK(hipMemset(M->m, 0, sizeof(float) * M->np));
    HIPCHK(hipMemset(M->v, 0, sizeof(float) * M->np));
    *out = guard.release();
    return OT_GS_OK;
  } catch (...) {
    return fail(OT_GS_ENOMEM, "mlp_create: host allocation failed");
  }
}

void ot_gs_mlp_destroy(ot_gs_mlp* M) { delete M; }

int ot_gs_mlp_n_params(const ot_gs_mlp* M) { return M ? M->np : -1; }

int ot_gs_mlp_set_params(ot_gs_mlp* M, const float* params, void* stream) {
  if (!M || !params) return fail(OT_GS_EINVAL, "mlp_set_params: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(M->p, params, sizeof(float) * M->np, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(M->m, 0, sizeof(float) * M->np, s));
  HIPCHK(hipMemsetAsync(M->v, 0, sizeof(float) * M->np, s));
  M->step = 0;
  return OT_GS_OK;
}

int ot_gs_mlp_get_params(ot_gs_mlp* M, float* params, void* stream) {
  if (!M || !params) return fail(OT_GS_EINVAL, "mlp_get_params: NULL argument");
  HIPCHK(hipMemcpyAsync(params, M->p, sizeof(float) * M->np, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return OT_GS_OK;
}

int ot_gs_mlp_forward(ot_gs_mlp* M, const float* F, long long n_rows, float* out, void* stream) {
  if (!M || !F || !out || n_rows < 0) return fail(OT_GS_EINVAL, "mlp_forward: bad arguments");
  return ws_infer(M, F, n_rows, out, (hipStream_t)stream);
}

int ot_gs_mlp_loss_grad(ot_gs_mlp* M, const float* F, const float* y, int n_rows, double* loss,
                        float* grad, void* stream) {
  if (!M || !F || !y || n_rows < 1 || n_rows > M->max_rows)
    return fail(OT_GS_EINVAL, "mlp_loss_grad: bad arguments (1 <= n_rows <= max_rows)");
  hipStream_t s = (hipStream_t)stream;
  TRY(ws_loss_grad(M, F, y, n_rows, s));
  if (loss) HIPCHK(hipMemcpyAsync(loss, M->loss, sizeof(double), hipMemcpyDeviceToDevice, s));
  if (grad) HIPCHK(hipMemcpyAsync(grad, M->g, sizeof(float) * M->np, hipMemcpyDeviceToDevice, s));
  return OT_GS_OK;
}

int ot_gs_mlp_train(ot_gs_mlp* M, const float* F, const float* y, long long n_rows, int batch, int epochs,
                    float lr, double* loss_trace, void* stream) {
  if (!M || !F || !y || n_rows < 1 || batch < 1 || batch > M->max_rows || epochs < 0 || !(lr > 0.f))
    return fail(OT_GS_EINVAL, "mlp_train: bad arguments (1 <= batch <= max_rows, lr > 0)");
  hipStream_t s = (hipStream_t)stream;
  long long t = 0;
  for (int e = 0; e < epochs; ++e)
    for (long long r0 = 0; r0 < n_rows; r0 += batch, ++t) {
      const int nb = (int)std::min<long long>(batch, n_rows - r0);
      TRY(ws_loss_grad(M, F + r0 * M->din, y + r0, nb, s));
      TRY(ws_adam(M, lr, s));
      if (loss_trace) HIPCHK(hipMemcpyAsync(loss_trace + t, M->loss, sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  return OT_GS_OK;
}

int ot_gs_features(const ot_gs_problem* probs, int count, const float* scales, float* F, void* stream) {
  return ws_features(probs, count, scales, F, (hipStream_t)stream);
}

int ot_gs_cost_scale(ot_gs_handle* h, float* scales) {
  if (!h || !scales) return fail(OT_GS_EINVAL, "cost_scale: NULL argument");
  for (int k = 0; k < h->count; ++k) scales[k] = h->inst[k].d.cscale;
  return OT_GS_OK;
}

int ot_gs_warm_start(ot_gs_handle* h, ot_gs_mlp* M, const ot_gs_problem* probs, float* alpha_out,
                     float* beta_out, void* stream) {
  if (!h || !M || !probs || !alpha_out || !beta_out) return fail(OT_GS_EINVAL, "warm_start: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if (M->din != probs[0].dim + 8)
    return fail(OT_GS_EINVAL, "warm_start: the network takes %d inputs, the features have %d", M->din,
                probs[0].dim + 8);
  std::vector<float> sc(h->count);
  TRY(ot_gs_cost_scale(h, sc.data()));
  long long tn = 0, tm = 0;
  for (int k = 0; k < h->count; ++k) {
    tn += probs[k].n_src;
    tm += probs[k].n_tgt;
    if (probs[k].n_src != h->inst[k].d.ns || probs[k].n_tgt != h->inst[k].d.nt)
      return fail(OT_GS_ESHAPE, "warm_start: instance %d does not match the handle", k);
  }
  float *F = nullptr, *o = nullptr;
  HIPCHK(hipMalloc(&F, sizeof(float) * (size_t)(tn + tm) * M->din));
  struct Free {
    float** a;
    float** b;
    ~Free() {
      if (*a) (void)hipFree(*a);
      if (*b) (void)hipFree(*b);
    }
  } fr{&F, &o};
  HIPCHK(hipMalloc(&o, sizeof(float) * (size_t)(tn + tm)));
  TRY(ws_features(probs, h->count, sc.data(), F, s));
  TRY(ws_infer(M, F, tn + tm, o, s));
  HIPCHK(hipMemcpyAsync(alpha_out, o, sizeof(float) * tn, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(beta_out, o + tn, sizeof(float) * tm, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return OT_GS_OK;
}

}  // extern "C"
