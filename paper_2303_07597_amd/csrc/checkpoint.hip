// Solver checkpoint: the L-BFGS state of a handle as one host byte string
// (ot_gs_solver_state_size / _save / _load).  Layout: a header naming the
// shapes it belongs to, then the device arrays in a fixed order, each
// copied verbatim (so a restored state continues bit for bit).
#include "otgs_internal.h"

namespace otgs {

struct CkptHeader {
  char magic[8];        // "OTGSLBF1"
  int count, hist;
  int xref_used, pad;
  long long vtot, tot_rows, tot_cols_pad;
  unsigned long long shape_sig;   // instance shapes and parameters
};

// FNV-1a over every instance's (n_src, n_tgt, groups, gamma, mu)
static unsigned long long ckpt_signature(const ot_gs_handle* h) {
  unsigned long long x = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
      x ^= b[i];
      x *= 1099511628211ull;
    }
  };
  for (int k = 0; k < h->count; ++k) {
    const InstDev& d = h->inst[k].d;
    const int v[3] = {d.ns, d.nt, d.Le};
    mix(v, sizeof v);
    mix(&d.gamma64, sizeof d.gamma64);
    mix(&d.thr, sizeof d.thr);
  }
  return x;
}

// the state's device arrays in checkpoint order: pointer and bytes
static std::vector<std::pair<void*, size_t>> ckpt_parts(ot_gs_handle* h) {
  auto& V = h->sol;
  const size_t vt = (size_t)V.vtot, c = (size_t)h->count, hh = (size_t)V.hist;
  return {
      {V.st, sizeof(LbState) * c},
      {V.gram, sizeof(double) * 2 * hh * hh * c},
      {V.X, sizeof(float) * vt},
      {V.G, sizeof(float) * vt},
      {V.Dv, sizeof(float) * vt},
      {V.S, sizeof(float) * vt * hh},
      {V.Y, sizeof(float) * vt * hh},
      {V.xref, sizeof(double) * vt},
      {V.obj_const, sizeof(double) * c},
      {h->inst_mode, sizeof(int) * c},
      {h->alpha, sizeof(float) * (size_t)h->tot_rows},
      {h->beta, sizeof(float) * (size_t)h->tot_cols_pad},
  };
}

static size_t ckpt_bytes(ot_gs_handle* h) {
  size_t n = sizeof(CkptHeader);
  for (auto& p : ckpt_parts(h)) n += p.second;
  return n;
}

}  // namespace otgs

using namespace otgs;

extern "C" {

int ot_gs_solver_state_size(ot_gs_handle* h, size_t* bytes) {
  if (!h || !bytes) return fail(OT_GS_EINVAL, "solver_state_size: NULL argument");
  if (!h->sol.lb_valid) return fail(OT_GS_EINVAL, "solver_state_size: the handle holds no L-BFGS solver state");
  *bytes = ckpt_bytes(h);
  return OT_GS_OK;
}

int ot_gs_solver_save(ot_gs_handle* h, void* host_buf, size_t bytes, void* stream) {
  if (!h || !host_buf) return fail(OT_GS_EINVAL, "solver_save: NULL argument");
  if (!h->sol.lb_valid) return fail(OT_GS_EINVAL, "solver_save: the handle holds no L-BFGS solver state");
  const size_t need = ckpt_bytes(h);
  if (bytes < need) return fail(OT_GS_EINVAL, "solver_save: buffer of %zu bytes, the state needs %zu", bytes, need);
  hipStream_t s = (hipStream_t)stream;
  CkptHeader H;
  std::memset(&H, 0, sizeof H);
  std::memcpy(H.magic, "OTGSLBF1", 8);
  H.count = h->count;
  H.hist = h->sol.hist;
  H.xref_used = h->sol.xref_used ? 1 : 0;
  H.vtot = h->sol.vtot;
  H.tot_rows = h->tot_rows;
  H.tot_cols_pad = h->tot_cols_pad;
  H.shape_sig = ckpt_signature(h);
  unsigned char* out = (unsigned char*)host_buf;
  std::memcpy(out, &H, sizeof H);
  size_t off = sizeof H;
  for (auto& p : ckpt_parts(h)) {
    HIPCHK(hipMemcpyAsync(out + off, p.first, p.second, hipMemcpyDeviceToHost, s));
    off += p.second;
  }
  HIPCHK(hipStreamSynchronize(s));
  return OT_GS_OK;
}

int ot_gs_solver_load(ot_gs_handle* h, const void* host_buf, size_t bytes, void* stream) {
  if (!h || !host_buf) return fail(OT_GS_EINVAL, "solver_load: NULL argument");
  if (bytes < sizeof(CkptHeader)) return fail(OT_GS_EINVAL, "solver_load: %zu bytes hold no state header", bytes);
  CkptHeader H;
  std::memcpy(&H, host_buf, sizeof H);
  if (std::memcmp(H.magic, "OTGSLBF1", 8) != 0) return fail(OT_GS_EINVAL, "solver_load: not a solver state");
  if (H.count != h->count || H.tot_rows != h->tot_rows || H.tot_cols_pad != h->tot_cols_pad ||
      H.shape_sig != ckpt_signature(h))
    return fail(OT_GS_EINVAL, "solver_load: the state belongs to other instances than this handle's");
  if (H.hist < 1 || H.hist > HMAX) return fail(OT_GS_EINVAL, "solver_load: history size %d out of range", H.hist);
  hipStream_t s = (hipStream_t)stream;
  TRY(ensure_solver(h, H.hist, s));
  if (h->sol.vtot != H.vtot) return fail(OT_GS_EINVAL, "solver_load: vector length differs");
  const size_t need = ckpt_bytes(h);
  if (bytes < need) return fail(OT_GS_EINVAL, "solver_load: %zu bytes, the state needs %zu", bytes, need);
  const unsigned char* in = (const unsigned char*)host_buf;
  size_t off = sizeof H;
  for (auto& p : ckpt_parts(h)) {
    HIPCHK(hipMemcpyAsync(p.first, in + off, p.second, hipMemcpyHostToDevice, s));
    off += p.second;
  }
  HIPCHK(hipStreamSynchronize(s));
  h->sol.lb_valid = true;
  h->sol.cw_valid = false;   // the working cost is rebuilt from xref by the resumed solve
  h->sol.xref_used = H.xref_used != 0;
  return OT_GS_OK;
}

}  // extern "C"
