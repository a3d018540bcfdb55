// The sparse plan without device allocations: the per-call scratch of
// ot_gs_plan_csr (segment counts, row totals, segment offsets) lives in one
// fixed device array instead of memory allocated per call, for callers that
// cannot allocate.  Same kernels and results as ot_gs_plan_csr.
#include <mutex>

#include "otgs_internal.h"

namespace otgs {

constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;   // OT_GS_STATIC_SCRATCH_BYTES

// Each GPU the library runs on holds its own copy until the process ends.
// Host code never passes this name to a kernel or a copy: it stands for the
// array only on the device; the host uses the address hipGetSymbolAddress
// gives for the current device.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static void* g_scratch_dev[MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// Device address of the current device's scratch array (looked up once per
// device, with that device current).
static int scratch_ptr(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(OT_GS_EDEVICE, "plan_csr_static: device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(OT_GS_EDEVICE, "plan_csr_static: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return OT_GS_OK;
}

// Exclusive prefix of the row totals into row_ptr[0..rows] by one workgroup
// (each thread a contiguous run of rows, then a scan of the runs), so the
// count call needs no host buffer.
__global__ void __launch_bounds__(1024) k_csr_scan(const long long* __restrict__ tot, long long rows,
                                                   long long* __restrict__ row_ptr) {
  __shared__ long long part[1024];
  const int t = threadIdx.x;
  const long long per = (rows + 1023) / 1024;
  const long long r0 = t * per, r1 = min(rows, r0 + per);
  long long s = 0;
  for (long long i = r0; i < r1; ++i) s += tot[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const long long v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  long long acc = part[t] - s;   // exclusive prefix of this thread's run
  for (long long i = r0; i < r1; ++i) {
    row_ptr[i] = acc;
    acc += tot[i];
  }
  if (t == 1023) row_ptr[rows] = part[1023];
}

}  // namespace otgs

using namespace otgs;

extern "C" int ot_gs_plan_csr_static(ot_gs_handle* h, const float* alpha, const float* beta, long long* row_ptr,
                                     int* col_idx, float* val, long long* nnz, void* stream) {
  if (!h || !alpha || !beta || !row_ptr) return fail(OT_GS_EINVAL, "plan_csr_static: NULL argument");
  if (col_idx ? !val : !nnz)
    return fail(OT_GS_EINVAL, "plan_csr_static: count needs nnz, fill needs col_idx and val");
  long long cstride = 1;
  for (int k = 0; k < h->count; ++k) cstride = std::max<long long>(cstride, h->inst[k].d.njb);
  const long long rows = h->tot_rows;
  // scratch: segment counts (int) at 0, then row totals (count call) or
  // segment offsets (fill call), both int64, 256-byte aligned
  const size_t cnt_bytes = ((size_t)rows * cstride * sizeof(int) + 255) & ~(size_t)255;
  const size_t tail_bytes = (size_t)rows * (col_idx ? cstride : 1) * sizeof(long long);
  if (cnt_bytes + tail_bytes > STATIC_SCRATCH_BYTES)
    return fail(OT_GS_EINVAL,
                "plan_csr_static: needs %zu bytes of scratch (%lld rows x %lld column blocks), more than the "
                "fixed %zu; use ot_gs_plan_csr",
                cnt_bytes + tail_bytes, rows, cstride, STATIC_SCRATCH_BYTES);
  void* base = nullptr;
  TRY(scratch_ptr(&base));
  // no per-kernel timing events in this call (creating them allocates)
  struct TimingOff {
    bool& on;
    bool was;
    ~TimingOff() { on = was; }
  } timing_off{h->timing.on, h->timing.on};
  h->timing.on = false;
  int* cnt = (int*)base;
  long long* tail = (long long*)((unsigned char*)base + cnt_bytes);
  hipStream_t s = (hipStream_t)stream;
  TRY(gather(h, alpha, beta, s));
  TRY(evaluate(h, OT_GS_DENSE, nullptr, nullptr, s, true));
  // every (row, column block) count of the instances is written by the
  // count pass, so nothing left by an earlier call is read
  CsrSink K{cnt, nullptr, cstride, nullptr, nullptr};
  TRY(csr_pass<CSR_COUNT>(h, K, s));
  const dim3 rgrid((unsigned)std::min<long long>(ceil_div(h->max_ns, 256), 1024), h->count);
  if (!col_idx) {
    hipLaunchKernelGGL(k_csr_rowsum, rgrid, dim3(256), 0, s, h->d_inst, (const int*)cnt, cstride, tail);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_csr_scan, dim3(1), dim3(1024), 0, s, (const long long*)tail, rows, row_ptr);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(nnz, row_ptr + rows, sizeof(long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return OT_GS_OK;
  }
  TRY(clear_err(h, s));
  hipLaunchKernelGGL(k_csr_segoff, rgrid, dim3(256), 0, s, h->d_inst, (const int*)cnt, cstride,
                     (const long long*)row_ptr, tail, h->err);
  LAUNCHCHK();
  K.seg = tail;
  K.col = col_idx;
  K.val = val;
  TRY(csr_pass<CSR_FILL>(h, K, s));
  int herr = 0;
  TRY(sync_err(h, s, &herr));
  if (herr & 16)
    return fail(OT_GS_EINVAL, "plan_csr_static: row counts differ from row_ptr (a point other than the count call's)");
  return OT_GS_OK;
}
