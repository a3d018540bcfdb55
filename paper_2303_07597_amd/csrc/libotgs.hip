// Single translation unit of libotgs (kernels and host code), compiled by
// hipcc for gfx950 into a shared library with the C ABI of include/otgs.h.
#include "layout.hip"
#include "grad.hip"
#include "screen.hip"
#include "lbfgs.hip"
#include "agd.hip"
#include "inspect.hip"
#include "api.hip"
#include "checkpoint.hip"
#include "plan_static.hip"
#include "transport.hip"
#include "mlp.hip"
#include "api_ws.hip"
