// Stencil sweeps for FP32 blocks, FP64 arithmetic (residuals).
#include "stencil_impl.h"

namespace xls {
#define XLS_INST_STENCIL(TS, TC)                                                                  \
  template void launch_stencil<TS, TC>(StencilMode, const OpTables<TC>&, const TS*, int64_t, int, \
                                       const TC*, TS*, const TS*, double, double, double,         \
                                       const double*, double*, double*, hipStream_t,               \
                                       const StencilLaunch&, double*);                            \
  template void launch_proj_forward<TS, TC>(const OpTables<TC>&, const TS*, int64_t, int, TC*,    \
                                            hipStream_t);
XLS_INST_STENCIL(float, double)
}  // namespace xls
