// Stencil sweeps for FP32 blocks, FP32 arithmetic.
#include "stencil_impl.h"

namespace xls {
#define XLS_INST_STENCIL(TS, TC)                                                                  \
  template void launch_stencil<TS, TC>(StencilMode, const OpTables<TC>&, const TS*, int64_t, int, \
                                       const TC*, TS*, const TS*, double, double, double,         \
                                       const double*, double*, double*, hipStream_t,               \
                                       const StencilLaunch&, double*);                            \
  template void launch_proj_forward<TS, TC>(const OpTables<TC>&, const TS*, int64_t, int, TC*,    \
                                            hipStream_t);
XLS_INST_STENCIL(float, float)
template void launch_filter_half<float, float>(const OpTables<float>&, const float*, const uint16_t*, int64_t, int64_t,
                                             int, const float*, float*, const uint16_t*, double, double, double,
                                             hipStream_t, const StencilLaunch&);
template void launch_proj_forward<_Float16, float>(const OpTables<float>&, const _Float16*, int64_t, int, float*,
                                                 hipStream_t);
template FilterGroup<float>* filter_group_build<float>(const std::vector<FilterGroupOp<float>>&);
template void filter_group_step<float>(FilterGroup<float>*, int, hipStream_t);
template int filter_group_steps<float>(const FilterGroup<float>*);
template void filter_group_free<float>(FilterGroup<float>*);
}  // namespace xls
