// Stencil sweeps for FP64 blocks, FP64 arithmetic.
#define XLS_STENCIL_DEFINE_HOST 1
#include "stencil_impl.h"

namespace xls {
#define XLS_INST_STENCIL(TS, TC)                                                                  \
  template void launch_stencil<TS, TC>(StencilMode, const OpTables<TC>&, const TS*, int64_t, int, \
                                       const TC*, TS*, const TS*, double, double, double,         \
                                       const double*, double*, double*, hipStream_t,               \
                                       const StencilLaunch&, double*);                            \
  template void launch_proj_forward<TS, TC>(const OpTables<TC>&, const TS*, int64_t, int, TC*,    \
                                            hipStream_t);
XLS_INST_STENCIL(double, double)
template void launch_filter_half<double, double>(const OpTables<double>&, const double*, const uint16_t*, int64_t, int64_t,
                                             int, const double*, double*, const uint16_t*, double, double, double,
                                             hipStream_t, const StencilLaunch&);
template void launch_proj_forward<_Float16, double>(const OpTables<double>&, const _Float16*, int64_t, int, double*,
                                                 hipStream_t);
template FilterGroup<double>* filter_group_build<double>(const std::vector<FilterGroupOp<double>>&);
template void filter_group_step<double>(FilterGroup<double>*, int, hipStream_t);
template int filter_group_steps<double>(const FilterGroup<double>*);
template void filter_group_free<double>(FilterGroup<double>*);
}  // namespace xls
