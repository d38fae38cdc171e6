// pf_stage_inst.hip -- instances of the fused stage kernels for one number of
// order parameters, PF_NPHI, and one number of buffer groups, PF_NG (the build
// compiles this file once per supported pair, in parallel; the batched kernel
// uses one group and is built with PF_NG = 1).
#include "pf_stage.hpp"

#if !defined(PF_NPHI) || !defined(PF_NG)
#error "compile with -DPF_NPHI=<number of order parameters> -DPF_NG=<1, 2 or 4>"
#endif

namespace pf {
template hipError_t launch_stage_n<float, PF_NPHI, PF_NG>(int, const StageArgs<float> &, int, hipStream_t);
template hipError_t launch_stage_n<double, PF_NPHI, PF_NG>(int, const StageArgs<double> &, int, hipStream_t);
#if PF_NG == 1
template hipError_t launch_batch_euler_n<float, PF_NPHI>(const BatchArgs<float> &, int, hipStream_t);
template hipError_t launch_batch_euler_n<double, PF_NPHI>(const BatchArgs<double> &, int, hipStream_t);
#endif
}  // namespace pf
