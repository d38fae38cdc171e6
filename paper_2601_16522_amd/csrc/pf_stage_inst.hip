// pf_stage_inst.hip -- instances of the fused stage kernels for one number of
// order parameters, PF_NPHI (the build compiles this file once per supported
// value, in parallel).
#include "pf_stage.hpp"

#ifndef PF_NPHI
#error "compile with -DPF_NPHI=<number of order parameters>"
#endif

namespace pf {
template hipError_t launch_stage_n<float, PF_NPHI>(int, const StageArgs<float> &, int, hipStream_t);
template hipError_t launch_stage_n<double, PF_NPHI>(int, const StageArgs<double> &, int, hipStream_t);
template hipError_t launch_batch_euler_n<float, PF_NPHI>(const BatchArgs<float> &, int, hipStream_t);
template hipError_t launch_batch_euler_n<double, PF_NPHI>(const BatchArgs<double> &, int, hipStream_t);
}  // namespace pf
