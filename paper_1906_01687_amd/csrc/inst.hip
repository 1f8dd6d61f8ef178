// inst.hip -- explicit instantiations of the gradient, derivative and batched
// gradient launch templates for one mode count, GCP_INST_D (set on the
// compiler command line).  The build compiles this file once per d = 1..8, so
// the kernels of the eight mode counts compile in parallel.
#include "batched_kernels.hpp"
#include "grad_kernels.hpp"

#ifndef GCP_INST_D
#error "compile inst.hip with -DGCP_INST_D=<mode count>"
#endif

namespace gcp {

template void grad_launch<GCP_INST_D, false>(const GradArgs&, const ScatterPlan&, int, int, hipStream_t, hipEvent_t,
                                             hipEvent_t);
template void grad_launch<GCP_INST_D, true>(const GradArgs&, const ScatterPlan&, int, int, hipStream_t, hipEvent_t,
                                            hipEvent_t);
template void loss_launch<GCP_INST_D>(const LossArgs&, int, int, hipStream_t);
template void batched_grad_launch<GCP_INST_D>(const BatchLaunch&, const BatchGradArgs&, hipStream_t, hipEvent_t,
                                              hipEvent_t);

}  // namespace gcp
