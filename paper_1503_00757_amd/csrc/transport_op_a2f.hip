// Instantiation of the full-Newton A2 incremental-adjoint stage (both precisions); one
// translation unit per stage op so that the many kernel shapes compile in parallel.
#include "transport_kernels.hpp"

namespace regnk {
template hipError_t launch_stage_op<float, OP_A2F>(int, const StageArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_stage_op<double, OP_A2F>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
}  // namespace regnk
