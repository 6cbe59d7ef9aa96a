// Instantiation of the S1 transport stage (FP64; the state solve always runs in FP64); one
// translation unit per stage op so that the many kernel shapes compile in parallel.
#include "transport_kernels.hpp"

namespace regnk {
template hipError_t launch_stage_op<double, OP_S1>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
}  // namespace regnk
