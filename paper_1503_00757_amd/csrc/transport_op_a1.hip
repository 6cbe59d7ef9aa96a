// Instantiation of the A1 transport pass for both precisions (one translation unit per pass op
// so that the many kernel shapes compile in parallel).
#include "transport_kernels.hpp"

namespace regnk {
template hipError_t launch_pass_op<float, OP_A1>(int, int, const PassArgs<float>&, hipStream_t);
template hipError_t launch_pass_op<double, OP_A1>(int, int, const PassArgs<double>&, hipStream_t);
}  // namespace regnk
