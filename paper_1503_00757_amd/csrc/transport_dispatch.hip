// Dispatch of the transport passes (kernels in transport_kernels.hpp, instantiated per op in
// transport_op_*.hip).
#include "transport_kernels.hpp"

namespace regnk {

#define REGNK_EXTERN_OP(OPN)                                                                              \
    extern template hipError_t launch_pass_op<float, OPN>(int, int, const PassArgs<float>&, hipStream_t); \
    extern template hipError_t launch_pass_op<double, OPN>(int, int, const PassArgs<double>&, hipStream_t);
REGNK_EXTERN_OP(OP_S1)
REGNK_EXTERN_OP(OP_S2)
REGNK_EXTERN_OP(OP_A1)
REGNK_EXTERN_OP(OP_A2)
REGNK_EXTERN_OP(OP_I1)
REGNK_EXTERN_OP(OP_I2)
REGNK_EXTERN_OP(OP_GRAD)
#undef REGNK_EXTERN_OP

template <typename T>
hipError_t launch_pass(int op, int axis, int var, const PassArgs<T>& a, hipStream_t s) {
    switch (op) {
        case OP_S1: return launch_pass_op<T, OP_S1>(axis, var, a, s);
        case OP_S2: return launch_pass_op<T, OP_S2>(axis, var, a, s);
        case OP_A1: return launch_pass_op<T, OP_A1>(axis, var, a, s);
        case OP_A2: return launch_pass_op<T, OP_A2>(axis, var, a, s);
        case OP_I1: return launch_pass_op<T, OP_I1>(axis, var, a, s);
        case OP_I2: return launch_pass_op<T, OP_I2>(axis, var, a, s);
        case OP_GRAD: return launch_pass_op<T, OP_GRAD>(axis, var, a, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_body_end(long nn, T w, const T* lam, const T* G, T* B, hipStream_t s) {
    int blocks = (int)((nn + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((body_end_kernel<T>), dim3(blocks), dim3(256), 0, s, nn, w, lam, G, B);
    return hipGetLastError();
}

template hipError_t launch_pass<float>(int, int, int, const PassArgs<float>&, hipStream_t);
template hipError_t launch_pass<double>(int, int, int, const PassArgs<double>&, hipStream_t);
template hipError_t launch_body_end<float>(long, float, const float*, const float*, float*, hipStream_t);
template hipError_t launch_body_end<double>(long, double, const double*, const double*, double*, hipStream_t);

}  // namespace regnk
