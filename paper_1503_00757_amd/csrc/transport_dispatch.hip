// Dispatch of the transport stages (kernels in transport_kernels.hpp, instantiated per op in
// transport_op_*.hip) and the pointwise helpers of the state solve.
#include "transport_kernels.hpp"

namespace regnk {

bool stage_variant_fits_f32(int n1, int n2, int var) {
    if (n1 != n2 || !is_pow2_len(n1)) return var == 0;   // two launches with fixed shapes
    switch (n1) {
        case 64: return var_ok<float, 64>(var);
        case 128: return var_ok<float, 128>(var);
        case 256: return var_ok<float, 256>(var);
        case 512: return var_ok<float, 512>(var);
        case 1024: return var_ok<float, 1024>(var);
        case 2048: return var_ok<float, 2048>(var);
    }
    return var == 0;   // short grids: one fixed shape
}

extern template hipError_t launch_stage_op<float, OP_A1>(int, const StageArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<float, OP_A2>(int, const StageArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<float, OP_I1>(int, const StageArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<float, OP_I2>(int, const StageArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<float, OP_A1F>(int, const StageArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<float, OP_A2F>(int, const StageArgs<float>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<double, OP_S1>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<double, OP_S2>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<double, OP_A1>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<double, OP_A2>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<double, OP_I1>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<double, OP_I2>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<double, OP_GRAD>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<double, OP_A1F>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_stage_op<double, OP_A2F>(int, const StageArgs<double>&, hipStream_t, hipEvent_t, hipEvent_t);

template <>
hipError_t launch_stage<float>(int op, int var, const StageArgs<float>& a, hipStream_t s, hipEvent_t t0,
                               hipEvent_t t1) {
    switch (op) {
        case OP_A1: return launch_stage_op<float, OP_A1>(var, a, s, t0, t1);
        case OP_A2: return launch_stage_op<float, OP_A2>(var, a, s, t0, t1);
        case OP_I1: return launch_stage_op<float, OP_I1>(var, a, s, t0, t1);
        case OP_I2: return launch_stage_op<float, OP_I2>(var, a, s, t0, t1);
        case OP_A1F: return launch_stage_op<float, OP_A1F>(var, a, s, t0, t1);
        case OP_A2F: return launch_stage_op<float, OP_A2F>(var, a, s, t0, t1);
    }
    return hipErrorInvalidValue;
}

template <>
hipError_t launch_stage<double>(int op, int var, const StageArgs<double>& a, hipStream_t s, hipEvent_t t0,
                                hipEvent_t t1) {
    switch (op) {
        case OP_S1: return launch_stage_op<double, OP_S1>(var, a, s, t0, t1);
        case OP_S2: return launch_stage_op<double, OP_S2>(var, a, s, t0, t1);
        case OP_A1: return launch_stage_op<double, OP_A1>(var, a, s, t0, t1);
        case OP_A2: return launch_stage_op<double, OP_A2>(var, a, s, t0, t1);
        case OP_I1: return launch_stage_op<double, OP_I1>(var, a, s, t0, t1);
        case OP_I2: return launch_stage_op<double, OP_I2>(var, a, s, t0, t1);
        case OP_GRAD: return launch_stage_op<double, OP_GRAD>(var, a, s, t0, t1);
        case OP_A1F: return launch_stage_op<double, OP_A1F>(var, a, s, t0, t1);
        case OP_A2F: return launch_stage_op<double, OP_A2F>(var, a, s, t0, t1);
    }
    return hipErrorInvalidValue;
}

__global__ void clk_init_kernel(unsigned long long* clk, int pairs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < pairs) {
        clk[2 * i] = ~0ull;
        clk[2 * i + 1] = 0ull;
    }
}

hipError_t launch_clk_init(unsigned long long* clk, int pairs, hipStream_t s) {
    if (pairs < 1) return hipSuccess;
    hipLaunchKernelGGL(clk_init_kernel, dim3((pairs + 255) / 256), dim3(256), 0, s, clk, pairs);
    return hipGetLastError();
}

static inline int pointwise_blocks(long nn) {
    long b = (nn + 255) / 256;
    return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

template <typename T>
hipError_t launch_finalize_state(long nn, const double* Q, const double* C, const double* mR, double* m1, T* lam,
                                 hipStream_t s) {
    hipLaunchKernelGGL((finalize_state_kernel<T>), dim3(pointwise_blocks(nn)), dim3(256), 0, s, nn, Q, C, mR, m1, lam);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_body_end(long nn, T w, const T* Q, const T* C, const T* G, T* B, hipStream_t s) {
    hipLaunchKernelGGL((body_end_kernel<T>), dim3(pointwise_blocks(nn)), dim3(256), 0, s, nn, w, Q, C, G, B);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_body_last(long nn, T w, bool first, const T* Q, const T* C, const T* X, const T* G, const T* G2,
                            T* B, T* keep, hipStream_t s) {
    hipLaunchKernelGGL((body_last_kernel<T>), dim3(pointwise_blocks(nn)), dim3(256), 0, s, nn, w, first, Q, C, X, G,
                       G2, B, keep);
    return hipGetLastError();
}

template hipError_t launch_body_last<float>(long, float, bool, const float*, const float*, const float*,
                                            const float*, const float*, float*, float*, hipStream_t);
template hipError_t launch_body_last<double>(long, double, bool, const double*, const double*, const double*,
                                             const double*, const double*, double*, double*, hipStream_t);
template hipError_t launch_finalize_state<float>(long, const double*, const double*, const double*, double*, float*,
                                                 hipStream_t);
template hipError_t launch_finalize_state<double>(long, const double*, const double*, const double*, double*, double*,
                                                  hipStream_t);
template hipError_t launch_body_end<float>(long, float, const float*, const float*, const float*, float*, hipStream_t);
template hipError_t launch_body_end<double>(long, double, const double*, const double*, const double*, double*,
                                            hipStream_t);

}  // namespace regnk
