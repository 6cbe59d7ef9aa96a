// CPU stand-in for the HIP device-code keywords used by the library's device headers, so that device
// functions can be compiled with g++ and checked on the host (test infrastructure only).  A block is
// emulated by one thread: __syncthreads is a no-op and cross-lane operations are not provided.
#pragma once
#include <cmath>
#include <cstddef>
#include <cstdint>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
inline void __syncthreads() {}
struct mock_dim3 {
    unsigned x = 0, y = 0, z = 0;
};
static mock_dim3 threadIdx, blockIdx, blockDim, gridDim;
inline double __shfl_xor(double v, int, int) { return v; }
typedef int hipError_t;
typedef void* hipStream_t;
