// CPU stand-in for the HIP runtime and device-code keywords used by the registration library's host
// driver (regnk_host.hip), so that the driver can be compiled with g++ and run against the
// range-checking launch functions of regmock_kernels.cpp (test infrastructure only).  Streams, events
// and graphs are inert handles; graph capture reports "not supported", so the driver takes its
// direct-launch path.  Device-code keywords compile device functions as host code (unused here).
#pragma once
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))
inline void __syncthreads() {}
struct mock_dim3 {
    unsigned x = 0, y = 0, z = 0;
};
static mock_dim3 threadIdx, blockIdx, blockDim, gridDim;
inline double __shfl_xor(double v, int, int) { return v; }

typedef int hipError_t;
enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorNotSupported = 801,
    hipErrorUnknown = 999
};
typedef struct mock_stream* hipStream_t;
typedef struct mock_event* hipEvent_t;
typedef struct mock_graph* hipGraph_t;
typedef struct mock_graph_exec* hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum { hipStreamNonBlocking = 1 };
enum hipStreamCaptureMode { hipStreamCaptureModeThreadLocal = 1 };
enum hipDeviceAttribute_t { hipDeviceAttributeWallClockRate = 1 };

bool mock_range_ok(const void* p, size_t bytes);   // defined by the harness
void mock_fail(const char* what);                  // records an out-of-range access
void mock_register_range(const void* p, size_t bytes);

inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) {
    if (k != hipMemcpyHostToDevice && !mock_range_ok(s, n)) {
        mock_fail("hipMemcpyAsync source");
        return hipErrorInvalidValue;
    }
    if (k != hipMemcpyDeviceToHost && !mock_range_ok(d, n)) {
        mock_fail("hipMemcpyAsync destination");
        return hipErrorInvalidValue;
    }
    std::memmove(d, s, n);
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = reinterpret_cast<hipStream_t>(0x1000);
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
    *g = nullptr;
    return hipErrorNotSupported;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, void*, size_t) { return hipErrorNotSupported; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
inline hipError_t hipEventCreate(hipEvent_t* e) {
    *e = reinterpret_cast<hipEvent_t>(0x2000);
    return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    *ms = 1.0f;
    return hipSuccess;
}
inline hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
    *v = 100000;
    return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t e) { return e ? "rejected by the CPU harness" : "no error"; }
#define HIP_SYMBOL(x) (&(x))
// a device symbol is a host object here: its address, registered as a valid range
template <typename S>
inline hipError_t hipGetSymbolAddress(void** p, S* sym) {
    *p = static_cast<void*>(sym);
    mock_register_range(sym, sizeof(S));
    return hipSuccess;
}
