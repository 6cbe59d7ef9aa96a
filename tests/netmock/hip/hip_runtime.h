// CPU stand-in for the few HIP runtime declarations the network host driver uses, so that the
// driver can be compiled with g++ and run against the bounds-checked CPU kernels of
// netmock_kernels.cpp (test infrastructure only).
#pragma once
#include <cstddef>
#include <cstdint>
#include <cstring>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidConfiguration = 9 };
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };

bool mock_range_ok(const void* p, size_t bytes);   // defined by the harness

inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) {
    if (k != hipMemcpyHostToDevice && !mock_range_ok(s, n)) return hipErrorInvalidValue;
    if (!mock_range_ok(d, n)) return hipErrorInvalidValue;
    std::memcpy(d, s, n);
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t e) { return e ? "out-of-range access in the CPU harness" : "no error"; }
