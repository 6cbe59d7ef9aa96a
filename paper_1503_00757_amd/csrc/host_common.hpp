// Error reporting shared by the host drivers of the library (the message is what reg_last_error
// returns; it is thread-local).
#pragma once

#include <hip/hip_runtime.h>

#include "regnk.h"

namespace regnk {
// Record a printf-style message for reg_last_error and return s.
reg_status fail(reg_status s, const char* fmt, ...);
}  // namespace regnk

#define CK(call)                                                                               \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::regnk::fail(REG_EDEVICE, "%s failed: %s (%s:%d)", #call,                  \
                                 hipGetErrorString(e_), __FILE__, __LINE__);                   \
    } while (0)

#define CKS(call)                                                                              \
    do {                                                                                       \
        reg_status s_ = (call);                                                                \
        if (s_ != REG_OK) return s_;                                                           \
    } while (0)
