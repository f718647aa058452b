// Error reporting and pointer helpers shared by the runtime sources of the
// library (one definition of the per-thread error text).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/xpbd.h"

namespace xpbd {

inline thread_local std::string g_error;

inline xpbd_status fail(xpbd_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::xpbd::fail(XPBD_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

// Device allocation owned by a batch or a network.
struct DeviceBuffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

inline bool is_device_pointer(const void *p)
{
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // plain pageable host memory is not registered
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace xpbd
