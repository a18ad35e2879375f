// im_host.h -- host-side helpers shared by the translation units of libim.
#pragma once

#include <hip/hip_runtime.h>

#include "im.h"

// record a thread-local error message (returned by im_last_error) and
// return `code`
int im_fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIPCHK(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return im_fail(IM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)
