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

// internal entry points shared between the translation units
struct UndState;                                     // undirected.hip
void und_state_free(UndState *st);
// pair[e] = canonical arc of e's undirected pair (row32: the validated
// 32-bit row offsets); host-synchronous, IM_EINVAL unless symmetric
int und_pair_ids(const im_graph *g, const uint32_t *row32, uint32_t *pair, im_workspace *ws,
                 hipStream_t s);
UndState **im_ws_und(im_workspace *ws);              // im.hip
int im_ws_validate(const im_graph *g, im_workspace *ws, hipStream_t s, uint32_t *row32);
void im_ws_set_last_stream(im_workspace *ws, hipStream_t s);
// exclusive prefix sum of len uint32 values (in and out may not alias);
// sums: scratch of im_scan_sums_len(len) uint32
uint64_t im_scan_sums_len(uint64_t len);
void im_exclusive_scan(const uint32_t *in, uint32_t *out, uint64_t len, uint32_t *sums,
                       hipStream_t s);
