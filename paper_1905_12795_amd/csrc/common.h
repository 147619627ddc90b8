// Internal helpers shared by the library's translation units (error state,
// HIP call checking, alignment). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "empso.h"

namespace empso {

void set_error(const char *fmt, ...);
void clear_error();

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace empso

// Evaluate a HIP call; on failure record the message and return EMPSO_EHIP.
#define EMPSO_HIP(call)                                                              \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            empso::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                             __FILE__, __LINE__);                                    \
            return EMPSO_EHIP;                                                       \
        }                                                                            \
    } while (0)

#define EMPSO_FAIL(code, ...)            \
    do {                                 \
        empso::set_error(__VA_ARGS__);   \
        return (code);                   \
    } while (0)
