// Internal access to a context for library modules outside runtime.cpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "jacc.h"

namespace jr {
bool dry(const jacc_ctx *c);
bool failed(const jacc_ctx *c);           // sticky device error
hipStream_t stream0(const jacc_ctx *c);   // stream of partition 0
int alloc(jacc_ctx *c, size_t bytes, void **out);
void release(jacc_ctx *c, void *p);
int device_error(jacc_ctx *c, hipError_t e, const char *what);  // makes the context sticky
int error(jacc_ctx *c, int code, const char *msg);
}  // namespace jr
