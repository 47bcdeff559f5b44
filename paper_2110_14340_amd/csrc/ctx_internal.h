// Internal access to a context for library modules outside runtime.cpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <map>
#include <vector>

#include "jacc.h"

namespace jr {
bool dry(const jacc_ctx *c);
bool failed(const jacc_ctx *c);           // sticky device error
bool in_batch(const jacc_ctx *c);         // a batch capture is open (no device work may be issued)
hipStream_t stream0(const jacc_ctx *c);   // stream of partition 0
int alloc(jacc_ctx *c, size_t bytes, void **out);
void release(jacc_ctx *c, void *p);
int device_error(jacc_ctx *c, hipError_t e, const char *what);  // makes the context sticky
int error(jacc_ctx *c, int code, const char *msg);
// reason of a failed context-free call, read back by jacc_last_error(NULL)
// on the calling thread
void set_thread_error(const char *msg);
// descriptor, byte size and partition count of the array whose host copy
// starts at `host` (JACC_ERR_NOT_PRESENT when there is none)
int array_info(jacc_ctx *c, const void *host, jacc_array_desc *d, size_t *bytes, int *K);
// the cost model attached to the context (owned by it: `release_model` is
// called at finalize or when another model is attached)
void *attached_model(const jacc_ctx *c);
void attach_model(jacc_ctx *c, void *model, void (*release_model)(void *));
// configuration the attached model picks for a stencil loop run eagerly on
// its arrays' K partitions (fills cfg, returns true), or false
bool model_config(jacc_ctx *c, int kind, const int64_t *extent, int ndim, int K, jacc_config *cfg);
// JACC_TUNE=exhaustive: the context's tuned picks per loop signature, the
// timing database path (empty: none), and the configuration jacc_tune finds
// best among the non-persistent candidates for a stencil loop call at its
// arrays' K (tuned on first sight, outside batches; fills cfg, returns true)
std::map<std::vector<int64_t>, jacc_config> &tuned_picks(jacc_ctx *c);
const char *tune_db(const jacc_ctx *c);
bool tuned_config(jacc_ctx *c, int kind, const jacc_bounds *b, int nargs, const jacc_arg *args,
                  const double *scalars, int nscalars, jacc_config *cfg);
}  // namespace jr
