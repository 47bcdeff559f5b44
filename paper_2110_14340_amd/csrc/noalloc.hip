// Allocation-free heat step with fused residual (jacc_heat3d_noalloc).
//
// The same loop body, launch shape and reduction order as a one-partition
// JACC_LOOP_HEAT3D loop with a reduction, on caller-owned device buffers.
// The only memory the step needs beyond its inputs and outputs, the
// workgroup partials of the residual, lives in the file-scope array
// `scratch` below: one copy per device, held until the process ends.  Host
// code never passes `scratch` itself to a kernel (in host code the name is
// a host-side stand-in, not a device address): the device address of each
// device's copy is looked up once with hipGetSymbolAddress, with that device
// current, and kept in `g_scratch`.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx_internal.h"
#include "jacc.h"
#include "kernels.h"

namespace {
// 65,536 workgroup partials (512 KiB per device): with the default
// heat launch (256 columns x 8 rows x 8 planes per workgroup) this covers
// cubes up to 1026^3.
constexpr int64_t kScratchDoubles = JACC_NOALLOC_MAX_PARTIALS;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

int fail(int code, const char *msg) {
    jr::set_thread_error(msg);
    return code;
}

// Device address of the current device's scratch array (looked up on the
// first call on that device).
int device_scratch(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(JACC_ERR_DEVICE, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(JACC_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(JACC_ERR_DEVICE, e != hipSuccess ? hipGetErrorString(e) : "hipGetSymbolAddress gave NULL");
        g_scratch[dev] = (double *)p;
    }
    *out = g_scratch[dev];
    return JACC_OK;
}

// [a, a + na) and [b, b + nb) share a byte
bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace

extern "C" int jacc_heat3d_noalloc(const double *u_in, double *u_out, int64_t nz, int64_t ny, int64_t nx,
                                   double alpha, double *residual, void *stream) {
    if (!u_in || !u_out) return fail(JACC_ERR_INVALID, "NULL field pointer");
    if (nz < 1 || ny < 1 || nx < 1) return fail(JACC_ERR_INVALID, "extents must be positive");
    if (ny > (INT64_MAX / nx) || nz > INT64_MAX / (ny * nx) / (int64_t)sizeof(double))
        return fail(JACC_ERR_INVALID, "extents overflow");
    const int64_t cells = nz * ny * nx;
    const size_t bytes = (size_t)cells * sizeof(double);
    if (overlap(u_in, bytes, u_out, bytes)) return fail(JACC_ERR_INVALID, "u_in and u_out overlap");
    if (residual && (overlap(residual, sizeof(double), u_out, bytes) || overlap(residual, sizeof(double), u_in, bytes)))
        return fail(JACC_ERR_INVALID, "residual overlaps a field");

    jk::Launch L{};
    L.kind = JACC_LOOP_HEAT3D;
    L.ndim = 3;
    L.nargs = 2;
    const int64_t ext[3] = {nz, ny, nx};
    for (int d = 0; d < 3; ++d) {
        L.lo[d] = 1;
        L.hi[d] = ext[d] - 1 > 1 ? ext[d] - 1 : 1;  // an extent below 3 leaves no interior
        L.ext[d] = ext[d];
    }
    L.a[0] = {u_in, 0, nz, ny * nx};
    L.a[1] = {u_out, 0, nz, ny * nx};
    L.scalars[0] = alpha;
    L.part_rows = L.hi[0] - L.lo[0];
    L.cfg = jk::default_config(JACC_LOOP_HEAT3D, L, jk::Cfg{0, 0, 0, 0, 0, 0, 0, 0});
    if (jk::check_config(L) != 0) return fail(JACC_ERR_INVALID, "no valid launch for these extents");
    const int64_t wgs = jk::heat3d_workgroups(L);
    if (wgs > INT32_MAX) return fail(JACC_ERR_RANGE, "grid needs more workgroups than one launch takes");
    if (residual) {
        if (wgs > kScratchDoubles)
            return fail(JACC_ERR_RANGE, "grid needs more workgroup partials than the residual scratch holds");
        double *sp = nullptr;
        int rc = device_scratch(&sp);
        if (rc) return rc;
        L.wg_partials = sp;
        L.wg_capacity = kScratchDoubles;
        L.part_out = residual;
    }
    hipError_t e = jk::launch_loop(L, (hipStream_t)stream);
    if (e != hipSuccess) return fail(JACC_ERR_DEVICE, hipGetErrorString(e));
    return JACC_OK;
}
