// Debug fill of stale slab rows (contexts initialised with JACC_INIT_POISON):
// every byte of the range becomes 0xFF, a NaN for FP64 and FP32 elements,
// so a loop that reads rows the runtime left stale carries NaN into its
// output instead of an old value that might pass unnoticed.
#include "jacc.h"
#include "kernels.h"

namespace jk {

namespace {

constexpr int kFillThreads = 256;

__global__ void __launch_bounds__(kFillThreads)
fill_ones_kernel(uint32_t *base, int64_t pitch_words, int64_t width_words, int64_t height) {
    const int64_t n = width_words * height;
    for (int64_t k = (int64_t)blockIdx.x * kFillThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kFillThreads) {
        const int64_t r = k / width_words, w = k - r * width_words;
        base[r * pitch_words + w] = 0xFFFFFFFFu;
    }
}

}  // namespace

hipError_t launch_poison(void *base, size_t pitch_bytes, size_t width_bytes, int64_t height, hipStream_t s) {
    if (width_bytes == 0 || height <= 0) return hipSuccess;
    if (((uintptr_t)base | pitch_bytes | width_bytes) & 3u || width_bytes > pitch_bytes) return hipErrorInvalidValue;
    const int64_t ww = (int64_t)(width_bytes / 4), pw = (int64_t)(pitch_bytes / 4);
    const int64_t blocks = (ww * height + kFillThreads - 1) / kFillThreads;
    const unsigned grid = (unsigned)(blocks < 16384 ? blocks : 16384);
    hipLaunchKernelGGL(fill_ones_kernel, dim3(grid), dim3(kFillThreads), 0, s, (uint32_t *)base, pw, ww, height);
    return hipGetLastError();
}

}  // namespace jk
