// Device helpers shared by the HIP loop bodies (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

constexpr int kWave = 64;

typedef double dvec2 __attribute__((ext_vector_type(2)));

// VEC consecutive doubles from a (16-byte aligned when VEC == 2) address.
template <int VEC>
__device__ __forceinline__ void load_vec(const double *p, double (&v)[VEC]) {
    if constexpr (VEC == 2) {
        const dvec2 t = *reinterpret_cast<const dvec2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    } else {
        v[0] = *p;
    }
}

// Sum of `v` over the 64 lanes of a wave by a fixed butterfly (xor 1, 2, 4,
// ..., 32); every lane ends with the same value.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

// Workgroup sum in a fixed order: wave butterflies, then the wave results
// added in wave order by thread 0.  `sh` holds one double per wave.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nw = (blockDim.x * blockDim.y + kWave - 1) / kWave;
    v = wave_sum(v);
    if ((tid & (kWave - 1)) == 0) sh[tid / kWave] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
        for (int w = 0; w < nw; ++w) s += sh[w];
    return s;  // valid in thread 0
}

}  // namespace jk
