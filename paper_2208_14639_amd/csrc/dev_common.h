// Device helpers shared by the VV10 kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace vv10 {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 1/x in FP64: hardware estimate refined by two Newton steps
// (each step squares the relative error).  Used only for x > 0 and finite.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    return r;
}

// 1/x in FP32 (hardware estimate, about 1 ulp).
__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }

// Sum over the 64 lanes of a wave in a fixed butterfly order; every lane
// receives the same total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace vv10
