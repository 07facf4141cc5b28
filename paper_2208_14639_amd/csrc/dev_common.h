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

// Barrier for the compiler only: the memory accesses before it are issued
// before those after it.
__device__ __forceinline__ void mem_order() { asm volatile("" ::: "memory"); }

// Adds one tile row's FP32 sums v[0..N) into its FP64 partials y[0], y[16],
// ..., y[16 (N - 1)] (N column blocks of 16); first: y is written, not read.
// Each partial element has a single writer (one lane of one workgroup), so a
// plain read-add-write suffices and the order of the additions, and the
// result, are fixed.  The row's loads are issued together before the adds
// (one wait per row), and rows are added one at a time so that their loads
// do not all occupy registers at once.
template <int N>
__device__ __forceinline__ void add_row(double *y, const float *v, bool first) {
    if (first) {
#pragma unroll
        for (int k = 0; k < N; ++k) y[16 * k] = (double)v[k];
    } else {
        double t[N];
#pragma unroll
        for (int k = 0; k < N; ++k) t[k] = y[16 * k];
#pragma unroll
        for (int k = 0; k < N; ++k) y[16 * k] = t[k] + (double)v[k];
    }
    mem_order();
}

// 1/x in FP32 (hardware estimate, about 1 ulp).
__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }

// The self pair j = i of the inner sums (R = 0, so g = g' = kappa and
// s = g + g' = 2 kappa), in FP64.  Every pair loop, in every mode, leaves
// the self pair out and the kernel that finishes a sum adds it from these
// values: on a coarse grid the self term of a point with a large weight can
// dominate its row, and in FP32 or split-BF16 its rounding would then
// dominate the row's error.
//   phi = Phi_ii, h = 1/s + 1/g, m = 1/s^2 + 1/(s g) + 1/g^2,
//   phig = dPhi/dg = -Phi (1/g + 1/s), phigg = d2Phi/dg dg' = 2 Phi (1/(g g') + 1/s^2).
struct SelfPair {
    double phi, h, m, phig, phigg;
};

__device__ __forceinline__ SelfPair self_pair(double kappa) {
    const double ig = 1.0 / kappa, is = 0.5 * ig;
    SelfPair q;
    q.phi = -1.5 * ig * ig * is;
    q.h = is + ig;
    q.m = is * is + is * ig + ig * ig;
    q.phig = -q.phi * (ig + is);
    q.phigg = 2.0 * q.phi * (ig * ig + is * is);
    return q;
}

// K_pp of the self pair (the p-channel kernel value; K_pq, K_qp, K_qq carry a
// factor R^2 and vanish): Phi + c Phi_g + c Phi_g' + c^2 Phi_gg' with c = rho dkappa/drho.
__device__ __forceinline__ double self_kpp(double kappa, double c) {
    const SelfPair q = self_pair(kappa);
    return q.phi + 2.0 * c * q.phig + c * c * q.phigg;
}

// A mask that clears one bf16 of four packed words: word `word`, its high
// half if `high`, its low half otherwise; all ones when `mine` is false.
__device__ __forceinline__ uint4 bf16_clear_mask(bool mine, int word, bool high) {
    const uint32_t k = high ? 0x0000ffffu : 0xffff0000u;
    return (uint4){mine && word == 0 ? k : 0xffffffffu, mine && word == 1 ? k : 0xffffffffu,
                   mine && word == 2 ? k : 0xffffffffu, mine && word == 3 ? k : 0xffffffffu};
}

template <typename V>
__device__ __forceinline__ V bf16_apply_mask(V v, uint4 k) {
    uint4 u = __builtin_bit_cast(uint4, v);
    u.x &= k.x;
    u.y &= k.y;
    u.z &= k.z;
    u.w &= k.w;
    return __builtin_bit_cast(V, u);
}

// Sum over the 64 lanes of a wave in a fixed butterfly order; every lane
// receives the same total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace vv10
