// Perturbation-batched contraction (Section II.B, the pair part of the
// E_{G,G} inner sums), recombined into two well-scaled channels per point:
//
//   Y_i = sum_j K_ij X_j,   X_j = [p_j; q_j] (2 x P), K_ij (2 x 2):
//     K_pp = Phi + c_i Phi_g + c_j Phi_g' + c_i c_j Phi_gg'
//     K_pq = R^2 (Phi_g' + c_i Phi_gg')
//     K_qp = R^2 (Phi_g  + c_j Phi_gg')
//     K_qq = R^4 Phi_gg'
//   with p = w rho^x, q = w rho (omega_r rho^x + omega_g gamma^x),
//   c = rho dkappa/drho, Phi_g = -Phi (1/g + 1/s), Phi_g' = -Phi (1/g' + 1/s),
//   Phi_gg' = 2 Phi (1/(g g') + 1/s^2), s = g + g'.
//
// Summed over i and j, X_i^T K_ij X_j equals the paper's
// sum_ij w_i w_j [rho^A_i (f^{rho rho}_ij rho^B_j + f^{rho gamma}_ij gamma^B_j)
//                + gamma^A_i (f^{gamma rho}_ij rho^B_j + f^{gamma gamma}_ij gamma^B_j)]
// without the delta_ij local terms, which the assembly adds.
//
// This is a dense (2N x 2N) x (2N x P) product whose left operand is never
// stored: every (i, j) pair is formed once, in registers, directly in the
// MFMA A-operand layout.  X chunks are staged in LDS and shared by the waves
// of a workgroup (four, or eight for the split-BF16 form with eight or more
// column blocks); every wave owns 16 outer points and all columns of its
// column group, with accumulators in registers.  Three arithmetic modes:
//
//  FP64:   one pair per lane per 16 x 4 block, four v_mfma_f64_16x16x4 per
//          16 columns (K_pp X_p, K_pq X_q into Y_p; K_qp X_p, K_qq X_q into Y_q).
//  FP32:   the same scheme with v_mfma_f32_16x16x4 and FP32 pair arithmetic.
//  BF16X3: four pairs per lane per 16 x 16 block; the MFMA K index runs over
//          (j, channel), k = 2 (j mod 16) + c, so one v_mfma_f32_16x16x32_bf16
//          contracts K_pp, K_pq (or K_qp, K_qq) of 16 j with both channels of X.
//          Each operand is split as v = hi + lo with hi = bf16(v),
//          lo = bf16(v - hi), and three products hi*hi + hi*lo + lo*hi are
//          accumulated (relative error about 2^-16 per product).
//
// The mixed modes carry the factor -3/2 of Phi in X (the perturbation
// packing scales both channels), so their pair arithmetic forms K / (-3/2)
// with r = 1 / (g g' s) in place of Phi.  Using 1/(g g') = s r and
// 1/s = g g' r, each pair needs one reciprocal and
//   A = r (1/g + 1/s),  A' = r (1/g' + 1/s),  Q = 2 r (1/s^2 + 1/(g g')),
//   t1 = c_i Q - A',  t2 = c_j Q - A,
//   K_pp = r - c_i A + c_j t1,  K_pq = R^2 t1,  K_qp = R^2 t2,  K_qq = R^4 Q.
// They accumulate at most kFp32Run consecutive j points in FP32 (the MFMA
// accumulators) and then add those sums into the split's FP64 partials; the
// assembly sums the partials over splits in FP64.  So the sums are FP32
// within a tile of kFp32Run points and FP64 across tiles and splits.
#include <type_traits>

#include "dev_common.h"
#include "grid_tile.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

constexpr int kJC = 32;   // j points per LDS stage

template <int NCB>
constexpr int smem_f64() { return 2 * kJC * (int)sizeof(double4) + kJC * 2 * NCB * 16 * (int)sizeof(double); }

template <int NCB, bool SCR = false>
__device__ __forceinline__ void tile_f64(int64_t npad, int64_t jlen, int32_t Pp,
                                         const double4 *__restrict__ P0,
                                         const double4 *__restrict__ P1,
                                         const double *__restrict__ X, double *__restrict__ Yout,
                                         int64_t itile, int grp, int split, char *smem,
                                         const uint32_t *__restrict__ mask = nullptr) {
    constexpr int NC = NCB * 16;
    double4 *sA = reinterpret_cast<double4 *>(smem);
    double4 *sB = sA + kJC;
    double *sX = reinterpret_cast<double *>(sB + kJC);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int64_t ibase = itile * 64 + wave * 16;
    const int col0 = grp * NC;
    const int64_t jbeg = (int64_t)split * jlen;
    const int64_t jend = min(npad, jbeg + jlen);
    constexpr int kJJUnroll = SCR ? 1 : 2;   // screened: fewer live registers
    const double4 a0 = P0[ibase + m], a1 = P1[ibase + m];
    const double ci = a1.z;
    v4d accp[NCB], accq[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        accp[cb] = (v4d){0.0, 0.0, 0.0, 0.0};
        accq[cb] = (v4d){0.0, 0.0, 0.0, 0.0};
    }
    for (int64_t j0 = jbeg; j0 < jend; j0 += kJC) {
        __syncthreads();
        if (tid < kJC) {
            sA[tid] = P0[j0 + tid];
            sB[tid] = P1[j0 + tid];
        }
        // rows (j, c) for j in [j0, j0 + kJC), columns [col0, col0 + NC)
        constexpr int H2 = NC / 2;
        for (int e = tid; e < kJC * 2 * H2; e += 256) {
            const int row = e / H2, cc = e - row * H2;
            const double2 v = *reinterpret_cast<const double2 *>(X + (j0 * 2 + row) * Pp + col0 + 2 * cc);
            *reinterpret_cast<double2 *>(sX + row * NC + 2 * cc) = v;
        }
        __syncthreads();
        // the chunk that holds this wave's outer points leaves out the self pair
        const bool diag = ibase < j0 + kJC && ibase + 16 > j0;
        const int dself = diag ? (int)(ibase - j0) + m - kq : -1;
#pragma unroll kJJUnroll
        for (int jj = 0; jj < kJC; jj += 4) {
            const int jl = jj + kq;
            const double4 b0 = sA[jl], b1 = sB[jl];
            const double dx = a0.x - b0.x, dy = a0.y - b0.y, dz = a0.z - b0.z;
            const double R2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
            const double g = __builtin_fma(a0.w, R2, a1.x);
            const double gp = __builtin_fma(b0.w, R2, b1.x);
            const double s = g + gp, t = g * gp;
            const double r = rcp64(t * s);
            const double phi = -1.5 * r;
            const double ig = gp * s * r, igp = g * s * r, is = t * r;
            const double Pg = -phi * (ig + is);
            const double Pgp = -phi * (igp + is);
            const double Pgg = 2.0 * phi * __builtin_fma(ig, igp, is * is);
            const double cj = b1.z;
            const double kpp0 = phi + ci * Pg + cj * __builtin_fma(ci, Pgg, Pgp);
            const double kpp = jj == dself ? 0.0 : kpp0;
            const double kpq = R2 * __builtin_fma(ci, Pgg, Pgp);
            const double kqp = R2 * __builtin_fma(cj, Pgg, Pg);
            const double kqq = R2 * R2 * Pgg;
            const double *xr = sX + (jl * 2) * NC + m;
            const uint32_t mw = SCR ? mask[((j0 + jj) >> 4) * ((Pp >> 4) / NCB) + grp] : 0u;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                if (SCR && !((mw >> cb) & 1u)) continue;
                const double xp = xr[cb * 16];
                accp[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(kpp, xp, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(kqp, xp, accq[cb], 0, 0, 0);
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                if (SCR && !((mw >> cb) & 1u)) continue;
                const double xq = xr[NC + cb * 16];
                accp[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(kpq, xq, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(kqq, xq, accq[cb], 0, 0, 0);
            }
        }
    }
    // D layout of v_mfma_f64_16x16x4 (measured on gfx950): item r of lane l
    // holds row 4 r + l/16, column l%16
    double *Yb = Yout + (int64_t)split * npad * 2 * Pp;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = ibase + 4 * r + kq;
            Yb[(row * 2 + 0) * Pp + col0 + cb * 16 + m] = accp[cb][r];
            Yb[(row * 2 + 1) * Pp + col0 + cb * 16 + m] = accq[cb][r];
        }
}

// ---------------------------------------------------------------------------
// FP32 MFMA
// ---------------------------------------------------------------------------
// The four kernel-derivative values of pair (i, j), divided by -3/2 (see the
// file header); a = (x, y, z, omega), b = (kappa, ., c, .) of each point.
__device__ __forceinline__ void pair_K(const float4 a0, const float4 a1, const float4 b0,
                                       const float4 b1, float &kpp, float &kpq, float &kqp,
                                       float &kqq) {
    const float dx = a0.x - b0.x, dy = a0.y - b0.y, dz = a0.z - b0.z;
    const float R2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const float gg = __builtin_fmaf(a0.w, R2, a1.x);
    const float gp = __builtin_fmaf(b0.w, R2, b1.x);
    const float s = gg + gp, t = gg * gp;
    const float r = rcp32(t * s);
    const float sr = s * r;                           // 1 / (g g')
    const float is = t * r;                           // 1 / s
    const float A = r * __builtin_fmaf(gp, sr, is);   // r (1/g + 1/s)
    const float Ap = r * __builtin_fmaf(gg, sr, is);  // r (1/g' + 1/s)
    const float Q = (r + r) * __builtin_fmaf(is, is, sr);
    const float ci = a1.z, cj = b1.z;
    const float t1 = __builtin_fmaf(ci, Q, -Ap);
    const float t2 = __builtin_fmaf(cj, Q, -A);
    kpp = __builtin_fmaf(cj, t1, __builtin_fmaf(-ci, A, r));
    kpq = R2 * t1;
    kqp = R2 * t2;
    kqq = (R2 * R2) * Q;
}

template <int NCB>
constexpr int smem_f32() { return 2 * kJC * (int)sizeof(float4) + kJC * 2 * NCB * 16 * (int)sizeof(float); }

template <int NCB, bool SCR = false>
__device__ __forceinline__ void tile_f32(int64_t npad, int64_t jlen, int32_t Pp,
                                         const float4 *__restrict__ P0,
                                         const float4 *__restrict__ P1,
                                         const float *__restrict__ X, double *__restrict__ Yout,
                                         int64_t itile, int grp, int split, char *smem,
                                         const uint32_t *__restrict__ mask = nullptr) {
    constexpr int NC = NCB * 16;
    static_assert(kFp32Run % kJC == 0, "FP32 runs end on chunk boundaries");
    float4 *sA = reinterpret_cast<float4 *>(smem);
    float4 *sB = sA + kJC;
    float *sX = reinterpret_cast<float *>(sB + kJC);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int64_t ibase = itile * 64 + wave * 16;
    const int col0 = grp * NC;
    const int64_t jbeg = (int64_t)split * jlen;
    const int64_t jend = min(npad, jbeg + jlen);
    constexpr int kJJUnroll = SCR ? 1 : 2;   // screened: fewer live registers
    const float4 a0 = P0[ibase + m], a1 = P1[ibase + m];
    v4f accp[NCB], accq[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        accp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        accq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
    }
    // D layout of the FP32 MFMAs (measured on gfx950): item r of lane l holds
    // row 4 (l/16) + r, column l%16.  The FP32 sums of each run of kFp32Run
    // points go into this split's FP64 partials.
    double *Yb = Yout + (int64_t)split * npad * 2 * Pp;
    bool first = true;
    auto flush = [&]() {
        // one base address formed here (the empty asm keeps it from being
        // hoisted out of the loop)
        int64_t off = (ibase + 4 * kq) * 2 * Pp + col0 + m;
        asm volatile("" : "+v"(off));
        double *y = Yb + off;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float vp[NCB], vq[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                vp[cb] = accp[cb][r];
                vq[cb] = accq[cb][r];
            }
            add_row<NCB>(y + (2 * r + 0) * (int64_t)Pp, vp, first);
            add_row<NCB>(y + (2 * r + 1) * (int64_t)Pp, vq, first);
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            accp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
            accq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        }
        first = false;
    };
    for (int64_t j0 = jbeg; j0 < jend; j0 += kJC) {
        __syncthreads();
        if (tid < kJC) {
            sA[tid] = P0[j0 + tid];
            sB[tid] = P1[j0 + tid];
        }
        constexpr int H4 = NC / 4;
        for (int e = tid; e < kJC * 2 * H4; e += 256) {
            const int row = e / H4, cc = e - row * H4;
            const float4 v = *reinterpret_cast<const float4 *>(X + (j0 * 2 + row) * Pp + col0 + 4 * cc);
            *reinterpret_cast<float4 *>(sX + row * NC + 4 * cc) = v;
        }
        __syncthreads();
        // the chunk that holds this wave's outer points leaves out the self pair
        const bool diag = ibase < j0 + kJC && ibase + 16 > j0;
        const int dself = diag ? (int)(ibase - j0) + m - kq : -1;
#pragma unroll kJJUnroll
        for (int jj = 0; jj < kJC; jj += 4) {
            const int jl = jj + kq;
            float kpp, kpq, kqp, kqq;
            pair_K(a0, a1, sA[jl], sB[jl], kpp, kpq, kqp, kqq);
            kpp = jj == dself ? 0.f : kpp;
            const float *xr = sX + (jl * 2) * NC + m;
            const uint32_t mw = SCR ? mask[((j0 + jj) >> 4) * ((Pp >> 4) / NCB) + grp] : 0u;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                if (SCR && !((mw >> cb) & 1u)) continue;
                const float xp = xr[cb * 16];
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kpp, xp, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kqp, xp, accq[cb], 0, 0, 0);
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                if (SCR && !((mw >> cb) & 1u)) continue;
                const float xq = xr[NC + cb * 16];
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kpq, xq, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kqq, xq, accq[cb], 0, 0, 0);
            }
        }
        if ((j0 + kJC - jbeg) % kFp32Run == 0 && j0 + kJC < jend) flush();
    }
    flush();
}

// ---------------------------------------------------------------------------
// split-BF16 MFMA
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

struct Aops {          // A operands of one 16 x 16 pair block (per lane: 4 pairs)
    bf16x8 ph, pl, qh, ql;
};

// Split two FP32 values into packed bf16 hi (round to nearest even) and lo
// (the rounded remainder): returns the packed words (v0 in the low half).
// The low half of hi is widened with a byte permute, which keeps the compiler
// from converting v0 a second time.  Contraction is off so that v - hi is a
// plain subtraction in every kernel that inlines this (a product fused into
// it in one kernel and not in another would break bitwise agreement between
// the single-molecule and batched contractions).
__device__ __forceinline__ void split2(float v0, float v1, uint32_t &hi, uint32_t &lo) {
#pragma clang fp contract(off)
    const bf16x2 h = {(__bf16)v0, (__bf16)v1};
    hi = __builtin_bit_cast(uint32_t, h);
    const float h0 = __uint_as_float(__builtin_amdgcn_perm(0u, hi, 0x01000c0cu));   // hi << 16
    const float h1 = __uint_as_float(hi & 0xffff0000u);
    const bf16x2 l = {(__bf16)(v0 - h0), (__bf16)(v1 - h1)};
    lo = __builtin_bit_cast(uint32_t, l);
}

// A operands of the block whose 4 j points of this lane are b0[jj], b1[jj].
__device__ __forceinline__ Aops form_A(const float4 a0, const float4 a1, const float4 *b0,
                                       const float4 *b1) {
    uint32_t ph[4], pl[4], qh[4], ql[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        float kpp, kpq, kqp, kqq;
        pair_K(a0, a1, b0[jj], b1[jj], kpp, kpq, kqp, kqq);
        split2(kpp, kpq, ph[jj], pl[jj]);
        split2(kqp, kqq, qh[jj], ql[jj]);
    }
    Aops A;
    A.ph = __builtin_bit_cast(bf16x8, (uint4){ph[0], ph[1], ph[2], ph[3]});
    A.pl = __builtin_bit_cast(bf16x8, (uint4){pl[0], pl[1], pl[2], pl[3]});
    A.qh = __builtin_bit_cast(bf16x8, (uint4){qh[0], qh[1], qh[2], qh[3]});
    A.ql = __builtin_bit_cast(bf16x8, (uint4){ql[0], ql[1], ql[2], ql[3]});
    return A;
}

// Clear K_pp of the self pair in the A operands of the diagonal block (lane
// (m, g) forms pairs (ibase + m, ibase + 4 g + e), e = 0..3; K_pp is the low
// half of word e of ph and pl).
__device__ __forceinline__ void mask_self(Aops &A, int m, int g) {
    const uint4 k = bf16_clear_mask(g == (m >> 2), m & 3, false);
    A.ph = bf16_apply_mask(A.ph, k);
    A.pl = bf16_apply_mask(A.pl, k);
}

// Software pipeline per wave (four waves and 16-point stages below eight
// column blocks; eight waves and 32-point stages from eight on):
//  * the X of a stage (hi and lo, all columns of the group) is
//    double-buffered in LDS; the next stage's X goes straight from global
//    memory into the other buffer (global_load_lds) while this stage's MFMAs
//    run, and one wait plus one barrier per stage publish it;
//  * the VALU forms the A operands of the next block from point data loaded
//    one block ahead straight from global memory; the instruction scheduler
//    interleaves it with the MFMAs of the current block (measured: forcing a
//    fixed MFMA/VALU interleave, staging point data through LDS or forcing
//    three waves per SIMD were all slower on the 20-water grid).
template <int NCB>
constexpr int smem_bf16x3() { return 2 * 2 * NCB * 16 * 4 * (int)sizeof(bf16x8); }

template <int NCB, bool SCR = false, int WAVES = 4>
__device__ __forceinline__ void tile_bf16x3(int64_t npad, int64_t jlen, int32_t Pp,
                                            const float4 *__restrict__ P0,
                                            const float4 *__restrict__ P1,
                                            const bf16x8 *__restrict__ Xhi,
                                            const bf16x8 *__restrict__ Xlo,
                                            double *__restrict__ Yout, int64_t itile, int grp,
                                            int split, char *smem,
                                            const uint32_t *__restrict__ mask = nullptr,
                                            char *smem2 = nullptr) {
    constexpr int NC = NCB * 16;
    static_assert(kFp32Run % 32 == 0, "FP32 runs end on stage boundaries");
    constexpr int UNITS = NC * 4;                       // 8-bf16 units per block and array
    constexpr int NT = 64 * WAVES;                      // threads of the workgroup
    constexpr int PER = (UNITS + NT - 1) / NT;          // units per thread and array
    typedef bf16x8 Buf[UNITS];
    Buf *sH = reinterpret_cast<Buf *>(smem);            // [buffer][col][g]
    Buf *sL = sH + 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int64_t ibase = itile * (16 * WAVES) + wave * 16;
    const int col0 = grp * NC;
    const int64_t jbeg = (int64_t)split * jlen;
    const int64_t jend = min(npad, jbeg + jlen);
    const float4 a0 = P0[ibase + m], a1 = P1[ibase + m];
    v4f accp[NCB], accq[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        accp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        accq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
    }
    // the FP32 sums of each run of kFp32Run points go into this split's FP64
    // partials (D layout: item r of lane (m, g) is row 4 g + r, column m)
    double *Yb = Yout + (int64_t)split * npad * 2 * Pp;
    bool first = true;
    auto flush = [&]() {
        // one base address formed here (the empty asm keeps it from being
        // hoisted out of the loop: 2 x 4 x NCB addresses would stay live)
        int64_t off = (ibase + 4 * g) * 2 * Pp + col0 + m;
        asm volatile("" : "+v"(off));
        double *y = Yb + off;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float vp[NCB], vq[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                vp[cb] = accp[cb][r];
                vq[cb] = accq[cb][r];
            }
            add_row<NCB>(y + (2 * r + 0) * (int64_t)Pp, vp, first);
            add_row<NCB>(y + (2 * r + 1) * (int64_t)Pp, vq, first);
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            accp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
            accq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        }
        first = false;
    };
    // X of one 16-point block straight from global memory into LDS buffer b
    // (global_load_lds_dwordx4: lane l of a wave writes the 16 bytes at the
    // wave's LDS base + 16 l, so unit e = tid + NT k lands at unit e; the
    // source is a uniform block base plus the lane's unit)
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    auto dma_x = [&](int64_t blk, int b) {
        const int64_t base = ((blk / 16) * Pp + col0) * 4;
        const bf16x8 *bh = Xhi + base, *bl = Xlo + base;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e0 = wv * 64 + NT * k;            // first unit of this wave (uniform)
            if (UNITS % NT == 0 || e0 < UNITS) {        // UNITS is a multiple of 64
                __builtin_amdgcn_global_load_lds(
                    static_cast<const void *>(bh + e0 + lane),
                    reinterpret_cast<__attribute__((address_space(3))) void *>(
                        reinterpret_cast<uintptr_t>(&sH[b][e0])), 16, 0, 0);
                __builtin_amdgcn_global_load_lds(
                    static_cast<const void *>(bl + e0 + lane),
                    reinterpret_cast<__attribute__((address_space(3))) void *>(
                        reinterpret_cast<uintptr_t>(&sL[b][e0])), 16, 0, 0);
            }
        }
    };
    // Screened form: X of a block through registers (loaded before the
    // block's MFMAs, stored to the other buffer after them).  Its pair
    // arithmetic sits between the column blocks' MFMA groups and waits for
    // point data there; with X loads straight into LDS pending, the compiler
    // makes that wait a full one (it treats the load counter as unordered),
    // which also waited for the next block's X (measured with this form at
    // twelve column blocks on the 20-water grid: 52.5 ms that way, 44.9 ms
    // through registers).
    bf16x8 rh[PER], rl[PER];
    auto load_x = [&](int64_t blk) {
        const int64_t base = ((blk / 16) * Pp + col0) * 4;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + NT * k;
            if (e < UNITS) {
                rh[k] = Xhi[base + e];
                rl[k] = Xlo[base + e];
            }
        }
    };
    auto store_x = [&](int b) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + NT * k;
            if (e < UNITS) {
                sH[b][e] = rh[k];
                sL[b][e] = rl[k];
            }
        }
    };
    // point data of this lane's 4 j of a block: j = blk + 4 g + jj
    float4 n0[4], n1[4];
    auto load_pts = [&](int64_t blk) {
        const int64_t jq = min(blk, npad - 16) + 4 * g;   // clamped: never read past npad
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            n0[jj] = P0[jq + jj];
            n1[jj] = P1[jq + jj];
        }
    };
    if constexpr (WAVES == 8) {
        // Stages of 32 points: the X of two 16-point blocks is staged at
        // once and the two blocks' MFMAs run between one pair of barriers.
        // The A operands alternate between two register sets, each formed
        // while the other's MFMAs run.
        // The two stage buffers are distinct LDS arrays (smem: buffer 0,
        // smem2: buffer 1), each hi then lo of two 16-point blocks; with the
        // stages unrolled in pairs the compiler sees that a stage's LDS reads
        // and its loads into the other buffer never alias, and waits for
        // those loads only at the stage's end.
        typedef bf16x8 Buf2[2 * UNITS];                 // [sub-block][col][g]
        Buf2 &H0 = *reinterpret_cast<Buf2 *>(smem), &L0 = *(reinterpret_cast<Buf2 *>(smem) + 1);
        Buf2 &H1 = *reinterpret_cast<Buf2 *>(smem2), &L1 = *(reinterpret_cast<Buf2 *>(smem2) + 1);
        constexpr int PER2 = (2 * UNITS + NT - 1) / NT;
        // X of points j .. j + 31 straight from global memory into LDS
        // (global_load_lds_dwordx4: lane l of a wave writes the 16 bytes at
        // the wave's LDS base + 16 l, so unit e = tid + NT k lands at unit e).
        // The source of piece k is a stage base (uniform, in SGPRs) plus a
        // per-lane 32-bit offset fixed over the stages; the LDS base is
        // uniform too, so a piece costs no 64-bit address arithmetic.
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        uint32_t xoff[PER2];
#pragma unroll
        for (int k = 0; k < PER2; ++k) {
            const int e = wv * 64 + NT * k + lane;
            const int sub = e >= UNITS;
            xoff[k] = (uint32_t)(sub * Pp * 4 + (e - sub * UNITS));
        }
        auto load2 = [&](int64_t j, Buf2 &H, Buf2 &L) {
            const int64_t base = ((j / 16) * Pp + col0) * 4;
            const bf16x8 *bh = Xhi + base, *bl = Xlo + base;
#pragma unroll
            for (int k = 0; k < PER2; ++k) {
                const int e0 = wv * 64 + NT * k;        // first unit of this wave (uniform)
                // 2 UNITS is a multiple of 64; when it is one of NT, every
                // wave loads PER2 pieces
                if ((2 * UNITS) % NT == 0 || e0 < 2 * UNITS) {
                    __builtin_amdgcn_global_load_lds(
                        static_cast<const void *>(bh + xoff[k]),
                        reinterpret_cast<__attribute__((address_space(3))) void *>(
                            reinterpret_cast<uintptr_t>(&H[e0])), 16, 0, 0);
                    __builtin_amdgcn_global_load_lds(
                        static_cast<const void *>(bl + xoff[k]),
                        reinterpret_cast<__attribute__((address_space(3))) void *>(
                            reinterpret_cast<uintptr_t>(&L[e0])), 16, 0, 0);
                }
            }
        };
        // screened: a column block whose mask bit is clear skips its MFMAs
        // (the mask word of the 16-point block at jb)
        auto mfmas = [&](const Aops &A, const bf16x8 *hp, const bf16x8 *lp, int64_t jb) {
            uint32_t mw = ~0u;
            if constexpr (SCR) mw = mask[(jb >> 4) * ((Pp >> 4) / NCB) + grp];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                if (SCR && !((mw >> cb) & 1u)) continue;
                const bf16x8 bh = hp[cb * 64], bl = lp[cb * 64];
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.ph, bh, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.qh, bh, accq[cb], 0, 0, 0);
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.pl, bh, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.ql, bh, accq[cb], 0, 0, 0);
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.ph, bl, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.qh, bl, accq[cb], 0, 0, 0);
            }
        };
        load_pts(jbeg);
        load2(jbeg, H0, L0);
        Aops cur = form_A(a0, a1, n0, n1);
        load_pts(jbeg + 16);
        __builtin_amdgcn_s_waitcnt(0);   // this wave's LDS loads are done
        __syncthreads();
        // one 32-point stage on buffer (Hc, Lc), loading the next into (Hn, Ln)
        auto stage = [&](int64_t j0, Buf2 &Hc, Buf2 &Lc, Buf2 &Hn, Buf2 &Ln) {
            if (j0 + 32 < jend) load2(j0 + 32, Hn, Ln);   // every wave finished reading it
            // the diagonal block: the self pair (i, i) of lane (m, g = m/4) is
            // its pair m mod 4, whose K_pp (the low half of word m mod 4 of ph,
            // pl) is cleared; K_pq, K_qp, K_qq vanish there (R = 0)
            if (j0 == ibase) mask_self(cur, m, g);
            Aops alt = form_A(a0, a1, n0, n1);      // points j0 + 16 ..
            load_pts(j0 + 32);
            mfmas(cur, Hc + m * 4 + g, Lc + m * 4 + g, j0);
            if (j0 + 16 == ibase) mask_self(alt, m, g);
            cur = form_A(a0, a1, n0, n1);           // points j0 + 32 ..
            load_pts(j0 + 48);
            mfmas(alt, Hc + UNITS + m * 4 + g, Lc + UNITS + m * 4 + g, j0 + 16);
            __builtin_amdgcn_s_waitcnt(0);   // this wave's LDS loads of the next stage
            __syncthreads();
        };
        // a split holds a whole number of 32-point stages (jbeg and jlen are
        // multiples of 32, npad of 256)
        static_assert(kFp32Run % 64 == 0, "FP32 runs end on stage pairs");
        for (int64_t j0 = jbeg; j0 < jend; j0 += 64) {
            stage(j0, H0, L0, H1, L1);
            if (j0 + 32 < jend) stage(j0 + 32, H1, L1, H0, L0);
            if ((j0 + 64 - jbeg) % kFp32Run == 0 && j0 + 64 < jend) flush();
        }
    } else {
    load_pts(jbeg);
    if constexpr (SCR) {
        load_x(jbeg);
        store_x(0);
    } else {
        dma_x(jbeg, 0);
    }
    Aops cur = form_A(a0, a1, n0, n1);
    load_pts(jbeg + 16);
    __builtin_amdgcn_s_waitcnt(0);   // this wave's LDS loads are done
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jbeg; j0 < jend; j0 += 16) {
        // the diagonal block: the self pair (i, i) of lane (m, g = m/4) is its
        // pair m mod 4, whose K_pp (the low half of word m mod 4 of ph, pl) is
        // cleared; K_pq, K_qp, K_qq vanish there (R = 0)
        if (j0 == ibase) mask_self(cur, m, g);
        const bool more = j0 + 16 < jend;
        if (more) {
            if constexpr (SCR) load_x(j0 + 16);
            else dma_x(j0 + 16, buf ^ 1);   // every wave finished reading it
        }
        const bf16x8 *hp = sH[buf] + m * 4 + g;
        const bf16x8 *lp = sL[buf] + m * 4 + g;
        Aops nxt;
        if constexpr (!SCR) {
            nxt = form_A(a0, a1, n0, n1);
            load_pts(j0 + 32);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const bf16x8 bh = hp[cb * 64], bl = lp[cb * 64];
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ph, bh, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.qh, bh, accq[cb], 0, 0, 0);
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.pl, bh, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ql, bh, accq[cb], 0, 0, 0);
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ph, bl, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.qh, bl, accq[cb], 0, 0, 0);
            }
        } else {
            // Screened: the skipped blocks are branches, which the compiler
            // does not schedule across, so the next block's A operands are
            // formed one pair at a time between the column blocks' MFMA
            // groups (the MFMAs in flight overlap the pair arithmetic).
            const uint32_t mw = mask[(j0 >> 4) * ((Pp >> 4) / NCB) + grp];
            uint32_t ph[4], pl[4], qh[4], ql[4];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                if ((mw >> cb) & 1u) {
                    const bf16x8 bh = hp[cb * 64], bl = lp[cb * 64];
                    accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ph, bh, accp[cb], 0, 0, 0);
                    accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.qh, bh, accq[cb], 0, 0, 0);
                    accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.pl, bh, accp[cb], 0, 0, 0);
                    accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ql, bh, accq[cb], 0, 0, 0);
                    accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ph, bl, accp[cb], 0, 0, 0);
                    accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.qh, bl, accq[cb], 0, 0, 0);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    if (jj * NCB / 4 != cb) continue;      // pair jj after column block jj NCB/4
                    // empty asm statements pin the pair arithmetic to this
                    // point (after this column block's MFMAs are issued)
                    asm volatile("" : "+v"(n0[jj].x), "+v"(n0[jj].y), "+v"(n0[jj].z), "+v"(n0[jj].w),
                                 "+v"(n1[jj].x), "+v"(n1[jj].z));
                    float kpp, kpq, kqp, kqq;
                    pair_K(a0, a1, n0[jj], n1[jj], kpp, kpq, kqp, kqq);
                    split2(kpp, kpq, ph[jj], pl[jj]);
                    split2(kqp, kqq, qh[jj], ql[jj]);
                    asm volatile("" ::"v"(ph[jj]), "v"(pl[jj]), "v"(qh[jj]), "v"(ql[jj]));
                }
            }
            nxt.ph = __builtin_bit_cast(bf16x8, (uint4){ph[0], ph[1], ph[2], ph[3]});
            nxt.pl = __builtin_bit_cast(bf16x8, (uint4){pl[0], pl[1], pl[2], pl[3]});
            nxt.qh = __builtin_bit_cast(bf16x8, (uint4){qh[0], qh[1], qh[2], qh[3]});
            nxt.ql = __builtin_bit_cast(bf16x8, (uint4){ql[0], ql[1], ql[2], ql[3]});
            load_pts(j0 + 32);
        }
        cur = nxt;
        if constexpr (SCR) {
            if (more) store_x(buf ^ 1);
        }
        if ((j0 + 16 - jbeg) % kFp32Run == 0 && more) flush();
        __builtin_amdgcn_s_waitcnt(0);   // this wave's LDS loads of the next block
        __syncthreads();
        buf ^= 1;
    }
    }
    flush();
}

// One workgroup per (i tile, column group, j split): blockIdx = (tile, group, split).
// SCR: skip the (16-point, 16-column) blocks that the screening mask marks
// inactive (the MFMA work only; the kernel tile is still formed).
template <int NCB, bool SCR>
__global__ __launch_bounds__(256, 2) void k_contract_f64(int64_t npad, int64_t jlen, int32_t Pp,
                                                         const double4 *__restrict__ P0,
                                                         const double4 *__restrict__ P1,
                                                         const double *__restrict__ X,
                                                         double *__restrict__ Yout,
                                                         const uint32_t *__restrict__ mask) {
    __shared__ __attribute__((aligned(16))) char smem[smem_f64<NCB>()];
    tile_f64<NCB, SCR>(npad, jlen, Pp, P0, P1, X, Yout, blockIdx.x, blockIdx.y, blockIdx.z, smem,
                       mask);
}

template <int NCB, bool SCR>
__global__ __launch_bounds__(256, 2) void k_contract_f32(int64_t npad, int64_t jlen, int32_t Pp,
                                                         const float4 *__restrict__ P0,
                                                         const float4 *__restrict__ P1,
                                                         const float *__restrict__ X,
                                                         double *__restrict__ Yout,
                                                         const uint32_t *__restrict__ mask) {
    __shared__ __attribute__((aligned(16))) char smem[smem_f32<NCB>()];
    tile_f32<NCB, SCR>(npad, jlen, Pp, P0, P1, X, Yout, blockIdx.x, blockIdx.y, blockIdx.z, smem,
                       mask);
}

// Waves (16 outer points each) of the standalone split-BF16 kernel, by
// column blocks: with eight or more blocks the MFMA work per pair dominates
// and eight waves share each staged X block in 32-point stages (one barrier
// per two MFMA blocks: 56.5 -> 53.0 ms on the 20-water grid); with fewer,
// four waves in 16-point stages keep three to four waves per SIMD (the
// 32-point stages' registers would drop it to two).  Screened, the
// eight-wave form skips a column block's MFMAs behind a branch (its MFMA and
// VALU work do not overlap anyway: screened 20-water contraction 37.3 ms,
// against 45.0 in the four-wave screened form and 49-50 unscreened).
template <int NCB>
constexpr int bf16_waves() { return NCB >= kWideMinNcb ? 8 : 4; }

template <int NCB, bool SCR>
__global__ __launch_bounds__(64 * bf16_waves<NCB>(), 8 / bf16_waves<NCB>()) void k_contract_bf16x3(int64_t npad, int64_t jlen, int32_t Pp,
                                                            const float4 *__restrict__ P0,
                                                            const float4 *__restrict__ P1,
                                                            const bf16x8 *__restrict__ Xhi,
                                                            const bf16x8 *__restrict__ Xlo,
                                                            double *__restrict__ Yout,
                                                            const uint32_t *__restrict__ mask) {
    __shared__ __attribute__((aligned(16))) char smem[smem_bf16x3<NCB>()];
    // the second stage buffer of the eight-wave form (a one-byte dummy otherwise)
    __shared__ __attribute__((aligned(16))) char smem2[bf16_waves<NCB>() == 8 ? smem_bf16x3<NCB>() : 1];
    tile_bf16x3<NCB, SCR, bf16_waves<NCB>()>(npad, jlen, Pp, P0, P1, Xhi, Xlo, Yout,
                                             blockIdx.x, blockIdx.y, blockIdx.z, smem, mask,
                                             smem2);
}

template <int NCB, bool SCR>
hipError_t run_mode(vv10_plan *p, const Workspace &ws) {
    dim3 grid((unsigned)(p->npad / 64), (unsigned)ws.ngroups, (unsigned)ws.jsplit);
    const uint32_t *mask = SCR ? ws.mask : nullptr;
    if (p->prec == VV10_FP64) {
        if constexpr (NCB <= 8)
            k_contract_f64<NCB, SCR><<<grid, 256, 0, p->stream>>>(
                p->npad, ws.jlen, ws.Pp, p->P0, p->P1, static_cast<const double *>(ws.X),
                static_cast<double *>(ws.Ypart), mask);
        else
            return hipErrorInvalidValue;
    } else if (p->prec == VV10_MIXED_FP32) {
        k_contract_f32<NCB, SCR><<<grid, 256, 0, p->stream>>>(
            p->npad, ws.jlen, ws.Pp, p->P0f, p->P1f, static_cast<const float *>(ws.X),
            static_cast<double *>(ws.Ypart), mask);
    } else {
        const bf16x8 *xh = static_cast<const bf16x8 *>(ws.X);
        const bf16x8 *xl = xh + (size_t)p->npad * ws.Pp * 2 / 8;
        constexpr int W = bf16_waves<NCB>();
        dim3 gridb((unsigned)(p->npad / (16 * W)), (unsigned)ws.ngroups, (unsigned)ws.jsplit);
        k_contract_bf16x3<NCB, SCR><<<gridb, 64 * W, 0, p->stream>>>(
            p->npad, ws.jlen, ws.Pp, p->P0f, p->P1f, xh, xl, static_cast<double *>(ws.Ypart), mask);
    }
    return hipGetLastError();
}

template <int NCB>
hipError_t run(vv10_plan *p, const Workspace &ws, bool screen) {
    return screen ? run_mode<NCB, true>(p, ws) : run_mode<NCB, false>(p, ws);
}

template <int NCB>
int occupancy(vv10_precision prec) {
    int nb = 0;
    hipError_t e;
    if (prec == VV10_FP64) {
        if constexpr (NCB <= 8)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_contract_f64<NCB, false>, 256, 0);
        else
            return 0;
    } else if (prec == VV10_MIXED_FP32) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_contract_f32<NCB, false>, 256, 0);
    } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_contract_bf16x3<NCB, false>,
                                                         64 * bf16_waves<NCB>(), 0);
        nb *= bf16_waves<NCB>() / 4;   // in units of 64-point tiles, as the other modes
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

template <typename F>
auto dispatch_ncb(int ncb, F &&f) -> decltype(f(std::integral_constant<int, 1>{})) {
    switch (ncb) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 5: return f(std::integral_constant<int, 5>{});
        case 6: return f(std::integral_constant<int, 6>{});
        case 7: return f(std::integral_constant<int, 7>{});
        case 8: return f(std::integral_constant<int, 8>{});
        case 9: return f(std::integral_constant<int, 9>{});
        case 10: return f(std::integral_constant<int, 10>{});
        case 11: return f(std::integral_constant<int, 11>{});
        case 12: return f(std::integral_constant<int, 12>{});
        default: return decltype(f(std::integral_constant<int, 1>{})){};
    }
}

// ---------------------------------------------------------------------------
// Persistent batched kernels: a fixed grid of workgroups pulls work items
// from an integer counter, one list and counter per kernel, each list
// largest first.  A contraction item is (molecule, i tile, column group,
// j split); a grid item is one grid-pass tile of one molecule for one atom
// group (the grid-position intermediates and the pair integrals).  Every
// item writes its own output slab, so the results do not depend on which
// workgroup ran which item.
// ---------------------------------------------------------------------------
template <int PREC>
struct PersistentTraits;
template <>
struct PersistentTraits<VV10_FP64> {
    static constexpr int kMaxNcb = 8;
    static constexpr int kSmem = smem_f64<8>();
    static constexpr int kWaves = 4;
};
template <>
struct PersistentTraits<VV10_MIXED_FP32> {
    static constexpr int kMaxNcb = 12;
    static constexpr int kSmem = smem_f32<12>();
    static constexpr int kWaves = 4;
};
template <>
struct PersistentTraits<VV10_MIXED_BF16X3> {
    // four waves: the eight-wave form of the standalone kernel (32-point
    // stages, X straight into two LDS buffers) spilled 32 registers here
    // when every column count shared one register allocation and was slower
    // on the 64-cluster batch (2.95 s per launch against 2.86 s); molecules
    // with kWideMinNcb or more blocks per group run it in a kernel of their
    // own (k_contract_persistent_wide), so this one serves the narrower
    // counts only, whose smaller register allocation leaves room for more
    // waves per SIMD
    static constexpr int kMaxNcb = kWideMinNcb - 1;
    static constexpr int kSmem = smem_bf16x3<kWideMinNcb - 1>();
    static constexpr int kWaves = 4;
};

template <int PREC, int NCB>
__device__ __forceinline__ void run_item(const BatchMol &d, const BatchItem &it, char *smem,
                                         char *smem2) {
    if constexpr (PREC == VV10_FP64) {
        tile_f64<NCB>(d.npad, d.jlen, d.Pp, static_cast<const double4 *>(d.P0),
                      static_cast<const double4 *>(d.P1), static_cast<const double *>(d.X),
                      static_cast<double *>(d.Ypart), it.itile, it.grp, it.split, smem);
    } else if constexpr (PREC == VV10_MIXED_FP32) {
        tile_f32<NCB>(d.npad, d.jlen, d.Pp, static_cast<const float4 *>(d.P0),
                      static_cast<const float4 *>(d.P1), static_cast<const float *>(d.X),
                      static_cast<double *>(d.Ypart), it.itile, it.grp, it.split, smem);
    } else {
        const bf16x8 *xh = static_cast<const bf16x8 *>(d.X);
        tile_bf16x3<NCB, false, PersistentTraits<PREC>::kWaves>(
            d.npad, d.jlen, d.Pp, static_cast<const float4 *>(d.P0),
            static_cast<const float4 *>(d.P1), xh, xh + d.npad * d.Pp * 2 / 8,
            static_cast<double *>(d.Ypart), it.itile, it.grp, it.split, smem, nullptr, smem2);
    }
}

// Grid items of a batch: one wave per workgroup pulls one grid tile of one
// molecule and atom group at a time (with the pair integrals, as the Hessian
// call forms them).  A kernel of its own keeps the grid pass's register
// allocation (and the standalone grid kernel's waves per SIMD), where the
// contraction kernels' allocations would hold it to two waves per SIMD.  At
// four waves per SIMD the mixed form spills 8 registers; three waves without
// spills measured slower on the 64-cluster batch (2625-2628 ms per launch
// against 2614-2619).
template <int PREC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(PREC == VV10_FP64 ? 3 : 4))) void k_grid_persistent(
    const BatchMol *__restrict__ mols, const BatchItem *__restrict__ items, int32_t n_items,
    int32_t *__restrict__ counter) {
    using T = std::conditional_t<PREC == VV10_FP64, double, float>;
    using T4 = std::conditional_t<PREC == VV10_FP64, double4, float4>;
    __shared__ T4 sA[kGridTile], sB[kGridTile];
    const int lane = threadIdx.x;
    for (;;) {
        int32_t k = 0;
        if (lane == 0) k = atomicAdd(counter, 1);
        k = __builtin_amdgcn_readfirstlane(k);   // lane 0's value, uniform
        if (k >= n_items) break;                  // every wave leaves once the list is drained
        const BatchItem it = items[k];
        const BatchMol d = mols[it.mol];
        // grid_unit orders its LDS writes after the previous reads itself
        grid_unit<T, T4, true, false>(d.n_atom, d.Pp, d.bgroups, d.npad, d.seg, d.tile_i0,
                                      d.tile_n, d.tile_atom, static_cast<const T4 *>(d.P0),
                                      static_cast<const T4 *>(d.P1), d.Pd, d.Z, nullptr, d.Dpart,
                                      d.Igrp, it.itile, it.grp, lane, sA, sB);
    }
}

template <int PREC>
__global__ __launch_bounds__(64 * PersistentTraits<PREC>::kWaves, 8 / PersistentTraits<PREC>::kWaves) void k_contract_persistent(
    const BatchMol *__restrict__ mols, const BatchItem *__restrict__ items, int32_t n_items,
    int32_t *__restrict__ counter) {
    constexpr int W = PersistentTraits<PREC>::kWaves;
    __shared__ __attribute__((aligned(16))) char smem[PersistentTraits<PREC>::kSmem];
    // the second stage buffer of the eight-wave form (a one-byte dummy otherwise)
    __shared__ __attribute__((aligned(16))) char smem2[W == 8 ? PersistentTraits<PREC>::kSmem : 1];
    __shared__ int32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t k = __builtin_amdgcn_readfirstlane(next);   // uniform: item data in SGPRs
        __syncthreads();
        if (k >= n_items) break;          // every workgroup leaves once the list is drained
        const BatchItem it = items[k];
        const BatchMol d = mols[it.mol];
        switch (d.ncb) {
#define VV10_CASE(c) \
    case c:          \
        if constexpr (c <= PersistentTraits<PREC>::kMaxNcb) run_item<PREC, c>(d, it, smem, smem2); \
        break;
            VV10_CASE(1) VV10_CASE(2) VV10_CASE(3) VV10_CASE(4) VV10_CASE(5) VV10_CASE(6)
            VV10_CASE(7) VV10_CASE(8) VV10_CASE(9) VV10_CASE(10) VV10_CASE(11) VV10_CASE(12)
#undef VV10_CASE
            default: break;
        }
        __syncthreads();                   // LDS is reused by the next item
    }
}

// Wide items of a split-BF16 batch (eight to twelve column blocks): the
// eight-wave form of the standalone kernel (128-point i tiles, 32-point
// stages with X straight into two LDS buffers) pulls them from a list and a
// counter of its own.  Only these column counts share its register
// allocation, which keeps the form's two waves per SIMD without spills
// (every column count in one kernel spilled it).
__global__ __launch_bounds__(512, 1) void k_contract_persistent_wide(
    const BatchMol *__restrict__ mols, const BatchItem *__restrict__ items, int32_t n_items,
    int32_t *__restrict__ counter) {
    static_assert(bf16_waves<kWideMinNcb>() == 8 && bf16_waves<12>() == 8,
                  "wide items run the eight-wave form");
    __shared__ __attribute__((aligned(16))) char smem[smem_bf16x3<12>()];
    __shared__ __attribute__((aligned(16))) char smem2[smem_bf16x3<12>()];
    __shared__ int32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t k = __builtin_amdgcn_readfirstlane(next);   // uniform: item data in SGPRs
        __syncthreads();
        if (k >= n_items) break;          // every workgroup leaves once the list is drained
        const BatchItem it = items[k];
        const BatchMol d = mols[it.mol];
        const bf16x8 *xh = static_cast<const bf16x8 *>(d.X);
        const bf16x8 *xl = xh + d.npad * d.Pp * 2 / 8;
        const float4 *p0 = static_cast<const float4 *>(d.P0);
        const float4 *p1 = static_cast<const float4 *>(d.P1);
        double *y = static_cast<double *>(d.Ypart);
        switch (d.ncb) {
#define VV10_CASE(c)                                                                         \
    case c:                                                                                  \
        tile_bf16x3<c, false, 8>(d.npad, d.jlen, d.Pp, p0, p1, xh, xl, y, it.itile, it.grp, \
                                 it.split, smem, nullptr, smem2);                            \
        break;
            VV10_CASE(8) VV10_CASE(9) VV10_CASE(10) VV10_CASE(11) VV10_CASE(12)
#undef VV10_CASE
            default: break;
        }
        __syncthreads();                   // LDS is reused by the next item
    }
}

__global__ void k_zero_counter(int32_t *c) { *c = 0; }

// ---------------------------------------------------------------------------
// Fused split-BF16 contraction for weights that move with the nuclei (one
// column group of at most four blocks): the pair geometry of each (i, j) is
// formed once for the main 2 x 2 kernel and for the three weight rows
// Y_pv, Y_qv, Y_vv of the weight contraction (weights.hip).  A stage is a
// 32-point j block: the main contraction takes it as two 16-point
// sub-blocks, the weight contraction as one K of 32 whose order follows the
// same lanes' pairs, k = 8 g + e for the point 4 g + e (e < 4) or
// 16 + 4 g + e - 4 (e >= 4) of the block, which is the order in which the
// weight packing stores v.
// ---------------------------------------------------------------------------
// The four main values and the three weight values (r - c_i A, -R^2 A, r)
// of pair (i, j), all divided by -3/2; the main values are those of pair_K.
__device__ __forceinline__ void pair_KW(const float4 a0, const float4 a1, const float4 b0,
                                        const float4 b1, float *k) {
    const float dx = a0.x - b0.x, dy = a0.y - b0.y, dz = a0.z - b0.z;
    const float R2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const float gg = __builtin_fmaf(a0.w, R2, a1.x);
    const float gp = __builtin_fmaf(b0.w, R2, b1.x);
    const float s = gg + gp, t = gg * gp;
    const float r = rcp32(t * s);
    const float sr = s * r;
    const float is = t * r;
    const float A = r * __builtin_fmaf(gp, sr, is);
    const float Ap = r * __builtin_fmaf(gg, sr, is);
    const float Q = (r + r) * __builtin_fmaf(is, is, sr);
    const float ci = a1.z, cj = b1.z;
    const float t1 = __builtin_fmaf(ci, Q, -Ap);
    const float t2 = __builtin_fmaf(cj, Q, -A);
    const float base = __builtin_fmaf(-ci, A, r);
    k[0] = __builtin_fmaf(cj, t1, base);    // kpp
    k[1] = R2 * t1;                         // kpq
    k[2] = R2 * t2;                         // kqp
    k[3] = (R2 * R2) * Q;                   // kqq
    k[4] = base;                            // kpv
    k[5] = -R2 * A;                         // kqv
    k[6] = r;                               // kvv
}

template <int NCB>
constexpr int smem_bf16x3_w() {
    return 2 * 6 * NCB * 16 * 4 * (int)sizeof(bf16x8) + 2 * 64 * (int)sizeof(float4);
}

template <int NCB>
__global__ __launch_bounds__(256, 2) void k_contract_bf16x3_w(
    int64_t npad, int64_t jlen, int32_t Pp, const float4 *__restrict__ P0,
    const float4 *__restrict__ P1, const bf16x8 *__restrict__ Xhi, const bf16x8 *__restrict__ Xlo,
    const bf16x8 *__restrict__ Vhi, const bf16x8 *__restrict__ Vlo, double *__restrict__ Yout,
    double *__restrict__ Ywout) {
    constexpr int NC = NCB * 16;
    constexpr int UNITS = NC * 4;           // 8-bf16 units of one array and block
    constexpr int NARR = 6;                 // main hi (2 sub-blocks), main lo (2), weight hi, lo
    constexpr int TOT = NARR * UNITS;
    constexpr int PER = (TOT + 255) / 256;
    __shared__ __attribute__((aligned(16))) char smem[smem_bf16x3_w<NCB>()];
    bf16x8 *sX = reinterpret_cast<bf16x8 *>(smem);                 // [2][NARR][UNITS]
    float4 *sP = reinterpret_cast<float4 *>(sX + 2 * TOT);         // [2][P0, P1][32]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int64_t ibase = (int64_t)blockIdx.x * 64 + wave * 16;
    const int64_t jbeg = (int64_t)blockIdx.z * jlen;
    const int64_t jend = min(npad, jbeg + jlen);
    const float4 a0 = P0[ibase + m], a1 = P1[ibase + m];
    v4f accp[NCB], accq[NCB], awp[NCB], awq[NCB], awv[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        accp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        accq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        awp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        awq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        awv[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
    }
    // the FP32 sums of each run of kFp32Run points go into this split's FP64
    // partials (D layout: item r of lane l holds row 4 (l/16) + r, column l%16)
    double *Yb = Yout + (int64_t)blockIdx.z * npad * 2 * Pp;
    double *Yw = Ywout + (int64_t)blockIdx.z * npad * 3 * Pp;
    bool first = true;
    auto flush = [&]() {
        // base addresses formed here (the empty asm keeps them from being
        // hoisted out of the loop)
        int64_t ob = (ibase + 4 * g) * 2 * Pp + m, ow = (ibase + 4 * g) * 3 * Pp + m;
        asm volatile("" : "+v"(ob), "+v"(ow));
        double *yb = Yb + ob, *yw = Yw + ow;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float v[5][NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                v[0][cb] = accp[cb][r];
                v[1][cb] = accq[cb][r];
                v[2][cb] = awp[cb][r];
                v[3][cb] = awq[cb][r];
                v[4][cb] = awv[cb][r];
            }
            add_row<NCB>(yb + (2 * r + 0) * (int64_t)Pp, v[0], first);
            add_row<NCB>(yb + (2 * r + 1) * (int64_t)Pp, v[1], first);
            add_row<NCB>(yw + (3 * r + 0) * (int64_t)Pp, v[2], first);
            add_row<NCB>(yw + (3 * r + 1) * (int64_t)Pp, v[3], first);
            add_row<NCB>(yw + (3 * r + 2) * (int64_t)Pp, v[4], first);
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            accp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
            accq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
            awp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
            awq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
            awv[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        }
        first = false;
    };
    bf16x8 rx[PER];
    float4 rp = {0.f, 0.f, 0.f, 0.f};
    // unit e = a UNITS + u of a block: a = 0, 1 main hi of sub-block 0, 1;
    // 2, 3 main lo; 4, 5 weight hi, lo
    auto load = [&](int64_t j0) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            if (e < TOT) {
                const int a = e / UNITS, u = e - a * UNITS;
                const bf16x8 *src = a < 4 ? (a < 2 ? Xhi : Xlo) + ((j0 / 16 + (a & 1)) * Pp) * 4
                                          : (a == 4 ? Vhi : Vlo) + ((j0 / 32) * Pp) * 4;
                rx[k] = src[u];
            }
        }
        if (tid < 64) rp = (tid < 32 ? P0 : P1)[j0 + (tid & 31)];
    };
    auto store = [&](int b) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            if (e < TOT) sX[b * TOT + e] = rx[k];
        }
        if (tid < 64) sP[b * 64 + tid] = rp;
    };
    load(jbeg);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jbeg; j0 < jend; j0 += 32) {
        const bool more = j0 + 32 < jend;
        if (more) load(j0 + 32);
        const float4 *q0 = sP + buf * 64, *q1 = q0 + 32;
        uint32_t mh[2][4], ml[2][4], nh[2][4], nl[2][4];
        uint32_t vph[4], vpl[4], vqh[4], vql[4], vvh[4], vvl[4];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            const int sb = e >> 2, jj = e & 3;
            const int jl = 16 * sb + 4 * g + jj;
            float k0[7], k1[7];
            pair_KW(a0, a1, q0[jl], q1[jl], k0);
            pair_KW(a0, a1, q0[jl + 1], q1[jl + 1], k1);
            split2(k0[0], k0[1], mh[sb][jj], ml[sb][jj]);
            split2(k0[2], k0[3], nh[sb][jj], nl[sb][jj]);
            split2(k1[0], k1[1], mh[sb][jj + 1], ml[sb][jj + 1]);
            split2(k1[2], k1[3], nh[sb][jj + 1], nl[sb][jj + 1]);
            split2(k0[4], k1[4], vph[e >> 1], vpl[e >> 1]);
            split2(k0[5], k1[5], vqh[e >> 1], vql[e >> 1]);
            split2(k0[6], k1[6], vvh[e >> 1], vvl[e >> 1]);
        }
        Aops A[2];
#pragma unroll
        for (int sb = 0; sb < 2; ++sb) {
            A[sb].ph = __builtin_bit_cast(bf16x8, (uint4){mh[sb][0], mh[sb][1], mh[sb][2], mh[sb][3]});
            A[sb].pl = __builtin_bit_cast(bf16x8, (uint4){ml[sb][0], ml[sb][1], ml[sb][2], ml[sb][3]});
            A[sb].qh = __builtin_bit_cast(bf16x8, (uint4){nh[sb][0], nh[sb][1], nh[sb][2], nh[sb][3]});
            A[sb].ql = __builtin_bit_cast(bf16x8, (uint4){nl[sb][0], nl[sb][1], nl[sb][2], nl[sb][3]});
        }
        bf16x8 wph = __builtin_bit_cast(bf16x8, (uint4){vph[0], vph[1], vph[2], vph[3]});
        bf16x8 wpl = __builtin_bit_cast(bf16x8, (uint4){vpl[0], vpl[1], vpl[2], vpl[3]});
        const bf16x8 wqh = __builtin_bit_cast(bf16x8, (uint4){vqh[0], vqh[1], vqh[2], vqh[3]});
        const bf16x8 wql = __builtin_bit_cast(bf16x8, (uint4){vql[0], vql[1], vql[2], vql[3]});
        bf16x8 wvh = __builtin_bit_cast(bf16x8, (uint4){vvh[0], vvh[1], vvh[2], vvh[3]});
        bf16x8 wvl = __builtin_bit_cast(bf16x8, (uint4){vvl[0], vvl[1], vvl[2], vvl[3]});
        {
            // The stage that holds the outer points: the self pair (i, i) is
            // point off = ibase - j0 + m of the stage, formed by lane group
            // (off mod 16)/4 as main pair off mod 4 of sub-block off/16 (K_pp
            // cleared) and as weight K entry e = 4 (off/16) + off mod 4 (the
            // rows r - c_i A and r cleared; -R^2 A vanishes there).  The masks
            // are applied in every stage (all ones off the diagonal): a branch
            // here would split the stage into a VALU block and an MFMA block
            // that the compiler then cannot interleave (measured on the
            // weighted hexamer: 3.44-3.55 ms with the branch, 2.41 ms without).
            const bool diag = j0 == (ibase & ~(int64_t)31);
            const int off = (int)(ibase - j0) + m, sb = (off >> 4) & 1, jj = off & 3;
            const bool mine = diag && g == ((off & 15) >> 2);
            const uint4 km0 = bf16_clear_mask(mine && sb == 0, jj, false);
            const uint4 km1 = bf16_clear_mask(mine && sb == 1, jj, false);
            A[0].ph = bf16_apply_mask(A[0].ph, km0);
            A[0].pl = bf16_apply_mask(A[0].pl, km0);
            A[1].ph = bf16_apply_mask(A[1].ph, km1);
            A[1].pl = bf16_apply_mask(A[1].pl, km1);
            const int e = 4 * sb + jj;
            const uint4 kw = bf16_clear_mask(mine, e >> 1, e & 1);
            wph = bf16_apply_mask(wph, kw);
            wpl = bf16_apply_mask(wpl, kw);
            wvh = bf16_apply_mask(wvh, kw);
            wvl = bf16_apply_mask(wvl, kw);
        }
        const bf16x8 *xb = sX + buf * TOT + m * 4 + g;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) {
                const bf16x8 bh = xb[sb * UNITS + cb * 64], bl = xb[(2 + sb) * UNITS + cb * 64];
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[sb].ph, bh, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[sb].qh, bh, accq[cb], 0, 0, 0);
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[sb].pl, bh, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[sb].ql, bh, accq[cb], 0, 0, 0);
                accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[sb].ph, bl, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[sb].qh, bl, accq[cb], 0, 0, 0);
            }
            const bf16x8 vh = xb[4 * UNITS + cb * 64], vl = xb[5 * UNITS + cb * 64];
            awp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wph, vh, awp[cb], 0, 0, 0);
            awq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wqh, vh, awq[cb], 0, 0, 0);
            awv[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wvh, vh, awv[cb], 0, 0, 0);
            awp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wpl, vh, awp[cb], 0, 0, 0);
            awq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wql, vh, awq[cb], 0, 0, 0);
            awv[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wvl, vh, awv[cb], 0, 0, 0);
            awp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wph, vl, awp[cb], 0, 0, 0);
            awq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wqh, vl, awq[cb], 0, 0, 0);
            awv[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wvh, vl, awv[cb], 0, 0, 0);
        }
        if (more) store(buf ^ 1);
        if ((j0 + 32 - jbeg) % kFp32Run == 0 && more) flush();
        __syncthreads();
        buf ^= 1;
    }
    flush();
}

template <int NCB>
hipError_t run_weighted(vv10_plan *p, const Workspace &ws, const WeightWork &ww) {
    dim3 grid((unsigned)(p->npad / 64), 1u, (unsigned)ws.jsplit);
    const bf16x8 *xh = static_cast<const bf16x8 *>(ws.X);
    const bf16x8 *xl = xh + (size_t)p->npad * ws.Pp * 2 / 8;
    const bf16x8 *vh = static_cast<const bf16x8 *>(ww.Xv);
    const bf16x8 *vl = vh + (size_t)p->npad * ws.Pp / 8;
    k_contract_bf16x3_w<NCB><<<grid, 256, 0, p->stream>>>(
        p->npad, ws.jlen, ws.Pp, p->P0f, p->P1f, xh, xl, vh, vl, static_cast<double *>(ws.Ypart),
        static_cast<double *>(ww.Ypart));
    return hipGetLastError();
}

}  // namespace

int contract_blocks_per_cu(vv10_precision prec, int ncb) {
    return dispatch_ncb(ncb, [&](auto c) { return occupancy<decltype(c)::value>(prec); });
}

hipError_t launch_contract(vv10_plan *p, const Workspace &ws, bool screen) {
    if (ws.ncb < 1 || ws.ncb > max_ncb(p->prec)) return hipErrorInvalidValue;
    return dispatch_ncb(ws.ncb, [&](auto c) { return run<decltype(c)::value>(p, ws, screen); });
}

bool fused_weighted_contract(const vv10_plan *p, const Workspace &ws) {
    return p->prec == VV10_MIXED_BF16X3 && ws.ngroups == 1 && ws.ncb <= 4;
}

hipError_t launch_contract_weighted(vv10_plan *p, const Workspace &ws, const WeightWork &ww) {
    if (!fused_weighted_contract(p, ws)) return hipErrorInvalidValue;
    switch (ws.ncb) {
        case 1: return run_weighted<1>(p, ws, ww);
        case 2: return run_weighted<2>(p, ws, ww);
        case 3: return run_weighted<3>(p, ws, ww);
        case 4: return run_weighted<4>(p, ws, ww);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace vv10

namespace vv10 {

int persistent_waves(vv10_precision prec) {
    if (prec == VV10_FP64) return PersistentTraits<VV10_FP64>::kWaves;
    if (prec == VV10_MIXED_FP32) return PersistentTraits<VV10_MIXED_FP32>::kWaves;
    return PersistentTraits<VV10_MIXED_BF16X3>::kWaves;
}

int persistent_blocks_per_cu(vv10_precision prec) {
    int nb = 0;
    hipError_t e;
    const int nt = 64 * persistent_waves(prec);
    if (prec == VV10_FP64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_contract_persistent<VV10_FP64>, nt, 0);
    else if (prec == VV10_MIXED_FP32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_contract_persistent<VV10_MIXED_FP32>, nt, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_contract_persistent<VV10_MIXED_BF16X3>, nt, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

int persistent_wide_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_contract_persistent_wide, 512, 0) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}
hipError_t launch_contract_persistent_wide(const BatchMol *mols, const BatchItem *items,
                                           int32_t n_items, int32_t *counter, int n_blocks,
                                           hipStream_t stream) {
    k_zero_counter<<<1, 1, 0, stream>>>(counter);
    k_contract_persistent_wide<<<n_blocks, 512, 0, stream>>>(mols, items, n_items, counter);
    return hipGetLastError();
}
int persistent_grid_blocks_per_cu(vv10_precision prec) {
    int nb = 0;
    hipError_t e;
    if (prec == VV10_FP64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_grid_persistent<VV10_FP64>, 64, 0);
    else if (prec == VV10_MIXED_FP32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_grid_persistent<VV10_MIXED_FP32>, 64, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_grid_persistent<VV10_MIXED_BF16X3>, 64, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}
hipError_t launch_grid_persistent(vv10_precision prec, const BatchMol *mols,
                                  const BatchItem *items, int32_t n_items, int32_t *counter,
                                  int n_blocks, hipStream_t stream) {
    k_zero_counter<<<1, 1, 0, stream>>>(counter);
    if (prec == VV10_FP64)
        k_grid_persistent<VV10_FP64><<<n_blocks, 64, 0, stream>>>(mols, items, n_items, counter);
    else if (prec == VV10_MIXED_FP32)
        k_grid_persistent<VV10_MIXED_FP32><<<n_blocks, 64, 0, stream>>>(mols, items, n_items, counter);
    else
        k_grid_persistent<VV10_MIXED_BF16X3><<<n_blocks, 64, 0, stream>>>(mols, items, n_items, counter);
    return hipGetLastError();
}
hipError_t launch_contract_persistent(vv10_precision prec, const BatchMol *mols,
                                      const BatchItem *items, int32_t n_items, int32_t *counter,
                                      int n_blocks, hipStream_t stream) {
    k_zero_counter<<<1, 1, 0, stream>>>(counter);
    const int nt = 64 * persistent_waves(prec);
    if (prec == VV10_FP64)
        k_contract_persistent<VV10_FP64><<<n_blocks, nt, 0, stream>>>(mols, items, n_items, counter);
    else if (prec == VV10_MIXED_FP32)
        k_contract_persistent<VV10_MIXED_FP32><<<n_blocks, nt, 0, stream>>>(mols, items, n_items, counter);
    else
        k_contract_persistent<VV10_MIXED_BF16X3><<<n_blocks, nt, 0, stream>>>(mols, items, n_items, counter);
    return hipGetLastError();
}

}  // namespace vv10
