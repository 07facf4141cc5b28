// Weight-derivative terms for grids whose quadrature weights move with the
// nuclei (Section II.A, E^A_w; Section II.B, E_{w,w}, E_{G,w}, E_{w,gr} and
// F^A_w).
//
// The caller passes w^x_i = dw_i/dX_x for every perturbation x = 3 B + b
// (grid points moving with their owner atoms).  A rigid translation of the
// molecule and its grid leaves every weight unchanged, so the owner-atom
// slot follows from the others,
//   w^{(O(i),b)}_i = -sum_{B != O(i)} w^{(B,b)}_i,
// and those entries of w_x are not read.
//
// The pair part is one contraction with a single channel v^x_j = w^x_j rho_j
// and three outputs per outer point i,
//   Y_pv = sum_j (Phi + c_i Phi_g) v_j  = E^{xw}_i + c_i U^{xw}_i
//   Y_qv = sum_j R^2 Phi_g v_j          = W^{xw}_i
//   Y_vv = sum_j Phi v_j                = E^{xw}_i
// with Phi_g = -Phi (1/g + 1/s), s = g + g', c = rho dkappa/drho: the inner
// integrals E^{Bw}, U^{Bw}, W^{Bw} already combined the way E_{G,w} and F^A_w
// use them.  The mixed modes carry -3/2 in v and form r - c_i A, -R^2 A and
// r with r = 1/(g g' s), A = r (1/g + 1/s).
//
// Arithmetic modes as in the main contraction:
//  FP64, FP32: v_mfma_{f64,f32}_16x16x4, one pair per lane per 4 j, three
//              MFMAs per 16 columns (one per output);
//  BF16X3:     v_mfma_f32_16x16x32_bf16 with K over a 32-point j block of the
//              one channel (each lane forms 8 pairs per block: the points
//              4 g .. 4 g + 3 of both 16-point halves, g = lane/16), hi/lo split
//              of both operands and three products per output.  When the
//              columns form one group of at most four blocks the main
//              contraction forms these pairs anyway, and the fused kernel of
//              contract.hip evaluates both from one pair geometry.
#include "dev_common.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

// Owner-atom slot of w^x by translational invariance: Wown[i][b].
__global__ __launch_bounds__(256) void k_wown(int64_t n, int32_t n_atom,
                                              const int32_t *__restrict__ atom_of,
                                              const double *__restrict__ w_x,
                                              double *__restrict__ Wown) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int O = atom_of[i];
    double s[3] = {0.0, 0.0, 0.0};
    for (int B = 0; B < n_atom; ++B) {
        if (B == O) continue;
#pragma unroll
        for (int b = 0; b < 3; ++b) s[b] += w_x[(int64_t)(3 * B + b) * n + i];
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) Wown[i * 3 + b] = -s[b];
}

// Lw[i][x] = w^x_i (owner slot from Wown, zero for padding) and the packed
// channel v = sc w^x_i rho_i (sc = 1 in FP64, -3/2 in the mixed modes):
// FP64/FP32 [npad][Pp]; BF16X3 hi then lo, each [npad/32][Pp][32] with the
// point o of a 32-point block at K position 8 ((o mod 16)/4) + o mod 4 + 4 (o/16),
// so that the 8 K values of lane group g are the points 4 g .. 4 g + 3 of
// both 16-point halves (the pairs the main contraction's lanes form).
constexpr int TT = 32;
template <int MODE>
__global__ __launch_bounds__(256) void k_wprep(int64_t n, int64_t npad, int32_t P, int32_t Pp,
                                               const double *__restrict__ w_x,
                                               const int32_t *__restrict__ atom_of,
                                               const double *__restrict__ Wown,
                                               const double *__restrict__ F, void *__restrict__ Xv,
                                               double *__restrict__ Lw) {
    __shared__ double sw[TT][TT + 1];
    const int64_t i0 = (int64_t)blockIdx.x * TT;
    const int x0 = blockIdx.y * TT;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;   // 32 x 8
    for (int k = 0; k < TT; k += 8) {
        const int x = x0 + ty + k;
        const int64_t i = i0 + tx;
        sw[ty + k][tx] = (x < P && i < n) ? w_x[(int64_t)x * n + i] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < TT; k += 8) {
        const int64_t i = i0 + ty + k;
        const int x = x0 + tx;
        if (i >= npad || x >= Pp) continue;
        double wx = 0.0;
        if (i < n && x < P) wx = (x / 3 == atom_of[i]) ? Wown[i * 3 + x % 3] : sw[tx][ty + k];
        Lw[i * Pp + x] = wx;
        const double sc = MODE == VV10_FP64 ? 1.0 : -1.5;
        const double v = sc * wx * F[F_RHO * npad + i];
        if (MODE == VV10_FP64) {
            static_cast<double *>(Xv)[i * Pp + x] = v;
        } else if (MODE == VV10_MIXED_FP32) {
            static_cast<float *>(Xv)[i * Pp + x] = (float)v;
        } else {
            __bf16 *Xh = static_cast<__bf16 *>(Xv);
            __bf16 *Xl = Xh + npad * Pp;
            const int oo = (int)(i % 32);
            const int64_t o = ((i / 32) * Pp + x) * 32 + 8 * ((oo & 15) >> 2) + (oo & 3) + 4 * (oo >> 4);
            const __bf16 h = (__bf16)(float)v;
            Xh[o] = h;
            Xl[o] = (__bf16)(float)(v - (double)(float)h);
        }
    }
}

constexpr int kJC = 32;   // j points per LDS stage (FP64, FP32)

// ---------------------------------------------------------------------------
// FP64 / FP32 MFMA (16 x 16 x 4): lane (m, kq) forms pair (ibase + m, j + kq).
// ---------------------------------------------------------------------------
template <typename T>
struct WTraits;
template <>
struct WTraits<double> {
    typedef double4 P4;
    typedef v4d Acc;
    static __device__ __forceinline__ Acc mfma(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // D layout (measured on gfx950): item r of lane l holds row 4 r + l/16
    static __device__ __forceinline__ int row(int r, int kq) { return 4 * r + kq; }
};
template <>
struct WTraits<float> {
    typedef float4 P4;
    typedef v4f Acc;
    static __device__ __forceinline__ Acc mfma(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // item r of lane l holds row 4 (l/16) + r
    static __device__ __forceinline__ int row(int r, int kq) { return 4 * kq + r; }
};

// The three kernel values of pair (i, j): FP64 forms them with Phi, FP32
// divided by -3/2.  a = (x, y, z, omega), b = (kappa, a, c, .).
__device__ __forceinline__ void pair_w(const double4 a0, const double4 a1, const double4 b0,
                                       const double4 b1, double &kpv, double &kqv, double &kvv) {
    const double dx = a0.x - b0.x, dy = a0.y - b0.y, dz = a0.z - b0.z;
    const double R2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    const double g = __builtin_fma(a0.w, R2, a1.x);
    const double gp = __builtin_fma(b0.w, R2, b1.x);
    const double s = g + gp, t = g * gp;
    const double r = rcp64(t * s);
    const double phi = -1.5 * r;
    const double ig = gp * s * r, is = t * r;
    const double Pg = -phi * (ig + is);
    kpv = __builtin_fma(a1.z, Pg, phi);
    kqv = R2 * Pg;
    kvv = phi;
}

__device__ __forceinline__ void pair_w(const float4 a0, const float4 a1, const float4 b0,
                                       const float4 b1, float &kpv, float &kqv, float &kvv) {
    const float dx = a0.x - b0.x, dy = a0.y - b0.y, dz = a0.z - b0.z;
    const float R2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const float g = __builtin_fmaf(a0.w, R2, a1.x);
    const float gp = __builtin_fmaf(b0.w, R2, b1.x);
    const float s = g + gp, t = g * gp;
    const float r = rcp32(t * s);
    const float A = r * __builtin_fmaf(gp, s * r, t * r);   // r (1/g + 1/s)
    kpv = __builtin_fmaf(-a1.z, A, r);
    kqv = -R2 * A;
    kvv = r;
}

template <typename T, int NCB>
constexpr int smem_w() {
    return 2 * kJC * (int)sizeof(typename WTraits<T>::P4) + kJC * NCB * 16 * (int)sizeof(T);
}

template <typename T, int NCB>
__global__ __launch_bounds__(256, 2) void k_wcontract(int64_t npad, int64_t jlen, int32_t Pp,
                                                      const typename WTraits<T>::P4 *__restrict__ P0,
                                                      const typename WTraits<T>::P4 *__restrict__ P1,
                                                      const T *__restrict__ X, double *__restrict__ Yout) {
    typedef typename WTraits<T>::P4 P4;
    typedef typename WTraits<T>::Acc Acc;
    constexpr int NC = NCB * 16;
    static_assert(kFp32Run % kJC == 0, "FP32 runs end on chunk boundaries");
    __shared__ __attribute__((aligned(16))) char smem[smem_w<T, NCB>()];
    P4 *sA = reinterpret_cast<P4 *>(smem);
    P4 *sB = sA + kJC;
    T *sX = reinterpret_cast<T *>(sB + kJC);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int64_t ibase = (int64_t)blockIdx.x * 64 + wave * 16;
    const int col0 = blockIdx.y * NC;
    const int64_t jbeg = (int64_t)blockIdx.z * jlen;
    const int64_t jend = min(npad, jbeg + jlen);
    const P4 a0 = P0[ibase + m], a1 = P1[ibase + m];
    Acc accp[NCB], accq[NCB], accv[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        accp[cb] = (Acc){0, 0, 0, 0};
        accq[cb] = (Acc){0, 0, 0, 0};
        accv[cb] = (Acc){0, 0, 0, 0};
    }
    // the partials are FP64: FP64 sums are stored once at the end; FP32 sums
    // go in after each run of kFp32Run points
    double *Yb = Yout + (int64_t)blockIdx.z * npad * 3 * Pp;
    bool first = true;
    auto flush = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = ibase + WTraits<T>::row(r, kq);
            double *y = Yb + row * 3 * Pp + col0 + m;
            if constexpr (sizeof(T) == 8) {
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    y[0 * Pp + cb * 16] = accp[cb][r];
                    y[1 * Pp + cb * 16] = accq[cb][r];
                    y[2 * Pp + cb * 16] = accv[cb][r];
                }
            } else {
                float v[3][NCB];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    v[0][cb] = accp[cb][r];
                    v[1][cb] = accq[cb][r];
                    v[2][cb] = accv[cb][r];
                }
                add_row<NCB>(y + 0 * (int64_t)Pp, v[0], first);
                add_row<NCB>(y + 1 * (int64_t)Pp, v[1], first);
                add_row<NCB>(y + 2 * (int64_t)Pp, v[2], first);
            }
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            accp[cb] = (Acc){0, 0, 0, 0};
            accq[cb] = (Acc){0, 0, 0, 0};
            accv[cb] = (Acc){0, 0, 0, 0};
        }
        first = false;
    };
    for (int64_t j0 = jbeg; j0 < jend; j0 += kJC) {
        __syncthreads();
        if (tid < kJC) {
            sA[tid] = P0[j0 + tid];
            sB[tid] = P1[j0 + tid];
        }
        for (int e = tid; e < kJC * NC; e += 256) {
            const int row = e / NC, cc = e - row * NC;
            sX[e] = X[(j0 + row) * Pp + col0 + cc];
        }
        __syncthreads();
        // the chunk that holds this wave's outer points leaves out the self
        // pair (its rows Phi + c_i Phi_g and Phi; R^2 Phi_g vanishes there)
        const bool diag = ibase < j0 + kJC && ibase + 16 > j0;
        const int dself = diag ? (int)(ibase - j0) + m - kq : -1;
#pragma unroll 2
        for (int jj = 0; jj < kJC; jj += 4) {
            const int jl = jj + kq;
            T kpv, kqv, kvv;
            pair_w(a0, a1, sA[jl], sB[jl], kpv, kqv, kvv);
            kpv = jj == dself ? T(0) : kpv;
            kvv = jj == dself ? T(0) : kvv;
            const T *xr = sX + jl * NC + m;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const T xv = xr[cb * 16];
                accp[cb] = WTraits<T>::mfma(kpv, xv, accp[cb]);
                accq[cb] = WTraits<T>::mfma(kqv, xv, accq[cb]);
                accv[cb] = WTraits<T>::mfma(kvv, xv, accv[cb]);
            }
        }
        if constexpr (sizeof(T) == 4)
            if ((j0 + kJC - jbeg) % kFp32Run == 0 && j0 + kJC < jend) flush();
    }
    flush();
}

// ---------------------------------------------------------------------------
// split-BF16 MFMA (16 x 16 x 32), K over 32 consecutive j
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Packed bf16 hi (round to nearest even) and lo (rounded remainder) of two
// FP32 values, v0 in the low half; contraction off so that v - hi is a plain
// subtraction.
__device__ __forceinline__ void wsplit2(float v0, float v1, uint32_t &hi, uint32_t &lo) {
#pragma clang fp contract(off)
    const bf16x2 h = {(__bf16)v0, (__bf16)v1};
    hi = __builtin_bit_cast(uint32_t, h);
    const float h0 = __uint_as_float(__builtin_amdgcn_perm(0u, hi, 0x01000c0cu));   // hi << 16
    const float h1 = __uint_as_float(hi & 0xffff0000u);
    const bf16x2 l = {(__bf16)(v0 - h0), (__bf16)(v1 - h1)};
    lo = __builtin_bit_cast(uint32_t, l);
}

struct WAops {   // A operands of one 16 x 32 pair block (per lane: 8 pairs)
    bf16x8 ph, pl, qh, ql, vh, vl;
};

__device__ __forceinline__ WAops form_wA(const float4 a0, const float4 a1, const float4 *b0,
                                         const float *bk) {
    uint32_t ph[4], pl[4], qh[4], ql[4], vh[4], vl[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        float p0, q0, v0, p1, q1, v1;
        pair_w(a0, a1, b0[e], make_float4(bk[e], 0.f, 0.f, 0.f), p0, q0, v0);
        pair_w(a0, a1, b0[e + 1], make_float4(bk[e + 1], 0.f, 0.f, 0.f), p1, q1, v1);
        wsplit2(p0, p1, ph[e / 2], pl[e / 2]);
        wsplit2(q0, q1, qh[e / 2], ql[e / 2]);
        wsplit2(v0, v1, vh[e / 2], vl[e / 2]);
    }
    WAops A;
    A.ph = __builtin_bit_cast(bf16x8, (uint4){ph[0], ph[1], ph[2], ph[3]});
    A.pl = __builtin_bit_cast(bf16x8, (uint4){pl[0], pl[1], pl[2], pl[3]});
    A.qh = __builtin_bit_cast(bf16x8, (uint4){qh[0], qh[1], qh[2], qh[3]});
    A.ql = __builtin_bit_cast(bf16x8, (uint4){ql[0], ql[1], ql[2], ql[3]});
    A.vh = __builtin_bit_cast(bf16x8, (uint4){vh[0], vh[1], vh[2], vh[3]});
    A.vl = __builtin_bit_cast(bf16x8, (uint4){vl[0], vl[1], vl[2], vl[3]});
    return A;
}

template <int NCB>
constexpr int smem_wbf16() { return 2 * 2 * NCB * 16 * 4 * (int)sizeof(bf16x8); }

// Pipeline as in the main split-BF16 contraction: the X block (hi, lo) is
// double-buffered in LDS and the A operands of the next block are formed
// while the current block's MFMAs run.
template <int NCB>
__global__ __launch_bounds__(256, 2) void k_wcontract_bf16x3(int64_t npad, int64_t jlen, int32_t Pp,
                                                             const float4 *__restrict__ P0,
                                                             const float4 *__restrict__ P1,
                                                             const bf16x8 *__restrict__ Xhi,
                                                             const bf16x8 *__restrict__ Xlo,
                                                             double *__restrict__ Yout) {
    constexpr int NC = NCB * 16;
    static_assert(kFp32Run % 32 == 0, "FP32 runs end on block boundaries");
    constexpr int UNITS = NC * 4;                       // 8-bf16 units per block and array
    constexpr int PER = (UNITS + 255) / 256;
    typedef bf16x8 Buf[UNITS];
    __shared__ __attribute__((aligned(16))) char smem[smem_wbf16<NCB>()];
    Buf *sH = reinterpret_cast<Buf *>(smem);            // [buffer][col][g]
    Buf *sL = sH + 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int64_t ibase = (int64_t)blockIdx.x * 64 + wave * 16;
    const int col0 = blockIdx.y * NC;
    const int64_t jbeg = (int64_t)blockIdx.z * jlen;
    const int64_t jend = min(npad, jbeg + jlen);
    const float4 a0 = P0[ibase + m], a1 = P1[ibase + m];
    v4f accp[NCB], accq[NCB], accv[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        accp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        accq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        accv[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
    }
    // the FP32 sums of each run of kFp32Run points go into this split's FP64
    // partials (D layout: item r of lane l holds row 4 (l/16) + r, column l%16)
    double *Yb = Yout + (int64_t)blockIdx.z * npad * 3 * Pp;
    bool first = true;
    auto flush = [&]() {
        // one base address formed here (the empty asm keeps it from being
        // hoisted out of the loop)
        int64_t off = (ibase + 4 * g) * 3 * Pp + col0 + m;
        asm volatile("" : "+v"(off));
        double *y = Yb + off;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float v[3][NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                v[0][cb] = accp[cb][r];
                v[1][cb] = accq[cb][r];
                v[2][cb] = accv[cb][r];
            }
            add_row<NCB>(y + (3 * r + 0) * (int64_t)Pp, v[0], first);
            add_row<NCB>(y + (3 * r + 1) * (int64_t)Pp, v[1], first);
            add_row<NCB>(y + (3 * r + 2) * (int64_t)Pp, v[2], first);
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            accp[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
            accq[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
            accv[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
        }
        first = false;
    };
    bf16x8 rh[PER], rl[PER];
    auto load_x = [&](int64_t blk) {
        const int64_t base = ((blk / 32) * Pp + col0) * 4;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            if (e < UNITS) {
                rh[k] = Xhi[base + e];
                rl[k] = Xlo[base + e];
            }
        }
    };
    auto store_x = [&](int buf) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            if (e < UNITS) {
                sH[buf][e] = rh[k];
                sL[buf][e] = rl[k];
            }
        }
    };
    // this lane's 8 j of a block (K position 8 g + e): j = blk + 4 g + e for
    // e < 4 and blk + 16 + 4 g + e - 4 for e >= 4
    float4 n0[8];
    float nk[8];
    const float *P1s = reinterpret_cast<const float *>(P1);
    auto load_pts = [&](int64_t blk) {
        const int64_t jq = min(blk, npad - 32) + 4 * g;   // clamped: never read past npad
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t j = jq + (e < 4 ? e : 12 + e);
            n0[e] = P0[j];
            nk[e] = P1s[4 * j];
        }
    };
    load_pts(jbeg);
    load_x(jbeg);
    WAops cur = form_wA(a0, a1, n0, nk);
    load_pts(jbeg + 32);
    store_x(0);
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jbeg; j0 < jend; j0 += 32) {
        if (j0 == (ibase & ~(int64_t)31)) {
            // the block that holds the outer points: the self pair is point
            // off = ibase - j0 + m of the block, K entry e = (off mod 16) mod 4
            // + 4 (off/16) of lane group (off mod 16)/4; its rows r - c_i A
            // and r are cleared (-R^2 A vanishes there)
            const int off = (int)(ibase - j0) + m;
            const int e = (off & 3) + ((off >> 4) << 2);
            const uint4 k = bf16_clear_mask(g == ((off & 15) >> 2), e >> 1, e & 1);
            cur.ph = bf16_apply_mask(cur.ph, k);
            cur.pl = bf16_apply_mask(cur.pl, k);
            cur.vh = bf16_apply_mask(cur.vh, k);
            cur.vl = bf16_apply_mask(cur.vl, k);
        }
        const bool more = j0 + 32 < jend;
        if (more) load_x(j0 + 32);
        const WAops nxt = form_wA(a0, a1, n0, nk);
        load_pts(j0 + 64);
        const bf16x8 *hp = sH[buf] + m * 4 + g;
        const bf16x8 *lp = sL[buf] + m * 4 + g;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const bf16x8 bh = hp[cb * 64], bl = lp[cb * 64];
            accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ph, bh, accp[cb], 0, 0, 0);
            accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.qh, bh, accq[cb], 0, 0, 0);
            accv[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.vh, bh, accv[cb], 0, 0, 0);
            accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.pl, bh, accp[cb], 0, 0, 0);
            accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ql, bh, accq[cb], 0, 0, 0);
            accv[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.vl, bh, accv[cb], 0, 0, 0);
            accp[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.ph, bl, accp[cb], 0, 0, 0);
            accq[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.qh, bl, accq[cb], 0, 0, 0);
            accv[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.vh, bl, accv[cb], 0, 0, 0);
        }
        cur = nxt;
        if (more) store_x(buf ^ 1);
        if ((j0 + 32 - jbeg) % kFp32Run == 0 && more) flush();
        __syncthreads();
        buf ^= 1;
    }
    flush();
}

template <int NCB>
hipError_t run_w(vv10_plan *p, const WeightWork &ww) {
    const Workspace &ws = p->ws;
    dim3 grid((unsigned)(p->npad / 64), (unsigned)ww.groups, (unsigned)ws.jsplit);
    if (p->prec == VV10_FP64) {
        if constexpr (NCB <= 4)
            k_wcontract<double, NCB><<<grid, 256, 0, p->stream>>>(
                p->npad, ws.jlen, ws.Pp, p->P0, p->P1, static_cast<const double *>(ww.Xv),
                static_cast<double *>(ww.Ypart));
        else
            return hipErrorInvalidValue;
    } else if (p->prec == VV10_MIXED_FP32) {
        k_wcontract<float, NCB><<<grid, 256, 0, p->stream>>>(
            p->npad, ws.jlen, ws.Pp, p->P0f, p->P1f, static_cast<const float *>(ww.Xv),
            static_cast<double *>(ww.Ypart));
    } else {
        const bf16x8 *xh = static_cast<const bf16x8 *>(ww.Xv);
        const bf16x8 *xl = xh + (size_t)p->npad * ws.Pp / 8;
        k_wcontract_bf16x3<NCB><<<grid, 256, 0, p->stream>>>(
            p->npad, ws.jlen, ws.Pp, p->P0f, p->P1f, xh, xl, static_cast<double *>(ww.Ypart));
    }
    return hipGetLastError();
}

}  // namespace

void weight_shape(int32_t Pp, vv10_precision prec, WeightWork &ww) {
    const int total = Pp / 16;
    const int cap = max_wncb(prec);
    ww.groups = 1;
    while (total % ww.groups || total / ww.groups > cap) ++ww.groups;
    ww.ncb = total / ww.groups;
}

hipError_t launch_weight_own(vv10_plan *p, const double *w_x, double *Wown) {
    k_wown<<<(unsigned)((p->n + 255) / 256), 256, 0, p->stream>>>(p->n, p->n_atom, p->atom_of, w_x,
                                                                  Wown);
    return hipGetLastError();
}

hipError_t launch_weight_prep(vv10_plan *p, const double *w_x) {
    const Workspace &ws = p->ws;
    const WeightWork &ww = p->ww;
    hipError_t e = launch_weight_own(p, w_x, ww.Wown);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)(p->npad / TT), (unsigned)((ws.Pp + TT - 1) / TT));
    if (p->prec == VV10_FP64)
        k_wprep<VV10_FP64><<<grid, 256, 0, p->stream>>>(p->n, p->npad, ws.P, ws.Pp, w_x, p->atom_of,
                                                         ww.Wown, p->F, ww.Xv, ww.Lw);
    else if (p->prec == VV10_MIXED_FP32)
        k_wprep<VV10_MIXED_FP32><<<grid, 256, 0, p->stream>>>(p->n, p->npad, ws.P, ws.Pp, w_x,
                                                               p->atom_of, ww.Wown, p->F, ww.Xv,
                                                               ww.Lw);
    else
        k_wprep<VV10_MIXED_BF16X3><<<grid, 256, 0, p->stream>>>(p->n, p->npad, ws.P, ws.Pp, w_x,
                                                                 p->atom_of, ww.Wown, p->F, ww.Xv,
                                                                 ww.Lw);
    return hipGetLastError();
}

hipError_t launch_weight_contract(vv10_plan *p) {
    const WeightWork &ww = p->ww;
    switch (ww.ncb) {
        case 1: return run_w<1>(p, ww);
        case 2: return run_w<2>(p, ww);
        case 3: return run_w<3>(p, ww);
        case 4: return run_w<4>(p, ww);
        case 5: return run_w<5>(p, ww);
        case 6: return run_w<6>(p, ww);
        case 7: return run_w<7>(p, ww);
        case 8: return run_w<8>(p, ww);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace vv10
