// Pair kernel: the inner integrals of Section II.A (E_i, U_i, W_i) and,
// in Hessian mode, those of Section II.B (A_i, B_i, C_i):
//   E_i = sum_j a_j Phi_ij
//   U_i = -sum_j a_j Phi_ij h_ij,           h = 1/(g+g') + 1/g
//   W_i = -sum_j a_j Phi_ij R^2 h_ij
//   {A,B,C}_i = sum_j 2 a_j Phi_ij (R^2)^{0,1,2} m_ij,
//                                        m = 1/(g+g')^2 + 1/((g+g')g) + 1/g^2
// with a_j = w_j rho_j and every j (j = i included).  One lane owns one
// outer point i; j points stream through LDS in chunks of 256 and are read
// as wave-wide broadcasts.  All 1/g, 1/g', 1/(g+g') come from one
// reciprocal of g g' (g+g').
//
// FP64 mode accumulates in FP64.  FP32 mode evaluates each pair in FP32,
// accumulates one 256-point chunk in FP32 and adds the chunk sums into
// FP64 accumulators.
#include "dev_common.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

constexpr int JC = 256;

template <bool HESS>
__global__ __launch_bounds__(256) void k_pair_f64(int64_t npad, const double4 *__restrict__ P0,
                                                  const double4 *__restrict__ P1,
                                                  double *__restrict__ I) {
    __shared__ double4 s0[JC], s1[JC];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double4 a0 = P0[i], a1 = P1[i];
    double E = 0, U = 0, W = 0, A = 0, B = 0, C = 0;
    for (int64_t j0 = 0; j0 < npad; j0 += JC) {
        __syncthreads();
        s0[threadIdx.x] = P0[j0 + threadIdx.x];
        s1[threadIdx.x] = P1[j0 + threadIdx.x];
        __syncthreads();
#pragma unroll 4
        for (int jj = 0; jj < JC; ++jj) {
            const double4 b0 = s0[jj], b1 = s1[jj];
            const double dx = a0.x - b0.x, dy = a0.y - b0.y, dz = a0.z - b0.z;
            const double R2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
            const double g = __builtin_fma(a0.w, R2, a1.x);
            const double gp = __builtin_fma(b0.w, R2, b1.x);
            const double s = g + gp, t = g * gp;
            const double r = rcp64(t * s);
            const double pa = -1.5 * b1.y * r;       // a_j Phi_ij
            const double ig = gp * s * r, is = t * r;
            const double u = pa * (ig + is);
            E += pa;
            U -= u;
            W = __builtin_fma(-u, R2, W);
            if (HESS) {
                const double m2 = 2.0 * pa * __builtin_fma(is, is, __builtin_fma(is, ig, ig * ig));
                A += m2;
                B = __builtin_fma(m2, R2, B);
                C = __builtin_fma(m2 * R2, R2, C);
            }
        }
    }
    I[I_E * npad + i] = E;
    I[I_U * npad + i] = U;
    I[I_W * npad + i] = W;
    if (HESS) {
        I[I_A * npad + i] = A;
        I[I_B * npad + i] = B;
        I[I_C * npad + i] = C;
    }
}

template <bool HESS>
__global__ __launch_bounds__(256) void k_pair_f32(int64_t npad, const float4 *__restrict__ P0,
                                                  const float4 *__restrict__ P1,
                                                  double *__restrict__ I) {
    __shared__ float4 s0[JC], s1[JC];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const float4 a0 = P0[i], a1 = P1[i];
    double E = 0, U = 0, W = 0, A = 0, B = 0, C = 0;
    for (int64_t j0 = 0; j0 < npad; j0 += JC) {
        __syncthreads();
        s0[threadIdx.x] = P0[j0 + threadIdx.x];
        s1[threadIdx.x] = P1[j0 + threadIdx.x];
        __syncthreads();
        float e = 0.f, uu = 0.f, ww = 0.f, aa = 0.f, bb = 0.f, cc = 0.f;
#pragma unroll 8
        for (int jj = 0; jj < JC; ++jj) {
            const float4 b0 = s0[jj], b1 = s1[jj];
            const float dx = a0.x - b0.x, dy = a0.y - b0.y, dz = a0.z - b0.z;
            const float R2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
            const float g = __builtin_fmaf(a0.w, R2, a1.x);
            const float gp = __builtin_fmaf(b0.w, R2, b1.x);
            const float s = g + gp, t = g * gp;
            const float r = rcp32(t * s);
            const float pa = -1.5f * b1.y * r;
            const float ig = gp * s * r, is = t * r;
            const float u = pa * (ig + is);
            e += pa;
            uu -= u;
            ww = __builtin_fmaf(-u, R2, ww);
            if (HESS) {
                const float m2 = 2.f * pa * __builtin_fmaf(is, is, __builtin_fmaf(is, ig, ig * ig));
                aa += m2;
                bb = __builtin_fmaf(m2, R2, bb);
                cc = __builtin_fmaf(m2 * R2, R2, cc);
            }
        }
        E += e;
        U += uu;
        W += ww;
        if (HESS) {
            A += aa;
            B += bb;
            C += cc;
        }
    }
    I[I_E * npad + i] = E;
    I[I_U * npad + i] = U;
    I[I_W * npad + i] = W;
    if (HESS) {
        I[I_A * npad + i] = A;
        I[I_B * npad + i] = B;
        I[I_C * npad + i] = C;
    }
}

// Potential and energy terms (Section II.A):
//   f^rho_i = beta + E_i + rho_i (kappa_r U_i + omega_r W_i)
//   f^gamma_i = rho_i omega_g W_i
//   energy = sum_i a_i (beta + E_i/2), reduced per block in a fixed order.
__global__ __launch_bounds__(256) void k_potential(int64_t n, int64_t npad, double beta,
                                                   const double4 *__restrict__ P1,
                                                   double *__restrict__ F,
                                                   const double *__restrict__ I,
                                                   double *__restrict__ f_rho,
                                                   double *__restrict__ f_gamma,
                                                   double *__restrict__ epart) {
    __shared__ double s[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (i < n) {
        const double Ei = I[I_E * npad + i], Ui = I[I_U * npad + i], Wi = I[I_W * npad + i];
        const double r = F[F_RHO * npad + i];
        const double fr = beta + Ei + r * (F[F_KAR * npad + i] * Ui + F[F_OMR * npad + i] * Wi);
        const double fg = r * F[F_OMG * npad + i] * Wi;
        F[F_FR * npad + i] = fr;
        F[F_FG * npad + i] = fg;
        if (f_rho) f_rho[i] = fr;
        if (f_gamma) f_gamma[i] = fg;
        e = P1[i].y * (beta + 0.5 * Ei);
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) epart[blockIdx.x] = s[0];
}

// Sum of the block partials in block order (one block).
__global__ __launch_bounds__(256) void k_sum_partials(int64_t nb, const double *__restrict__ part,
                                                      double *__restrict__ out) {
    __shared__ double s[256];
    double a = 0.0;
    // each thread sums a contiguous run so the order is fixed
    const int64_t per = (nb + 255) / 256;
    for (int64_t k = threadIdx.x * per; k < min(nb, (int64_t)(threadIdx.x + 1) * per); ++k)
        a += part[k];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

}  // namespace

hipError_t launch_pair_integrals(vv10_plan *p, bool hessian_mode) {
    const unsigned nb = (unsigned)(p->npad / 256);
    if (p->prec == VV10_FP64) {
        if (hessian_mode)
            k_pair_f64<true><<<nb, 256, 0, p->stream>>>(p->npad, p->P0, p->P1, p->I);
        else
            k_pair_f64<false><<<nb, 256, 0, p->stream>>>(p->npad, p->P0, p->P1, p->I);
    } else {
        if (hessian_mode)
            k_pair_f32<true><<<nb, 256, 0, p->stream>>>(p->npad, p->P0f, p->P1f, p->I);
        else
            k_pair_f32<false><<<nb, 256, 0, p->stream>>>(p->npad, p->P0f, p->P1f, p->I);
    }
    return hipGetLastError();
}

hipError_t launch_potential(vv10_plan *p, double *energy, double *f_rho, double *f_gamma) {
    const int64_t nb = p->npad / 256;
    double *epart = p->red;               // [nb] partials, then the energy at red[nb]
    k_potential<<<(unsigned)nb, 256, 0, p->stream>>>(p->n, p->npad, p->beta, p->P1, p->F, p->I,
                                                     f_rho, f_gamma, epart);
    k_sum_partials<<<1, 256, 0, p->stream>>>(nb, epart, energy ? energy : p->red + nb);
    return hipGetLastError();
}

}  // namespace vv10
