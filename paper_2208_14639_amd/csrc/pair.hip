// Pair kernel: the inner integrals of Section II.A (E_i, U_i, W_i) and,
// in Hessian mode, those of Section II.B (A_i, B_i, C_i):
//   E_i = sum_j a_j Phi_ij
//   U_i = -sum_j a_j Phi_ij h_ij,           h = 1/(g+g') + 1/g
//   W_i = -sum_j a_j Phi_ij R^2 h_ij
//   {A,B,C}_i = sum_j 2 a_j Phi_ij (R^2)^{0,1,2} m_ij,
//                                        m = 1/(g+g')^2 + 1/((g+g')g) + 1/g^2
// with a_j = w_j rho_j and every j (j = i included: its term is added in
// FP64, the loops run over j != i).  One lane owns one
// outer point i; j points stream through LDS and are read as wave-wide
// broadcasts.  All 1/g, 1/g', 1/(g+g') come from one reciprocal
// r = 1/(g g' (g+g')); the loop sums p = a_j r times h, R^2 h and
// m (R^2)^{0,1,2} (m = h^2 - 1/((g+g') g)), and the constant factors
// (a_j Phi = -3/2 p) are applied to the sums.
#include <algorithm>

#include "dev_common.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

constexpr int JC = 256;   // j points staged per block step; wave w takes [64 w, 64 w + 64)

// Sums of one wave's 64 j of an LDS chunk.  SELF: the chunk holds the
// outer points themselves (lane l's own point at jj = jself), whose pair is
// left out (added in FP64 at the end).
template <typename T, typename T4, bool HESS, bool SELF>
__device__ __forceinline__ void pair_run(const T4 a0, const T4 a1, const T4 *s0, const T4 *s1,
                                         int jbeg, int jself, T *c) {
#pragma unroll 8
    for (int jj = jbeg; jj < jbeg + 64; ++jj) {
        const T4 b0 = s0[jj], b1 = s1[jj];
        const T dx = a0.x - b0.x, dy = a0.y - b0.y, dz = a0.z - b0.z;
        const T R2 = dx * dx + dy * dy + dz * dz;
        const T g = a0.w * R2 + a1.x;
        const T gp = b0.w * R2 + b1.x;
        const T s = g + gp, t = g * gp;
        T r;
        if constexpr (sizeof(T) == 8) r = rcp64(t * s); else r = rcp32(t * s);
        T pj = b1.y * r;
        if (SELF) pj = jj == jself ? T(0) : pj;
        const T ig = gp * (s * r), is = t * r;
        const T h = ig + is;
        const T ph = pj * h;
        c[0] += pj;
        c[1] += ph;
        c[2] += ph * R2;
        if (HESS) {
            const T pm = pj * (h * h - is * ig);
            const T pmR2 = pm * R2;
            c[3] += pm;
            c[4] += pmR2;
            c[5] += pmR2 * R2;
        }
    }
}

// One workgroup = 4 waves sharing 64 outer points (one per lane); each wave
// takes a quarter of every 256-point j chunk, and the four partial sums are
// added in wave order at the end.  blockIdx.y selects a contiguous j range
// (a split); splits write partial integrals [split][6][npad] that
// k_sum_integrals adds in split order.  Mixed mode evaluates in FP32 and
// adds each 64-point run into FP64 accumulators.  The self pair is left out
// of the loops; the split that holds the outer points adds it in FP64 from
// the FP64 point data Pd (kappa, a = w rho).
template <typename T, typename T4, bool HESS>
__global__ __launch_bounds__(256) void k_pair(int64_t npad, int64_t jlen,
                                              const T4 *__restrict__ P0,
                                              const T4 *__restrict__ P1,
                                              const double4 *__restrict__ Pd,
                                              double *__restrict__ Ipart) {
    __shared__ T4 s0[JC], s1[JC];
    __shared__ double red[4][6][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tb = (int64_t)blockIdx.x * 64;
    const int64_t i = tb + lane;
    const int64_t jbeg = (int64_t)blockIdx.y * jlen;
    const int64_t jend = min(npad, jbeg + jlen);
    const T4 a0 = P0[i], a1 = P1[i];
    double E = 0, U = 0, W = 0, A = 0, B = 0, C = 0;
    for (int64_t j0 = jbeg; j0 < jend; j0 += JC) {
        __syncthreads();
        s0[threadIdx.x] = P0[j0 + threadIdx.x];
        s1[threadIdx.x] = P1[j0 + threadIdx.x];
        __syncthreads();
        T c[6] = {0, 0, 0, 0, 0, 0};
        if (j0 + 64 * wave == tb)   // this wave's run holds the outer points
            pair_run<T, T4, HESS, true>(a0, a1, s0, s1, 64 * wave, 64 * wave + lane, c);
        else
            pair_run<T, T4, HESS, false>(a0, a1, s0, s1, 64 * wave, 0, c);
        E += (double)c[0];
        U += (double)c[1];
        W += (double)c[2];
        if (HESS) {
            A += (double)c[3];
            B += (double)c[4];
            C += (double)c[5];
        }
    }
    red[wave][0][lane] = E;
    red[wave][1][lane] = U;
    red[wave][2][lane] = W;
    red[wave][3][lane] = A;
    red[wave][4][lane] = B;
    red[wave][5][lane] = C;
    __syncthreads();
    const int nout = HESS ? 6 : 3;
    // self pair (W, B, C have a factor R^2 and get none): E += a Phi,
    // U += -a Phi h, A += 2 a Phi m
    const bool own = tb >= jbeg && tb < jend;
    double self[6] = {0, 0, 0, 0, 0, 0};
    if (own) {
        const double4 pd = Pd[i];
        const SelfPair q = self_pair(pd.x);
        self[0] = pd.y * q.phi;
        self[1] = -pd.y * q.phi * q.h;
        self[3] = 2.0 * pd.y * q.phi * q.m;
    }
    for (int k = wave; k < nout; k += 4) {
        const double sc = k == 0 ? -1.5 : (k < 3 ? 1.5 : -3.0);   // E; U, W; A, B, C
        const double v = sc * (red[0][k][lane] + red[1][k][lane] + red[2][k][lane] + red[3][k][lane]);
        Ipart[((int64_t)blockIdx.y * NI + k) * npad + i] = v + self[k];
    }
}

// I[k][i] = sum over splits of Ipart[s][k][i], in split order.
__global__ __launch_bounds__(256) void k_sum_integrals(int64_t npad, int nout, int S,
                                                       const double *__restrict__ Ipart,
                                                       double *__restrict__ I) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)nout * npad) return;
    const int k = (int)(e / npad);
    const int64_t i = e - (int64_t)k * npad;
    double a = 0.0;
#pragma unroll 8
    for (int s = 0; s < S; ++s) a += Ipart[((int64_t)s * NI + k) * npad + i];
    I[k * npad + i] = a;
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
                                                   double *__restrict__ epart,
                                                   const int32_t *__restrict__ valid) {
    __shared__ double s[256];
    if (valid && *valid != 0) return;   // invalid inputs: no output is written
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (i < n) {
        const double Ei = I[I_E * npad + i], Ui = I[I_U * npad + i], Wi = I[I_W * npad + i];
        const double r = F[F_RHO * npad + i];
        const double fr = beta + Ei + r * (F[F_KAR * npad + i] * Ui + F[F_OMR * npad + i] * Wi);
        const double fg = r * F[F_OMG * npad + i] * Wi;
        F[F_FR * npad + i] = fr;
        F[F_FG * npad + i] = fg;
        F[F_F0 * npad + i] = r * (beta + Ei);
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
                                                      double *__restrict__ out,
                                                      const int32_t *__restrict__ valid) {
    __shared__ double s[256];
    if (valid && *valid != 0) return;
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

int pair_splits(int64_t npad) {
    // enough workgroups for about eight waves per SIMD on 256 CUs
    const int64_t blocks = npad / 64;
    int S = (int)std::min<int64_t>(16, std::max<int64_t>(1, (2048 + blocks - 1) / blocks));
    while (S > 1 && npad / S < JC) --S;
    return S;
}

hipError_t launch_pair_integrals(vv10_plan *p, bool hessian_mode, double *I_out) {
    const int S = pair_splits(p->npad);
    const int64_t jlen = ((p->npad / S + JC - 1) / JC) * JC;
    dim3 grid((unsigned)(p->npad / 64), (unsigned)S);
    double *Ipart = S == 1 ? I_out : p->Ipart;
    if (p->prec == VV10_FP64) {
        if (hessian_mode)
            k_pair<double, double4, true><<<grid, 256, 0, p->stream>>>(p->npad, jlen, p->P0, p->P1,
                                                                       p->P1, Ipart);
        else
            k_pair<double, double4, false><<<grid, 256, 0, p->stream>>>(p->npad, jlen, p->P0, p->P1,
                                                                        p->P1, Ipart);
    } else {
        if (hessian_mode)
            k_pair<float, float4, true><<<grid, 256, 0, p->stream>>>(p->npad, jlen, p->P0f, p->P1f,
                                                                     p->P1, Ipart);
        else
            k_pair<float, float4, false><<<grid, 256, 0, p->stream>>>(p->npad, jlen, p->P0f, p->P1f,
                                                                      p->P1, Ipart);
    }
    if (S > 1) {
        const int nout = hessian_mode ? 6 : 3;
        const int64_t tot = (int64_t)nout * p->npad;
        k_sum_integrals<<<(unsigned)((tot + 255) / 256), 256, 0, p->stream>>>(p->npad, nout, S, Ipart, I_out);
    }
    return hipGetLastError();
}

hipError_t launch_potential(vv10_plan *p, double *energy, double *f_rho, double *f_gamma,
                            const int32_t *valid) {
    const int64_t nb = p->npad / 256;
    double *epart = p->red;               // [nb] partials, then the energy at red[nb]
    k_potential<<<(unsigned)nb, 256, 0, p->stream>>>(p->n, p->npad, p->beta, p->P1, p->F, p->I,
                                                     f_rho, f_gamma, epart, valid);
    k_sum_partials<<<1, 256, 0, p->stream>>>(nb, epart, energy ? energy : p->red + nb, valid);
    return hipGetLastError();
}

}  // namespace vv10
