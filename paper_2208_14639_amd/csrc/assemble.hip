// Hessian assembly (Section II.B, nine-term split with the weight terms
// zero).  All FP64.
//
// 0. k_sum_splits adds the partial contractions of the j splits.
// 1. k_resp, per point i and perturbation x:
//      Yr = Y_p + rho omega_r Y_q + loc_rho,   Yg = rho omega_g Y_q + loc_gamma
//    (the paper's inner sums sum_j w_j (f^{rho rho}_ij rho^x_j + f^{rho gamma}_ij gamma^x_j)
//    and sum_j w_j (f^{gamma rho}_ij rho^x_j + f^{gamma gamma}_ij gamma^x_j); the local parts are
//    the delta_ij terms, written as derivatives along the perturbation:
//      dk = kappa_r rho^x, dw = omega_r rho^x + omega_g gamma^x,
//      loc_rho   = U dk + W dw + rho^x (kappa_r U + omega_r W)
//                + rho (A kappa_r dk + B (kappa_r dw + omega_r dk) + C omega_r dw)
//                + rho (kappa_rr rho^x U + (omega_rr rho^x + omega_rg gamma^x) W)
//      loc_gamma = rho^x omega_g W + rho (B omega_g dk + C omega_g dw)
//                + rho (omega_rg rho^x + omega_gg gamma^x) W),
//    the grid channels Zr = Z_p + rho omega_r Z_q, Zg = rho omega_g Z_q (with the
//    own-atom slot filled by translational invariance), and
//      R = w (Yr + 2 Zr, Yg + 2 Zg)   written over Y.
// 2. k_gemm: Hpart[s] = sum over a slice of points of L_i^T R_i, L = (rho^x, gamma^x),
//    so that sum_s Hpart[s] = E_GG + 2 E_{G,gr} (E_GG without the rho^{AB} term).
// 3. k_dsum, k_grgr: E_{gr,gr} from the tile sums of a_i D^B_i, reduced per
//    atom pair; diagonal blocks by translational invariance.
// 4. k_hess_final: H = sym(sum_s Hpart[s]) + sym(E_{gr,gr}), sym(M) = (M + M^T)/2.
// 5. gradient: E_G = sum_i w_i (f^rho_i rho^x_i + f^gamma_i gamma^x_i) and
//    E_gr = sum_{i in A} a_i E^{Agr}_i = -sum_{B != A} sum_{i in A} a_i E^{Bgr}_i.
#include "dev_common.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

// Y = Ypart[0] + ... + Ypart[S-1] over the j splits of the contraction, in
// split order and in FP64 (the partials are FP64 or FP32).
template <typename T>
__global__ __launch_bounds__(256) void k_sum_splits(int64_t len, int S, const T *__restrict__ Yp,
                                                    double *__restrict__ Y) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= len) return;
    double a = (double)Yp[k];
    for (int s = 1; s < S; ++s) a += (double)Yp[s * len + k];
    Y[k] = a;
}

__global__ __launch_bounds__(256) void k_resp(
    int64_t n, int64_t npad, int32_t P, int32_t Pp, int32_t n_atom,
    const int32_t *__restrict__ atom_of, const double *__restrict__ F,
    const double *__restrict__ I, const double *__restrict__ L, double *__restrict__ Y,
    const double *__restrict__ Z, double *__restrict__ resp_rho, double *__restrict__ resp_gamma) {
    const int x = blockIdx.y * 64 + (threadIdx.x & 63);
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n || x >= Pp) return;
    double *y0 = Y + (i * 2 + 0) * Pp + x;
    double *y1 = Y + (i * 2 + 1) * Pp + x;
    if (x >= P) {
        *y0 = 0.0;
        *y1 = 0.0;
        return;
    }
    const double w = F[F_W * npad + i], r = F[F_RHO * npad + i];
    const double omr = F[F_OMR * npad + i], omg = F[F_OMG * npad + i];
    const double kar = F[F_KAR * npad + i];
    const double omrr = F[F_OMRR * npad + i], omrg = F[F_OMRG * npad + i];
    const double omgg = F[F_OMGG * npad + i], karr = F[F_KARR * npad + i];
    const double U = I[I_U * npad + i], W = I[I_W * npad + i];
    const double Ai = I[I_A * npad + i], Bi = I[I_B * npad + i], Ci = I[I_C * npad + i];
    const double rx = L[(i * 2 + 0) * Pp + x], gx = L[(i * 2 + 1) * Pp + x];

    const double dk = kar * rx;
    const double dw = omr * rx + omg * gx;
    const double loc_r = U * dk + W * dw + rx * (kar * U + omr * W)
                       + r * (Ai * kar * dk + Bi * (kar * dw + omr * dk) + Ci * omr * dw)
                       + r * (karr * rx * U + (omrr * rx + omrg * gx) * W);
    const double loc_g = rx * omg * W + r * (Bi * omg * dk + Ci * omg * dw)
                       + r * (omrg * rx + omgg * gx) * W;
    const double yp = *y0, yq = *y1;
    const double Yr = yp + r * omr * yq + loc_r;
    const double Yg = r * omg * yq + loc_g;

    const int A = atom_of[i];
    const int B = x / 3, a = x - 3 * B;
    double zp, zq;
    if (B == A) {
        zp = 0.0;
        zq = 0.0;
        for (int C = 0; C < n_atom; ++C) {
            if (C == A) continue;
            zp -= Z[(i * 2 + 0) * Pp + 3 * C + a];
            zq -= Z[(i * 2 + 1) * Pp + 3 * C + a];
        }
    } else {
        zp = Z[(i * 2 + 0) * Pp + x];
        zq = Z[(i * 2 + 1) * Pp + x];
    }
    const double Zr = zp + r * omr * zq, Zg = r * omg * zq;
    *y0 = w * (Yr + 2.0 * Zr);
    *y1 = w * (Yg + 2.0 * Zg);
    if (resp_rho) resp_rho[(int64_t)x * n + i] = Yr;
    if (resp_gamma) resp_gamma[(int64_t)x * n + i] = Yg;
}

// Hpart[s][l][m] = sum_{i in slice s} sum_c L[i][c][l] R[i][c][m]
// 64 x 64 output tile per workgroup, 4 x 4 per thread, 16 (i, c) rows per step.
constexpr int GT = 64, GK = 16;
__global__ __launch_bounds__(256) void k_gemm(int64_t n, int64_t slice, int32_t Pp,
                                              const double *__restrict__ L,
                                              const double *__restrict__ R,
                                              double *__restrict__ Hpart) {
    __shared__ double sL[GK][GT];
    __shared__ double sR[GK][GT];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int l0 = blockIdx.x * GT, m0 = blockIdx.y * GT;
    const int64_t rbeg = (int64_t)blockIdx.z * slice * 2;
    const int64_t rend = min(2 * n, rbeg + slice * 2);
    double acc[4][4] = {};
    for (int64_t k0 = rbeg; k0 < rend; k0 += GK) {
        __syncthreads();
        for (int e = tid; e < GK * GT; e += 256) {
            const int kr = e / GT, cc = e - kr * GT;
            const int64_t row = k0 + kr;
            const bool ok = row < rend;
            sL[kr][cc] = (ok && l0 + cc < Pp) ? L[row * Pp + l0 + cc] : 0.0;
            sR[kr][cc] = (ok && m0 + cc < Pp) ? R[row * Pp + m0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kr = 0; kr < GK; ++kr) {
            double lv[4], rv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lv[q] = sL[kr][ty * 4 + q];
                rv[q] = sR[kr][tx * 4 + q];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_fma(lv[a], rv[b], acc[a][b]);
        }
    }
    double *H = Hpart + (int64_t)blockIdx.z * Pp * Pp;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int l = l0 + ty * 4 + a, m = m0 + tx * 4 + b;
            if (l < Pp && m < Pp) H[(int64_t)l * Pp + m] = acc[a][b];
        }
}

// DS[A][B][c] = sum over the tiles t of atom A of Dpart[t][B][c] (tile order).
__global__ __launch_bounds__(256) void k_dsum(int32_t n_atom, const int32_t *__restrict__ tile_first,
                                              const double *__restrict__ Dpart,
                                              double *__restrict__ DS) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)n_atom * n_atom * 9) return;
    const int A = (int)(k / (9LL * n_atom));
    const int rem = (int)(k - (int64_t)A * 9 * n_atom);   // B * 9 + c
    double v = 0.0;
    for (int t = tile_first[A]; t < tile_first[A + 1]; ++t) v += Dpart[(int64_t)t * n_atom * 9 + rem];
    DS[k] = v;
}

// E_{gr,gr}[(A,a)][(B,b)] = DS[A][B][(a,b)] for B != A, and the diagonal
// blocks -sum_{B != A} DS[A][B][(a,b)] (translational invariance).
__device__ __forceinline__ int sym_index(int a, int b) {
    if (a == b) return a;                 // xx, yy, zz
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? (hi == 1 ? 3 : 4) : 5;   // xy, xz, yz
}

__global__ __launch_bounds__(256) void k_grgr(int32_t n_atom, int32_t P, const double *__restrict__ DS,
                                              double *__restrict__ Hgr) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)P * P) return;
    const int l = (int)(k / P), m = (int)(k % P);
    const int A = l / 3, a = l % 3, B = m / 3, b = m % 3;
    const int c = sym_index(a, b);
    double v = 0.0;
    if (A != B) {
        v = DS[((int64_t)A * n_atom + B) * 9 + c];
    } else {
        for (int C = 0; C < n_atom; ++C)
            if (C != A) v -= DS[((int64_t)A * n_atom + C) * 9 + c];
    }
    Hgr[k] = v;
}

__global__ __launch_bounds__(256) void k_hess_final(int32_t P, int32_t Pp, int32_t S,
                                                    const double *__restrict__ Hpart,
                                                    const double *__restrict__ Hgr,
                                                    double *__restrict__ hess) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)P * P) return;
    const int l = (int)(k / P), m = (int)(k % P);
    double hlm = 0.0, hml = 0.0;
    for (int s = 0; s < S; ++s) {
        hlm += Hpart[((int64_t)s * Pp + l) * Pp + m];
        hml += Hpart[((int64_t)s * Pp + m) * Pp + l];
    }
    hess[k] = 0.5 * (hlm + hml) + 0.5 * (Hgr[(int64_t)l * P + m] + Hgr[(int64_t)m * P + l]);
}

// Gradient E_G partials: gpart[s][x] = sum_{i in slice s} w_i (f^rho_i L[i][0][x] + f^gamma_i L[i][1][x])
__global__ __launch_bounds__(256) void k_grad_part(int64_t n, int64_t npad, int64_t slice,
                                                   int32_t Pp, const double *__restrict__ F,
                                                   const double *__restrict__ L,
                                                   double *__restrict__ gpart) {
    const int64_t ib = (int64_t)blockIdx.x * slice, ie = min(n, ib + slice);
    for (int x = threadIdx.x; x < Pp; x += 256) {
        double a = 0.0;
        for (int64_t i = ib; i < ie; ++i) {
            const double w = F[F_W * npad + i];
            a += w * (F[F_FR * npad + i] * L[(i * 2 + 0) * Pp + x] +
                      F[F_FG * npad + i] * L[(i * 2 + 1) * Pp + x]);
        }
        gpart[(int64_t)blockIdx.x * Pp + x] = a;
    }
}

__global__ __launch_bounds__(256) void k_grad_final(int32_t n_atom, int32_t P, int32_t Pp,
                                                    int32_t nslices, const double *__restrict__ gpart,
                                                    const double *__restrict__ DS,
                                                    double *__restrict__ grad) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= P) return;
    double g = 0.0;
    for (int s = 0; s < nslices; ++s) g += gpart[(int64_t)s * Pp + x];
    const int A = x / 3, a = x % 3;
    double gr = 0.0;
    for (int B = 0; B < n_atom; ++B)
        if (B != A) gr -= DS[((int64_t)A * n_atom + B) * 9 + 6 + a];
    grad[x] = g + gr;
}

}  // namespace

hipError_t launch_assemble(vv10_plan *p, double *hess, double *grad, double *resp_rho,
                           double *resp_gamma) {
    const Workspace &ws = p->ws;
    const int64_t n = p->n;
    {
        const int64_t len = p->npad * 2 * ws.Pp;
        const unsigned nb = (unsigned)((len + 255) / 256);
        if (p->prec != VV10_FP64)
            k_sum_splits<float><<<nb, 256, 0, p->stream>>>(len, ws.jsplit,
                                                           static_cast<const float *>(ws.Ypart), ws.Y);
        else if (ws.Ypart != ws.Y)
            k_sum_splits<double><<<nb, 256, 0, p->stream>>>(len, ws.jsplit,
                                                            static_cast<const double *>(ws.Ypart), ws.Y);
    }
    {
        dim3 grid((unsigned)((n + 3) / 4), (unsigned)((ws.Pp + 63) / 64));
        k_resp<<<grid, 256, 0, p->stream>>>(n, p->npad, ws.P, ws.Pp, p->n_atom, p->atom_of, p->F,
                                            p->I, ws.L, ws.Y, ws.Z, resp_rho, resp_gamma);
    }
    const int64_t slice = (n + ws.gsplit - 1) / ws.gsplit;
    {
        dim3 grid((unsigned)((ws.Pp + GT - 1) / GT), (unsigned)((ws.Pp + GT - 1) / GT),
                  (unsigned)ws.gsplit);
        k_gemm<<<grid, 256, 0, p->stream>>>(n, slice, ws.Pp, ws.L, ws.Y, ws.Hpart);
    }
    const int64_t PP = (int64_t)ws.P * ws.P;
    const int64_t nds = (int64_t)p->n_atom * p->n_atom * 9;
    k_dsum<<<(unsigned)((nds + 255) / 256), 256, 0, p->stream>>>(p->n_atom, p->d_tile_first,
                                                                 ws.Dpart, ws.DS);
    k_grgr<<<(unsigned)((PP + 255) / 256), 256, 0, p->stream>>>(p->n_atom, ws.P, ws.DS, ws.Hgr);
    k_hess_final<<<(unsigned)((PP + 255) / 256), 256, 0, p->stream>>>(ws.P, ws.Pp, ws.gsplit,
                                                                      ws.Hpart, ws.Hgr, hess);
    if (grad) {
        const int ns = 256;
        const int64_t gs = (n + ns - 1) / ns;
        k_grad_part<<<ns, 256, 0, p->stream>>>(n, p->npad, gs, ws.Pp, p->F, ws.L, ws.gpart);
        k_grad_final<<<(unsigned)((ws.P + 255) / 256), 256, 0, p->stream>>>(
            p->n_atom, ws.P, ws.Pp, ns, ws.gpart, ws.DS, grad);
    }
    return hipGetLastError();
}

}  // namespace vv10
