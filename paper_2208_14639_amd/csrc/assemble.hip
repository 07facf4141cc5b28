// Hessian assembly (Section II.B, nine-term split).  All FP64.
//
// 1. k_resp, one wave per point i, lanes over the perturbations x:
//      Y = sum of the contraction's j-split partials (split order, FP64)
//          plus the self pair j = i, which the contraction leaves out:
//          Y_p += K_pp(i, i) p_i in FP64
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
//    the grid channels Zr = Z_p + rho omega_r Z_q, Zg = rho omega_g Z_q (the
//    own-atom slot filled by translational invariance, a wave reduction over
//    the other atoms' slots), and R = w (Yr + 2 Zr, Yg + 2 Zg), written over Y.
//    Optional outputs: Yr, Yg (response rows) and Yr + Zr, Yg + Zg (the
//    grid-level coefficients of the Fock nuclear derivative).
//    With weight derivatives w^x (weights that move with the nuclei) the
//    weight contraction's (Y_pv, Y_qv, Y_vv) and the grid channel
//    Ze = E^{xgr} (own slot by invariance again) add
//      Wr = Y_pv + rho omega_r Y_qv,  Wg = rho omega_g Y_qv
//      R += (2 w Wr + 2 w^x f^rho, 2 w Wg + 2 w^x f^gamma),
//      Rw = rho (Y_vv + 2 Ze)     (right factor of the w^x rows),
//    and Wr, Wg to the Fock coefficients (F^A_w without its first line).
// 2. k_gemm: per slice s of points, Hpart[s][l][m] = sum_i L_i^T R_i with
//    L = (rho^x, gamma^x) on FP64 MFMA, so that sum_s Hpart[s] = E_GG + 2 E_{G,gr}
//    (E_GG without the rho^{AB} term); row Pp of each slice holds the gradient
//    part E_G = sum_i w_i (f^rho_i rho^x_i + f^gamma_i gamma^x_i).  With
//    weight derivatives a second GEMM over the rows L = w^x, R = Rw adds
//    E_ww + 2 E_{w,gr} (E_ww = sum_i w^A_i rho_i E^{Bw}_i, symmetric) and, in
//    row Pp, E_w = sum_i w^x_i rho_i (beta + E_i); the R terms above add
//    2 E_{G,w}.  Symmetrised, this is the nine-term split without the
//    caller's rho^{AB} and w^{AB} sums.
// 3. k_hsum: Hsum = sum_s Hpart[s] in a fixed order (the w^x slices after
//    the others).
// 4. k_dsum: E_{gr,gr} tile sums of a_i D^B_i reduced per atom pair.
// 5. k_finish: H = sym(Hsum) + sym(E_{gr,gr}), sym(M) = (M + M^T)/2, with the
//    diagonal blocks of E_{gr,gr} from translational invariance, and the
//    gradient E_G + E_gr, E_gr = sum_{i in A} a_i E^{Agr}_i
//    = -sum_{B != A} sum_{i in A} a_i E^{Bgr}_i.
#include "dev_common.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

// Per-point quantities of the same-point (delta_ij) terms.
struct PointFields {
    double w, r, omr, omg, kar, omrr, omrg, omgg, karr, U, W, A, B, C;
};

__device__ __forceinline__ PointFields point_fields(const double *__restrict__ F,
                                                    const double *__restrict__ I, int64_t npad,
                                                    int64_t i) {
    PointFields f;
    f.w = F[F_W * npad + i];
    f.r = F[F_RHO * npad + i];
    f.omr = F[F_OMR * npad + i];
    f.omg = F[F_OMG * npad + i];
    f.kar = F[F_KAR * npad + i];
    f.omrr = F[F_OMRR * npad + i];
    f.omrg = F[F_OMRG * npad + i];
    f.omgg = F[F_OMGG * npad + i];
    f.karr = F[F_KARR * npad + i];
    f.U = I[I_U * npad + i];
    f.W = I[I_W * npad + i];
    f.A = I[I_A * npad + i];
    f.B = I[I_B * npad + i];
    f.C = I[I_C * npad + i];
    return f;
}

// Yr, Yg of one point and perturbation from the contraction's channel sums
// (yp, yq) and the perturbation values (rx = rho^x, gx = gamma^x).
__device__ __forceinline__ void point_response(const PointFields &f, double rx, double gx,
                                               double yp, double yq, double &Yr, double &Yg) {
    const double dk = f.kar * rx;
    const double dw = f.omr * rx + f.omg * gx;
    const double loc_r = f.U * dk + f.W * dw + rx * (f.kar * f.U + f.omr * f.W)
                       + f.r * (f.A * f.kar * dk + f.B * (f.kar * dw + f.omr * dk) + f.C * f.omr * dw)
                       + f.r * (f.karr * rx * f.U + (f.omrr * rx + f.omrg * gx) * f.W);
    const double loc_g = rx * f.omg * f.W + f.r * (f.B * f.omg * dk + f.C * f.omg * dw)
                       + f.r * (f.omrg * rx + f.omgg * gx) * f.W;
    Yr = yp + f.r * f.omr * yq + loc_r;
    Yg = f.r * f.omg * yq + loc_g;
}

// Inputs of the weight-derivative terms (all null without weight derivatives).
template <typename T>
struct WeightIn {
    const T *Ypart;        // [S][npad][3][Pp] (Y_pv, Y_qv, Y_vv) partials
    const double *Lw;      // [npad][Pp] w^x
    const double *Ze;      // [npad][Pp] E^{xgr} (own slot not written)
    double *Rw;            // [npad][Pp] output
};

// One wave per point; the partials are FP64 ([S][npad][2][Pp]; with one
// split they alias Y, read before R is written in place).
template <typename T, bool WT>
__global__ __launch_bounds__(256) void k_resp(
    int64_t n, int64_t npad, int32_t P, int32_t Pp, int32_t S, const int32_t *__restrict__ atom_of,
    const double4 *__restrict__ P1, const double *__restrict__ F, const double *__restrict__ I,
    const double *__restrict__ L, const T *Ypart, double *Y, const double *__restrict__ Z, WeightIn<T> wt,
    double *__restrict__ resp_rho, double *__restrict__ resp_gamma, double *__restrict__ fock_rho,
    double *__restrict__ fock_gamma) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n) return;
    const PointFields f = point_fields(F, I, npad, i);
    const int A = atom_of[i];
    // the self pair, left out of the contraction: K_pp p_i (and for the
    // weight rows (Phi + c Phi_g) v_i, Phi v_i), in FP64
    const double4 pd = P1[i];
    const double kself = self_kpp(pd.x, pd.z);
    const SelfPair sq = self_pair(pd.x);
    const double kself_pv = sq.phi + pd.z * sq.phig, kself_vv = sq.phi;
    const double *z0 = Z + (i * 2 + 0) * Pp, *z1 = Z + (i * 2 + 1) * Pp;
    const double *ze = WT ? wt.Ze + i * Pp : nullptr;

    // own-atom slot: -sum over the other atoms' slots of the same direction
    double own0[3] = {0.0, 0.0, 0.0}, own1[3] = {0.0, 0.0, 0.0}, own2[3] = {0.0, 0.0, 0.0};
    for (int x0 = 0; x0 < P; x0 += 64) {
        const int x = x0 + lane;
        const bool use = x < P && x / 3 != A;
        const double v0 = use ? z0[x] : 0.0, v1 = use ? z1[x] : 0.0;
        const double v2 = (WT && use) ? ze[x] : 0.0;
        const int a = x % 3;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            own0[d] -= wave_sum(a == d ? v0 : 0.0);
            own1[d] -= wave_sum(a == d ? v1 : 0.0);
            if (WT) own2[d] -= wave_sum(a == d ? v2 : 0.0);
        }
    }

    const int64_t len = npad * 2 * Pp;
    for (int x = lane; x < Pp; x += 64) {
        double *y0 = Y + (i * 2 + 0) * Pp + x;
        double *y1 = Y + (i * 2 + 1) * Pp + x;
        if (x >= P) {
            *y0 = 0.0;
            *y1 = 0.0;
            if (WT) wt.Rw[i * Pp + x] = 0.0;
            continue;
        }
        const int64_t o = (i * 2) * Pp + x;
        double yp = (double)Ypart[o], yq = (double)Ypart[o + Pp];
        for (int s = 1; s < S; ++s) {
            yp += (double)Ypart[s * len + o];
            yq += (double)Ypart[s * len + o + Pp];
        }
        yp += kself * (f.w * L[o]);
        double Yr, Yg;
        point_response(f, L[o], L[o + Pp], yp, yq, Yr, Yg);
        const int a = x % 3;
        const bool self = x / 3 == A;
        const double o0 = a == 0 ? own0[0] : (a == 1 ? own0[1] : own0[2]);
        const double o1 = a == 0 ? own1[0] : (a == 1 ? own1[1] : own1[2]);
        const double zp = self ? o0 : z0[x];
        const double zq = self ? o1 : z1[x];
        const double Zr = zp + f.r * f.omr * zq, Zg = f.r * f.omg * zq;
        double Wr = 0.0, Wg = 0.0;
        if (WT) {
            const int64_t lw = npad * 3 * Pp, ow = (i * 3) * Pp + x;
            double ypv = (double)wt.Ypart[ow], yqv = (double)wt.Ypart[ow + Pp];
            double yvv = (double)wt.Ypart[ow + 2 * Pp];
            for (int s = 1; s < S; ++s) {
                ypv += (double)wt.Ypart[s * lw + ow];
                yqv += (double)wt.Ypart[s * lw + ow + Pp];
                yvv += (double)wt.Ypart[s * lw + ow + 2 * Pp];
            }
            const double vself = wt.Lw[i * Pp + x] * f.r;   // v_i = w^x_i rho_i
            ypv += kself_pv * vself;
            yvv += kself_vv * vself;
            const double o2 = a == 0 ? own2[0] : (a == 1 ? own2[1] : own2[2]);
            const double zev = self ? o2 : ze[x];
            const double wx = wt.Lw[i * Pp + x];
            Wr = ypv + f.r * f.omr * yqv;
            Wg = f.r * f.omg * yqv;
            *y0 = f.w * (Yr + 2.0 * Zr + 2.0 * Wr) + 2.0 * wx * F[F_FR * npad + i];
            *y1 = f.w * (Yg + 2.0 * Zg + 2.0 * Wg) + 2.0 * wx * F[F_FG * npad + i];
            wt.Rw[i * Pp + x] = f.r * (yvv + 2.0 * zev);
        } else {
            *y0 = f.w * (Yr + 2.0 * Zr);
            *y1 = f.w * (Yg + 2.0 * Zg);
        }
        if (resp_rho) resp_rho[(int64_t)x * n + i] = Yr;
        if (resp_gamma) resp_gamma[(int64_t)x * n + i] = Yg;
        if (fock_rho) fock_rho[(int64_t)x * n + i] = Yr + Zr + Wr;
        if (fock_gamma) fock_gamma[(int64_t)x * n + i] = Yg + Zg + Wg;
    }
}

// Trial-density response: f^{rho,t}_i = Yr, f^{gamma,t}_i = Yg of
// point_response for every trial column t (the perturbation packing wrote
// L = (rho^t, 2 grad rho . grad rho^t), which carries the factor 2 of the
// gamma terms).  32 points x 64 columns per workgroup, transposed through
// LDS so that the [n_t][N] outputs are written along points.
constexpr int TRI = 32, TRX = 64;
template <typename T>
__global__ __launch_bounds__(256) void k_trial_resp(
    int64_t n, int64_t npad, int32_t P, int32_t Pp, int32_t S, const double4 *__restrict__ P1,
    const double *__restrict__ F, const double *__restrict__ I, const double *__restrict__ L,
    const T *__restrict__ Ypart, double *__restrict__ f_rho_t, double *__restrict__ f_gamma_t) {
    __shared__ double sR[TRI][TRX + 1], sG[TRI][TRX + 1];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * TRI;
    const int x = blockIdx.y * TRX + tx;
    const int64_t len = npad * 2 * Pp;
    for (int rr = ty; rr < TRI; rr += 4) {
        const int64_t i = i0 + rr;
        double Yr = 0.0, Yg = 0.0;
        if (i < n && x < P) {
            const int64_t o = (i * 2) * Pp + x;
            double yp = (double)Ypart[o], yq = (double)Ypart[o + Pp];
            for (int s = 1; s < S; ++s) {
                yp += (double)Ypart[s * len + o];
                yq += (double)Ypart[s * len + o + Pp];
            }
            // the self pair, left out of the contraction (FP64)
            const double4 pd = P1[i];
            yp += self_kpp(pd.x, pd.z) * (F[F_W * npad + i] * L[o]);
            point_response(point_fields(F, I, npad, i), L[o], L[o + Pp], yp, yq, Yr, Yg);
        }
        sR[rr][tx] = Yr;
        sG[rr][tx] = Yg;
    }
    __syncthreads();
    const int il = tid & (TRI - 1);
    for (int c = tid / TRI; c < TRX; c += 256 / TRI) {
        const int xx = blockIdx.y * TRX + c;
        const int64_t i = i0 + il;
        if (xx < P && i < n) {
            f_rho_t[(int64_t)xx * n + i] = sR[il][c];
            f_gamma_t[(int64_t)xx * n + i] = sG[il][c];
        }
    }
}

// Hpart[s] (rows 0..Pp-1) = sum over the rows k of slice s of L[k][l] R[k][m];
// row Pp = sum_k L[k][l] wf[k].  NCH = 2: rows k = 2 i + c of (rho^x, gamma^x)
// with wf[2i + c] = w_i (f^rho_i, f^gamma_i); NCH = 1: rows k = i of w^x with
// wf[i] = rho_i (beta + E_i).
// Workgroup (tl, tm, s): output tile rows 64 tl.., columns 64 tm..; its four
// waves take consecutive quarters of the slice, each on v_mfma_f64_16x16x4
// with L and R read straight from memory (A = L^T, B = R, K over rows), and
// are added in wave order through LDS.
template <int NCH>
__global__ __launch_bounds__(256, 2) void k_gemm(int64_t n, int64_t npad, int64_t slice,
                                                 int32_t Pp, const double *__restrict__ F,
                                                 const double *__restrict__ L,
                                                 const double *__restrict__ R,
                                                 double *__restrict__ Hpart) {
    __shared__ double sT[64 * 64 + 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ll = lane & 15, kk = lane >> 4;
    const int l0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
    const bool grad = blockIdx.y == 0;
    const int nlb = min(4, (Pp - l0) / 16), nmb = min(4, (Pp - m0) / 16);   // Pp % 16 == 0
    const int64_t rows = NCH * n;
    const int64_t sb = min(rows, (int64_t)blockIdx.z * slice * NCH), se = min(rows, sb + slice * NCH);
    const int64_t q = (se - sb + 3) / 4;
    const int64_t rb = min(se, sb + wave * q), re = min(se, rb + q);
    v4d acc[4][4];
    double gacc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
    // four k steps per iteration, their loads issued before their MFMAs, so
    // that several steps' loads are in flight together (one workgroup per
    // CU leaves little latency hiding to other waves); the MFMAs of each
    // accumulator still run in k order
    for (int64_t k00 = rb; k00 < re; k00 += 16) {
        // loads without branches, from clamped in-range addresses (finite
        // values); rows past the slice and columns past Pp are zeroed by a
        // multiplication, so that no load waits for another
        double av[4][4], bv[4][4], wa[4], wb[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int64_t k = k00 + 4 * st + kk;
            const bool ok = k < re;
            const int64_t kr = ok ? k : rb;
            const double on = ok ? 1.0 : 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a)
                av[st][a] = L[kr * Pp + min(l0 + 16 * a, Pp - 16) + ll] * (a < nlb ? on : 0.0);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                bv[st][b] = R[kr * Pp + min(m0 + 16 * b, Pp - 16) + ll] * (b < nmb ? on : 0.0);
            if (NCH == 2) {
                const int64_t pt = kr >> 1;
                wa[st] = F[F_W * npad + pt] * on;
                wb[st] = F[((kr & 1) ? F_FG : F_FR) * npad + pt];
            } else {
                wa[st] = F[F_F0 * npad + kr] * on;
                wb[st] = 1.0;
            }
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const double wf = NCH == 2 ? wa[st] * wb[st] : wa[st];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st][a], bv[st][b], acc[a][b],
                                                                     0, 0, 0);
            if (grad)
#pragma unroll
                for (int a = 0; a < 4; ++a) gacc[a] = __builtin_fma(av[st][a], wf, gacc[a]);
        }
    }
    // gradient: sum the four k lanes of each column
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gacc[a] += __shfl_xor(gacc[a], 16, 64);
        gacc[a] += __shfl_xor(gacc[a], 32, 64);
    }
    // D layout of v_mfma_f64_16x16x4 (measured on gfx950): item r of lane l
    // holds row 4 r + l/16, column l%16 of the 16 x 16 block
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double *d = sT + (16 * a + 4 * r + kk) * 64 + 16 * b + ll;
                        *d = w == 0 ? acc[a][b][r] : *d + acc[a][b][r];
                    }
            if (kk == 0)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    double *d = sT + 64 * 64 + 16 * a + ll;
                    *d = w == 0 ? gacc[a] : *d + gacc[a];
                }
        }
        __syncthreads();
    }
    double *H = Hpart + (int64_t)blockIdx.z * (Pp + 1) * Pp;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int rr = e >> 6, cc = e & 63;
        if (l0 + rr < Pp && m0 + cc < Pp) H[(int64_t)(l0 + rr) * Pp + m0 + cc] = sT[e];
    }
    if (grad && tid < 64 && l0 + tid < Pp) H[(int64_t)Pp * Pp + l0 + tid] = sT[64 * 64 + tid];
}

// Hsum[e] = sum_s Hpart[s][e], e < (Pp + 1) Pp, over the S slices of Hpart
// and then the S2 slices of H2: 64 entries per workgroup, the four waves sum
// consecutive quarters of the slices, added in wave order.
// 16 waves per 64 elements, each over a sixteenth of the slices, so that
// the few workgroups of a small Hessian keep enough loads in flight.
constexpr int kHsumWaves = 16;
__global__ __launch_bounds__(64 * kHsumWaves) void k_hsum(int64_t len, int S,
                                                          const double *__restrict__ Hpart, int S2,
                                                          const double *__restrict__ H2,
                                                          double *__restrict__ Hsum) {
    __shared__ double part[kHsumWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    const int St = S + S2;
    const int q = (St + kHsumWaves - 1) / kHsumWaves;
    const int sb = min(St, wave * q), se = min(St, sb + q);
    double a = 0.0;
    if (e < len)
#pragma unroll 16
        for (int s = sb; s < se; ++s)
            a += s < S ? Hpart[(int64_t)s * len + e] : H2[(int64_t)(s - S) * len + e];
    part[wave][lane] = a;
    __syncthreads();
    if (wave == 0 && e < len) {
        double t = part[0][lane];
#pragma unroll
        for (int w = 1; w < kHsumWaves; ++w) t += part[w][lane];
        Hsum[e] = t;
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
    // the own-atom slot (B = A) is never formed by the grid pass (its terms
    // follow from translational invariance in k_finish): zero, not read
    if (rem / 9 == A) {
        DS[k] = 0.0;
        return;
    }
    double v = 0.0;
#pragma unroll 8
    for (int t = tile_first[A]; t < tile_first[A + 1]; ++t) v += Dpart[(int64_t)t * n_atom * 9 + rem];
    DS[k] = v;
}

__device__ __forceinline__ int sym_index(int a, int b) {
    if (a == b) return a;                 // xx, yy, zz
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo == 0 ? (hi == 1 ? 3 : 4) : 5;   // xy, xz, yz
}

// E_{gr,gr}[(A,a)][(B,b)] = DS[A][B][(a,b)] for B != A; the diagonal blocks
// are -sum_{C != A} DS[A][C][(a,b)] (translational invariance).  The D sums
// are symmetric in the atom pair and formed for A < B only.
__device__ __forceinline__ double dsym(int32_t n_atom, const double *__restrict__ DS, int A, int B,
                                       int c) {
    const int lo = A < B ? A : B, hi = A < B ? B : A;
    return DS[((int64_t)lo * n_atom + hi) * 9 + c];
}

__device__ __forceinline__ double egrgr(int32_t n_atom, const double *__restrict__ DS, int A, int B,
                                        int c) {
    if (A != B) return dsym(n_atom, DS, A, B, c);
    // every load issued (the C = A entry is read and discarded), so that
    // they are in flight together
    double v = 0.0;
#pragma unroll 8
    for (int C = 0; C < n_atom; ++C) {
        const double d = dsym(n_atom, DS, A, C, c);
        v -= C != A ? d : 0.0;
    }
    return v;
}

// Threads k < P^2: hess[l][m]; threads P^2 <= k < P^2 + P: grad[k - P^2].
__global__ __launch_bounds__(256) void k_finish(int32_t n_atom, int32_t P, int32_t Pp,
                                                const double *__restrict__ Hsum,
                                                const double *__restrict__ DS,
                                                double *__restrict__ hess, double *__restrict__ grad) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t PP = (int64_t)P * P;
    if (k < PP) {
        if (!hess) return;
        const int l = (int)(k / P), m = (int)(k % P);
        const int A = l / 3, a = l % 3, B = m / 3, b = m % 3;
        const int c = sym_index(a, b);
        const double glm = egrgr(n_atom, DS, A, B, c), gml = egrgr(n_atom, DS, B, A, c);
        hess[k] = 0.5 * (Hsum[(int64_t)l * Pp + m] + Hsum[(int64_t)m * Pp + l]) + 0.5 * (glm + gml);
    } else if (grad && k < PP + P) {
        const int x = (int)(k - PP);
        const int A = x / 3, a = x % 3;
        double gr = 0.0;
        // sum_{i in A} a_i E^{Bgr}_i, formed for B > A; for B < A it is
        // minus the (B, A) sum (a_i e_ij symmetric, d_ij = -d_ji)
#pragma unroll 8
        for (int B = 0; B < n_atom; ++B) {
            const double d = B > A ? DS[((int64_t)A * n_atom + B) * 9 + 6 + a]
                                   : -DS[((int64_t)B * n_atom + A) * 9 + 6 + a];
            gr -= B != A ? d : 0.0;
        }
        grad[x] = Hsum[(int64_t)Pp * Pp + x] + gr;
    }
}

}  // namespace

// Gradient (Section II.A, first form of the grid part): for x = 3 A + a,
//   grad[x] = sum_i w_i (f^rho_i rho^x_i + f^gamma_i gamma^x_i)
//           [+ sum_i w^x_i rho_i (beta + E_i)]
//           - sum_{B > A} sum_{tiles t of A} Gpart[t][B][a]
//           + sum_{B < A} sum_{tiles t of B} Gpart[t][A][a]
// (the tile sums are antisymmetric in the atom pair; the pass forms B > A),
// gamma^x = 2 grad rho . grad rho^x; w^x (optional) with the owner slot from
// Wown.  One workgroup per x; both sums are fixed-order tree reductions,
// added at the end.
__global__ __launch_bounds__(256) void k_gradient(int64_t n, int64_t npad, int32_t n_atom,
                                                  const int32_t *__restrict__ tile_first,
                                                  const int32_t *__restrict__ atom_of,
                                                  const double *__restrict__ F,
                                                  const double *__restrict__ rho_x,
                                                  const double *__restrict__ grad_rho_x,
                                                  const double *__restrict__ w_x,
                                                  const double *__restrict__ Wown,
                                                  const double *__restrict__ Gpart,
                                                  double *__restrict__ grad) {
    __shared__ double sg[256], sr[256];
    const int tid = threadIdx.x, x = blockIdx.x, A = x / 3, a = x % 3;
    const double *rx = rho_x + (int64_t)x * n;
    const double *gx = grad_rho_x + (int64_t)x * n * 3;
    double eg = 0.0;
    for (int64_t i = tid; i < n; i += 256) {
        const double gam = 2.0 * (F[F_GX * npad + i] * gx[3 * i] + F[F_GY * npad + i] * gx[3 * i + 1] +
                                  F[F_GZ * npad + i] * gx[3 * i + 2]);
        eg += F[F_W * npad + i] * (F[F_FR * npad + i] * rx[i] + F[F_FG * npad + i] * gam);
        if (w_x) {
            const double wx = atom_of[i] == A ? Wown[i * 3 + a] : w_x[(int64_t)x * n + i];
            eg += wx * F[F_F0 * npad + i];
        }
    }
    // -sum_{B != A} sum_{t in A} Gpart[t][B]: the pass forms B > A; a B < A
    // term is minus the (B, A) one, i.e. +Gpart[t][A] over the tiles t of B
    const int t0 = tile_first[A], nt = tile_first[A + 1] - t0;
    double gr = 0.0;
    for (int k = tid; k < (n_atom - A - 1) * nt; k += 256) {
        const int B = A + 1 + k / nt, t = t0 + k % nt;
        gr -= Gpart[((int64_t)t * n_atom + B) * 3 + a];
    }
    for (int t = tid; t < t0; t += 256) gr += Gpart[((int64_t)t * n_atom + A) * 3 + a];
    sg[tid] = eg;
    sr[tid] = gr;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            sg[tid] += sg[tid + off];
            sr[tid] += sr[tid + off];
        }
        __syncthreads();
    }
    if (tid == 0) grad[x] = sg[0] + sr[0];
}

hipError_t launch_gradient(vv10_plan *p, const double *rho_x, const double *grad_rho_x,
                           const double *w_x, double *grad) {
    if (w_x) {
        const hipError_t e = launch_weight_own(p, w_x, p->wown);
        if (e != hipSuccess) return e;
    }
    k_gradient<<<(unsigned)(3 * p->n_atom), 256, 0, p->stream>>>(
        p->n, p->npad, p->n_atom, p->d_tile_first, p->atom_of, p->F, rho_x, grad_rho_x, w_x,
        p->wown, p->gw.Gpart, grad);
    return hipGetLastError();
}

hipError_t launch_trial_response(vv10_plan *p, double *f_rho_t, double *f_gamma_t) {
    const Workspace &ws = p->rws;
    dim3 grid((unsigned)((p->n + TRI - 1) / TRI), (unsigned)((ws.P + TRX - 1) / TRX));
    // the contraction partials are FP64 in every mode
    k_trial_resp<double><<<grid, 256, 0, p->stream>>>(
        p->n, p->npad, ws.P, ws.Pp, ws.jsplit, p->P1, p->F, p->Ir, ws.L,
        static_cast<const double *>(ws.Ypart), f_rho_t, f_gamma_t);
    return hipGetLastError();
}

hipError_t launch_assemble(vv10_plan *p, const vv10_nuclear_outputs &out, bool weighted) {
    const Workspace &ws = p->ws;
    const WeightWork &ww = p->ww;
    const int64_t n = p->n;
    double *hess = out.hess, *grad = out.grad;
    {
        const unsigned nb = (unsigned)((n + 3) / 4);
        // the contraction partials are FP64 in every mode
        const WeightIn<double> wt = {static_cast<const double *>(ww.Ypart), ww.Lw, ww.Ze, ww.Rw};
        if (weighted)
            k_resp<double, true><<<nb, 256, 0, p->stream>>>(
                n, p->npad, ws.P, ws.Pp, ws.jsplit, p->atom_of, p->P1, p->F, p->I, ws.L,
                static_cast<const double *>(ws.Ypart), ws.Y, ws.Z, wt, out.resp_rho,
                out.resp_gamma, out.fock_rho, out.fock_gamma);
        else
            k_resp<double, false><<<nb, 256, 0, p->stream>>>(
                n, p->npad, ws.P, ws.Pp, ws.jsplit, p->atom_of, p->P1, p->F, p->I, ws.L,
                static_cast<const double *>(ws.Ypart), ws.Y, ws.Z, wt, out.resp_rho,
                out.resp_gamma, out.fock_rho, out.fock_gamma);
    }
    if (!hess && !grad) return hipGetLastError();
    const int64_t slice = (n + ws.gsplit - 1) / ws.gsplit;
    const unsigned tiles = (unsigned)((ws.Pp + 63) / 64);
    {
        dim3 grid(tiles, tiles, (unsigned)ws.gsplit);
        k_gemm<2><<<grid, 256, 0, p->stream>>>(n, p->npad, slice, ws.Pp, p->F, ws.L, ws.Y, ws.Hpart);
        if (weighted)
            k_gemm<1><<<grid, 256, 0, p->stream>>>(n, p->npad, slice, ws.Pp, p->F, ww.Lw, ww.Rw,
                                                   ww.Hpart);
    }
    {
        const int64_t len = (int64_t)(ws.Pp + 1) * ws.Pp;
        k_hsum<<<(unsigned)((len + 63) / 64), 64 * kHsumWaves, 0, p->stream>>>(
            len, ws.gsplit, ws.Hpart, weighted ? ws.gsplit : 0, ww.Hpart, ws.Hsum);
    }
    const int64_t nds = (int64_t)p->n_atom * p->n_atom * 9;
    k_dsum<<<(unsigned)((nds + 255) / 256), 256, 0, p->stream>>>(p->n_atom, p->d_tile_first,
                                                                 ws.Dpart, ws.DS);
    const int64_t nt = (int64_t)ws.P * ws.P + ws.P;
    k_finish<<<(unsigned)((nt + 255) / 256), 256, 0, p->stream>>>(p->n_atom, ws.P, ws.Pp, ws.Hsum,
                                                                  ws.DS, hess, grad);
    return hipGetLastError();
}

}  // namespace vv10
