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
// stored: each 16 x 4 block of (i, j) pairs is formed once in registers, one
// pair per lane in the MFMA A-operand layout, and fed to four
// v_mfma_f64_16x16x4 per 16 perturbation columns (K_pp X_p, K_pq X_q into
// Y_p; K_qp X_p, K_qq X_q into Y_q).  X chunks are staged in LDS and shared
// by the four waves of a workgroup; every wave owns 16 outer points and all
// columns of its column group, with FP64 accumulators in registers.
#include "dev_common.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

constexpr int kJC = 32;   // j points per LDS stage

template <int NCB>
__global__ __launch_bounds__(256, 2) void k_contract_f64(
    int64_t npad, int64_t jlen, int32_t Pp, const double4 *__restrict__ P0,
    const double4 *__restrict__ P1, const double *__restrict__ X, double *__restrict__ Yout) {
    constexpr int NC = NCB * 16;
    __shared__ double4 sA[kJC], sB[kJC];
    __shared__ __attribute__((aligned(16))) double sX[kJC * 2 * NC];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int64_t ibase = (int64_t)blockIdx.x * 64 + wave * 16;
    const int col0 = blockIdx.y * NC;
    const int64_t jbeg = (int64_t)blockIdx.z * jlen;
    const int64_t jend = min(npad, jbeg + jlen);
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
#pragma unroll 2
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
            const double kpp = phi + ci * Pg + cj * __builtin_fma(ci, Pgg, Pgp);
            const double kpq = R2 * __builtin_fma(ci, Pgg, Pgp);
            const double kqp = R2 * __builtin_fma(cj, Pgg, Pg);
            const double kqq = R2 * R2 * Pgg;
            const double *xr = sX + (jl * 2) * NC + m;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const double xp = xr[cb * 16];
                accp[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(kpp, xp, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(kqp, xp, accq[cb], 0, 0, 0);
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const double xq = xr[NC + cb * 16];
                accp[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(kpq, xq, accp[cb], 0, 0, 0);
                accq[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(kqq, xq, accq[cb], 0, 0, 0);
            }
        }
    }
    // D layout of v_mfma_f64_16x16x4 (measured on gfx950): item r of lane l
    // holds row 4 r + l/16, column l%16
    double *Yb = Yout + (int64_t)blockIdx.z * npad * 2 * Pp;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = ibase + 4 * r + kq;
            Yb[(row * 2 + 0) * Pp + col0 + cb * 16 + m] = accp[cb][r];
            Yb[(row * 2 + 1) * Pp + col0 + cb * 16 + m] = accq[cb][r];
        }
}

template <int NCB>
hipError_t run_f64(vv10_plan *p) {
    const Workspace &ws = p->ws;
    const int64_t jlen = ((p->npad / ws.jsplit + kJC - 1) / kJC) * kJC;
    dim3 grid((unsigned)(p->npad / 64), (unsigned)ws.ngroups, (unsigned)ws.jsplit);
    k_contract_f64<NCB><<<grid, 256, 0, p->stream>>>(p->npad, jlen, ws.Pp, p->P0, p->P1, ws.X, ws.Y);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_contract(vv10_plan *p) {
    const Workspace &ws = p->ws;
    hipError_t e = hipErrorInvalidValue;
    if (p->prec == VV10_FP64) {
        switch (ws.ncb) {
            case 1: e = run_f64<1>(p); break;
            case 2: e = run_f64<2>(p); break;
            case 3: e = run_f64<3>(p); break;
            case 4: e = run_f64<4>(p); break;
            case 5: e = run_f64<5>(p); break;
            case 6: e = run_f64<6>(p); break;
            case 7: e = run_f64<7>(p); break;
            case 8: e = run_f64<8>(p); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;   // mixed contraction: see contract_mixed.hip
    }
    return e;
}

}  // namespace vv10
