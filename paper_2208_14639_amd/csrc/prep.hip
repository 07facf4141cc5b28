// Per-point preparation (Section II.A of the paper: omega, kappa and the
// first and second partial derivatives that the potential and the
// second-derivative matrices need) and perturbation packing (Section II.B:
// rho^x, gamma^x of the 3 N_atom nuclear perturbations).
//
// Both kernels are O(N) or O(N P) and bound by HBM bandwidth; everything
// here is FP64.
#include "dev_common.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Fill an int32 array with a value (used instead of a memset so that the
// launch sequence contains kernels only).
__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// Partial sums of the coordinates for the centroid shift (fixed order).
__global__ __launch_bounds__(256) void k_coord_partials(int64_t n, const double *coords,
                                                        double *part) {
    __shared__ double s[3][256];
    double a[3] = {0, 0, 0};
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        for (int k = 0; k < 3; ++k) a[k] += coords[3 * i + k];
    for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void k_coord_centroid(int nblk, int64_t n, double *part) {
    if (threadIdx.x < 3) {
        double t = 0.0;
#pragma unroll 16   // loads in flight together; the sum stays in block order
        for (int b = 0; b < nblk; ++b) t += part[3 * b + threadIdx.x];
        part[3 * nblk + threadIdx.x] = t / (double)n;
    }
}

// One thread per padded point.  Pad rows get benign values (omega = kappa = 1,
// zero weight) so that they contribute exact zeros to every sum.
__global__ __launch_bounds__(256) void k_prep(
    int64_t n, int64_t npad, int32_t n_atom, double b, double C,
    const double *__restrict__ coords, const double *__restrict__ w,
    const int32_t *__restrict__ atom_of, const double *__restrict__ rho,
    const double *__restrict__ grad, const double *__restrict__ centroid,
    double4 *__restrict__ P0, double4 *__restrict__ P1, float4 *__restrict__ P0f,
    float4 *__restrict__ P1f, double *__restrict__ F, int32_t *__restrict__ ao_out,
    int32_t *__restrict__ flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i >= n) {
        P0[i] = make_double4(0.0, 0.0, 0.0, 1.0);
        P1[i] = make_double4(1.0, 0.0, 0.0, 0.0);
        P0f[i] = make_float4(0.f, 0.f, 0.f, 1.f);
        P1f[i] = make_float4(1.f, 0.f, 0.f, 0.f);
        for (int f = 0; f < NF; ++f) F[f * npad + i] = 0.0;
        ao_out[i] = n_atom;
        return;
    }
    const double r = rho[i], wi = w[i];
    const double gx = grad[3 * i], gy = grad[3 * i + 1], gz = grad[3 * i + 2];
    const double x = coords[3 * i] - centroid[0];
    const double y = coords[3 * i + 1] - centroid[1];
    const double z = coords[3 * i + 2] - centroid[2];
    const int32_t A = atom_of[i];
    int32_t bad = 0;
    if (!(r > 0.0) || !isfinite(r) || !isfinite(wi) || !isfinite(gx) || !isfinite(gy) ||
        !isfinite(gz) || !isfinite(x) || !isfinite(y) || !isfinite(z))
        bad |= 1;
    if (A < 0 || A >= n_atom) bad |= 4;
    else if (i > 0 && atom_of[i - 1] > A) bad |= 2;
    if (bad) {
        atomicOr(flag, bad);
        return;
    }
    // first point of atom A records the segment start
    if (i == 0 || atom_of[i - 1] != A) flag[1 + A] = (int32_t)i;

    const double gam = gx * gx + gy * gy + gz * gz;
    const double ir = 1.0 / r;
    const double q = gam * ir * ir;                 // gamma / rho^2
    const double S = C * q * q + (4.0 * kPi / 3.0) * r;   // omega^2
    const double om = sqrt(S);
    const double ka = b * 1.5 * kPi * pow(r / (9.0 * kPi), 1.0 / 6.0);
    // derivatives of S = omega^2
    const double Sr = (4.0 * kPi / 3.0) - 4.0 * C * q * q * ir;
    const double Sg = 2.0 * C * q * ir * ir;
    const double Srr = 20.0 * C * q * q * ir * ir;
    const double Srg = -8.0 * C * q * ir * ir * ir;
    const double Sgg = 2.0 * C * ir * ir * ir * ir;
    const double iom = 1.0 / om;
    const double omr = 0.5 * Sr * iom, omg = 0.5 * Sg * iom;
    const double omrr = (0.5 * Srr - omr * omr) * iom;
    const double omrg = (0.5 * Srg - omr * omg) * iom;
    const double omgg = (0.5 * Sgg - omg * omg) * iom;
    const double kar = ka * ir / 6.0;
    const double karr = -5.0 * ka * ir * ir / 36.0;
    const double a = wi * r, c = r * kar;

    P0[i] = make_double4(x, y, z, om);
    P1[i] = make_double4(ka, a, c, 0.0);
    P0f[i] = make_float4((float)x, (float)y, (float)z, (float)om);
    P1f[i] = make_float4((float)ka, (float)a, (float)c, 0.f);
    F[F_W * npad + i] = wi;
    F[F_RHO * npad + i] = r;
    F[F_GX * npad + i] = gx;
    F[F_GY * npad + i] = gy;
    F[F_GZ * npad + i] = gz;
    F[F_OMR * npad + i] = omr;
    F[F_OMG * npad + i] = omg;
    F[F_KAR * npad + i] = kar;
    F[F_OMRR * npad + i] = omrr;
    F[F_OMRG * npad + i] = omrg;
    F[F_OMGG * npad + i] = omgg;
    F[F_KARR * npad + i] = karr;
    F[F_FR * npad + i] = 0.0;
    F[F_FG * npad + i] = 0.0;
    F[F_F0 * npad + i] = 0.0;
    ao_out[i] = A;
}

// Perturbation packing: for every point i and perturbation x,
//   gamma^x = 2 grad rho . grad rho^x,
//   p = w rho^x,  q = w rho (omega_r rho^x + omega_g gamma^x)   (the two channels)
//   L[i][0][x] = rho^x, L[i][1][x] = gamma^x  (FP64, for the assembly).
// The channels are stored as the contraction of the plan's mode reads them:
//   FP64 / FP32: X[i][c][x];
//   BF16X3: hi = bf16(v), lo = bf16(v - hi), each as [i/16][x][2 (i mod 16) + c].
// The mixed modes store -3/2 p and -3/2 q: their contraction forms the pair
// kernel divided by the -3/2 factor of Phi.
// A 32 x 32 (point x perturbation) tile is staged through LDS so that the
// [P][N] reads are coalesced.  With bmax (screening), also
//   bmax[i/16][x] = max over the 16-point block of max(|p|, |q|).
constexpr int TT = 32;
template <int MODE>
__global__ __launch_bounds__(256) void k_pert_prep(
    int64_t n, int64_t npad, int32_t P, int32_t Pp, const double *__restrict__ rho_x,
    const double *__restrict__ grad_rho_x, const double *__restrict__ F,
    void *__restrict__ Xv, double *__restrict__ L, float *__restrict__ bmax) {
    __shared__ double sr[TT][TT + 1];
    __shared__ double sg[TT][TT + 1];
    __shared__ float sm[2][8][TT];
    float mblk[2] = {0.f, 0.f};
    const int64_t i0 = (int64_t)blockIdx.x * TT;
    const int x0 = blockIdx.y * TT;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;   // 32 x 8
    // load: thread (tx, ty) reads point i0 + tx of perturbations x0 + ty + 8k
    for (int k = 0; k < TT; k += 8) {
        const int x = x0 + ty + k;
        const int64_t i = i0 + tx;
        double rx = 0.0, gxv = 0.0;
        if (x < P && i < n) {
            rx = rho_x[(int64_t)x * n + i];
            const double *gp = grad_rho_x + ((int64_t)x * n + i) * 3;
            gxv = 2.0 * (F[F_GX * npad + i] * gp[0] + F[F_GY * npad + i] * gp[1] +
                         F[F_GZ * npad + i] * gp[2]);
        }
        sr[ty + k][tx] = rx;
        sg[ty + k][tx] = gxv;
    }
    __syncthreads();
    // store: thread (tx, ty) writes perturbation x0 + tx of points i0 + ty + 8k
    for (int k = 0; k < TT; k += 8) {
        const int64_t i = i0 + ty + k;
        const int x = x0 + tx;
        if (i >= npad || x >= Pp) continue;
        const double rx = sr[tx][ty + k], gxv = sg[tx][ty + k];
        const double wi = F[F_W * npad + i], r = F[F_RHO * npad + i];
        const double sc = MODE == VV10_FP64 ? 1.0 : -1.5;
        const double p = sc * wi * rx;
        const double qv = sc * wi * r * (F[F_OMR * npad + i] * rx + F[F_OMG * npad + i] * gxv);
        mblk[k / 16] = fmaxf(mblk[k / 16], (float)fmax(fabs(p), fabs(qv)));
        if (MODE == VV10_FP64) {
            double *X = static_cast<double *>(Xv);
            X[(i * 2 + 0) * Pp + x] = p;
            X[(i * 2 + 1) * Pp + x] = qv;
        } else if (MODE == VV10_MIXED_FP32) {
            float *X = static_cast<float *>(Xv);
            X[(i * 2 + 0) * Pp + x] = (float)p;
            X[(i * 2 + 1) * Pp + x] = (float)qv;
        } else {
            sr[tx][ty + k] = p;     // this thread's element only: split below
            sg[tx][ty + k] = qv;
        }
        L[(i * 2 + 0) * Pp + x] = rx;
        L[(i * 2 + 1) * Pp + x] = gxv;
    }
    if constexpr (MODE == VV10_MIXED_BF16X3) {
        // thread -> (16-point block hb, column xo, quarter qq): the four points
        // i0 + 16 hb + 4 qq + e; their (p, q) hi and lo words are 16 B each,
        // and four adjacent threads write one column's 64 B run of a block.
        __syncthreads();
        const int qq = threadIdx.x & 3, xo = (threadIdx.x >> 2) & (TT - 1), hb = threadIdx.x >> 7;
        const int x = x0 + xo;
        const int io = 16 * hb + 4 * qq;
        if (x < Pp && i0 + io < npad) {
            uint32_t hw[4], lw[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double pv = sr[xo][io + e], qv = sg[xo][io + e];
                const __bf16 ph = (__bf16)(float)pv, qh = (__bf16)(float)qv;
                const __bf16 pl = (__bf16)(float)(pv - (double)(float)ph);
                const __bf16 ql = (__bf16)(float)(qv - (double)(float)qh);
                hw[e] = (uint32_t)__builtin_bit_cast(uint16_t, ph) |
                        ((uint32_t)__builtin_bit_cast(uint16_t, qh) << 16);
                lw[e] = (uint32_t)__builtin_bit_cast(uint16_t, pl) |
                        ((uint32_t)__builtin_bit_cast(uint16_t, ql) << 16);
            }
            // element offset ((i / 16) Pp + x) 32 + 2 (i mod 16) of the first point, in 16 B units
            const int64_t o = ((((i0 + io) / 16) * Pp + x) * 32 + 2 * ((i0 + io) % 16)) / 8;
            uint4 *Xh = static_cast<uint4 *>(Xv);
            uint4 *Xl = Xh + npad * 2 * Pp / 8;
            Xh[o] = (uint4){hw[0], hw[1], hw[2], hw[3]};
            Xl[o] = (uint4){lw[0], lw[1], lw[2], lw[3]};
        }
    }
    if (bmax) {   // uniform over the workgroup
        sm[0][ty][tx] = mblk[0];
        sm[1][ty][tx] = mblk[1];
        __syncthreads();
        const int x = x0 + tx;
        if (ty < 2 && x < Pp) {
            float m = 0.f;
#pragma unroll
            for (int t = 0; t < 8; ++t) m = fmaxf(m, sm[ty][t][tx]);
            bmax[(i0 / 16 + ty) * Pp + x] = m;
        }
    }
}

// Screening mask of the contraction (blocks of 16 points x 16 columns):
// colmax[x] = max over blocks of bmax[.][x]; a block is active when one of
// its columns has bmax > tau colmax.  mask[b][grp] holds one bit per column
// block of the contraction's column group (one scalar load per j block in
// the kernel).  count receives the number of active blocks (zeroed by
// k_screen_zero first).
__global__ void k_screen_zero(int32_t *count) { *count = 0; }

__global__ __launch_bounds__(256) void k_colmax(int64_t nblk, int32_t Pp, const float *__restrict__ bmax,
                                                float *__restrict__ colmax) {
    __shared__ float s[256];
    const int x = blockIdx.x;
    float m = 0.f;
    for (int64_t b = threadIdx.x; b < nblk; b += 256) m = fmaxf(m, bmax[b * Pp + x]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) colmax[x] = s[0];
}

__global__ __launch_bounds__(256) void k_mask(int64_t nblk, int32_t Pp, int32_t ncb, float tau,
                                              const float *__restrict__ bmax,
                                              const float *__restrict__ colmax,
                                              uint32_t *__restrict__ mask, int32_t *__restrict__ count) {
    const int ngroups = Pp / (16 * ncb);
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= nblk * ngroups) return;
    const int64_t b = k / ngroups;
    const int grp = (int)(k - b * ngroups);
    uint32_t bits = 0;
    for (int cb = 0; cb < ncb; ++cb) {
        bool active = false;
        for (int c = 0; c < 16; ++c) {
            const int x = (grp * ncb + cb) * 16 + c;
            active |= bmax[b * Pp + x] > tau * colmax[x];
        }
        if (active) bits |= 1u << cb;
    }
    mask[k] = bits;
    if (bits) atomicAdd(count, __popc(bits));
}

}  // namespace

hipError_t launch_prepare(vv10_plan *p, const double *coords, const double *w,
                          const int32_t *atom_of, const double *rho,
                          const double *grad_rho) {
    const int nb_part = 64;
    k_fill_i32<<<(p->n_atom + 2 + 255) / 256, 256, 0, p->stream>>>(p->flag, p->n_atom + 2, -1);
    k_fill_i32<<<1, 1, 0, p->stream>>>(p->flag, 1, 0);
    k_coord_partials<<<nb_part, 256, 0, p->stream>>>(p->n, coords, p->red);
    k_coord_centroid<<<1, 64, 0, p->stream>>>(nb_part, p->n, p->red);
    k_prep<<<(unsigned)(p->npad / 256), 256, 0, p->stream>>>(
        p->n, p->npad, p->n_atom, p->prm.b, p->prm.C, coords, w, atom_of, rho, grad_rho,
        p->red + 3 * nb_part, p->P0, p->P1, p->P0f, p->P1f, p->F, p->atom_of, p->flag);
    return hipGetLastError();
}

hipError_t launch_pert_prep(vv10_plan *p, const Workspace &ws, const double *rho_x,
                            const double *grad_rho_x, bool screen) {
    dim3 grid((unsigned)((p->npad + TT - 1) / TT), (unsigned)((ws.Pp + TT - 1) / TT));
    float *bmax = screen ? ws.bmax : nullptr;
    if (p->prec == VV10_FP64)
        k_pert_prep<VV10_FP64><<<grid, 256, 0, p->stream>>>(p->n, p->npad, ws.P, ws.Pp, rho_x,
                                                            grad_rho_x, p->F, ws.X, ws.L, bmax);
    else if (p->prec == VV10_MIXED_FP32)
        k_pert_prep<VV10_MIXED_FP32><<<grid, 256, 0, p->stream>>>(p->n, p->npad, ws.P, ws.Pp, rho_x,
                                                                  grad_rho_x, p->F, ws.X, ws.L, bmax);
    else
        k_pert_prep<VV10_MIXED_BF16X3><<<grid, 256, 0, p->stream>>>(p->n, p->npad, ws.P, ws.Pp, rho_x,
                                                                    grad_rho_x, p->F, ws.X, ws.L, bmax);
    if (!screen) return hipGetLastError();
    const int64_t nblk = p->npad / 16;
    k_colmax<<<(unsigned)ws.Pp, 256, 0, p->stream>>>(nblk, ws.Pp, ws.bmax, ws.colmax);
    k_screen_zero<<<1, 1, 0, p->stream>>>(ws.screen_count);
    const int64_t tot = nblk * ws.ngroups;
    k_mask<<<(unsigned)((tot + 255) / 256), 256, 0, p->stream>>>(nblk, ws.Pp, ws.ncb,
                                                                 (float)p->screen_tau, ws.bmax,
                                                                 ws.colmax, ws.mask, ws.screen_count);
    return hipGetLastError();
}

}  // namespace vv10
