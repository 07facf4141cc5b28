// Grid-position intermediates (Section II.B) for outer point i and atom
// B != O(i), as sums over the points j of atom B with d = r_j - r_i:
//   E^{Bgr}_i =  sum_j e_ij d,   e = -2 a_j Phi T
//   U^{Bgr}_i =  sum_j u_ij d,   u =  2 a_j Phi (T h + Q)
//   W^{Bgr}_i =  sum_j v_ij d,   v =  2 a_j Phi (R^2 (T h + Q) - h)
//   D^B_i     = -2 sum_j a_j Phi (2 S d d^T - T I)
// with T = omega_i/g + omega_j/g' + (omega_i+omega_j)/s, h = 1/s + 1/g,
// Q = omega_i/g^2 + (omega_i+omega_j)/s^2,
// S = T^2 + (omega_i/g)^2 + (omega_j/g')^2 + ((omega_i+omega_j)/s)^2.
//
// Outputs, per outer point i and atom B != O(i):
//   Z[i][0][3B+a] = E^{Bgr}_{i,a} + c_i U^{Bgr}_{i,a},  Z[i][1][3B+a] = W^{Bgr}_{i,a}
// (the two channels that multiply p and q in E_{G,gr}), and per tile t of
// outer points (all in one atom A) the sums
//   Dpart[t][B][0..5] = sum_{i in t} a_i D^B_i   (xx, yy, zz, xy, xz, yz)
//   Dpart[t][B][6..8] = sum_{i in t} a_i E^{Bgr}_i
// from which the assembly builds E_{gr,gr} and the grid part of the
// gradient.  The own-atom slot B = O(i) follows from translational
// invariance and is filled by the assembly.
//
// One wave per (tile of 64 outer points, group of atoms B); tiles never
// straddle atoms, so the D sums are plain wave reductions in a fixed order.
#include "dev_common.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

constexpr int TG = kGridTile;

__global__ __launch_bounds__(64) void k_grid_f64(
    int32_t n_atom, int32_t Pp, int32_t bgroups, const int64_t *__restrict__ seg,
    const int32_t *__restrict__ tile_i0, const int32_t *__restrict__ tile_n,
    const int32_t *__restrict__ tile_atom, const double4 *__restrict__ P0,
    const double4 *__restrict__ P1, double *__restrict__ Z, double *__restrict__ Dpart) {
    __shared__ double4 sA[TG], sB[TG];
    const int t = blockIdx.x, grp = blockIdx.y, lane = threadIdx.x;
    const int A = tile_atom[t];
    const int nt = tile_n[t];
    const bool live = lane < nt;
    const int64_t i = (int64_t)tile_i0[t] + (live ? lane : 0);
    const double4 a0 = P0[i], a1 = P1[i];
    const double ai = live ? a1.y : 0.0, ci = a1.z, oi = a0.w;
    for (int B = grp; B < n_atom; B += bgroups) {
        if (B == A) continue;
        const int64_t jb = seg[B], je = seg[B + 1];
        double ex = 0, ey = 0, ez = 0, ux = 0, uy = 0, uz = 0, vx = 0, vy = 0, vz = 0;
        double dxx = 0, dyy = 0, dzz = 0, dxy = 0, dxz = 0, dyz = 0;
        for (int64_t j0 = jb; j0 < je; j0 += TG) {
            __syncthreads();
            const int64_t j = j0 + lane;
            sA[lane] = P0[j < je ? j : jb];
            sB[lane] = P1[j < je ? j : jb];
            __syncthreads();
            const int cnt = (int)min((int64_t)TG, je - j0);
            for (int jj = 0; jj < cnt; ++jj) {
                const double4 b0 = sA[jj], b1 = sB[jj];
                const double dx = b0.x - a0.x, dy = b0.y - a0.y, dz = b0.z - a0.z;
                const double R2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
                const double g = __builtin_fma(oi, R2, a1.x);
                const double gp = __builtin_fma(b0.w, R2, b1.x);
                const double s = g + gp, tt = g * gp;
                const double r = rcp64(tt * s);
                const double pa = -1.5 * b1.y * r;       // a_j Phi_ij
                const double ig = gp * s * r, igp = g * s * r, is = tt * r;
                const double Ti = oi * ig, Tj = b0.w * igp, Ts = (oi + b0.w) * is;
                const double T = Ti + Tj + Ts;
                const double h = ig + is;
                const double TQ = __builtin_fma(T, h, __builtin_fma(Ti, ig, Ts * is));
                const double e = -2.0 * pa * T;
                const double u = 2.0 * pa * TQ;
                const double v = 2.0 * pa * __builtin_fma(R2, TQ, -h);
                const double S = __builtin_fma(T, T, __builtin_fma(Ti, Ti, __builtin_fma(Tj, Tj, Ts * Ts)));
                const double dd = -4.0 * pa * S;       // coefficient of d d^T
                const double di = -e;                  // coefficient of I (= 2 a_j Phi T)
                ex = __builtin_fma(e, dx, ex); ey = __builtin_fma(e, dy, ey); ez = __builtin_fma(e, dz, ez);
                ux = __builtin_fma(u, dx, ux); uy = __builtin_fma(u, dy, uy); uz = __builtin_fma(u, dz, uz);
                vx = __builtin_fma(v, dx, vx); vy = __builtin_fma(v, dy, vy); vz = __builtin_fma(v, dz, vz);
                const double ddx = dd * dx, ddy = dd * dy;
                dxx += __builtin_fma(ddx, dx, di);
                dyy += __builtin_fma(ddy, dy, di);
                dzz += __builtin_fma(dd * dz, dz, di);
                dxy = __builtin_fma(ddx, dy, dxy);
                dxz = __builtin_fma(ddx, dz, dxz);
                dyz = __builtin_fma(ddy, dz, dyz);
            }
        }
        if (live) {
            double *z0 = Z + (i * 2 + 0) * Pp + 3 * B;
            double *z1 = Z + (i * 2 + 1) * Pp + 3 * B;
            z0[0] = __builtin_fma(ci, ux, ex);
            z0[1] = __builtin_fma(ci, uy, ey);
            z0[2] = __builtin_fma(ci, uz, ez);
            z1[0] = vx;
            z1[1] = vy;
            z1[2] = vz;
        }
        const double red[9] = {ai * dxx, ai * dyy, ai * dzz, ai * dxy, ai * dxz, ai * dyz,
                               ai * ex, ai * ey, ai * ez};
        double *dp = Dpart + ((int64_t)t * n_atom + B) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double tot = wave_sum(red[k]);
            if (lane == 0) dp[k] = tot;
        }
    }
}

}  // namespace

hipError_t launch_grid_terms(vv10_plan *p) {
    const Workspace &ws = p->ws;
    if (p->prec != VV10_FP64) return hipErrorInvalidValue;
    dim3 grid((unsigned)p->ntiles, (unsigned)ws.bgroups);
    k_grid_f64<<<grid, TG, 0, p->stream>>>(p->n_atom, ws.Pp, ws.bgroups, p->d_seg, p->d_tile_i0,
                                          p->d_tile_n, p->d_tile_atom, p->P0, p->P1, ws.Z,
                                          ws.Dpart);
    return hipGetLastError();
}

}  // namespace vv10
