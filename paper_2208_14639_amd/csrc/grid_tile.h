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
// (the two channels that multiply p and q in E_{G,gr}), optionally
//   Ze[i][3B+a] = E^{Bgr}_{i,a}   (the channel of E_{w,gr}), and per tile t of
// outer points (all in one atom A) the sums
//   Dpart[t][B][0..5] = sum_{i in t} a_i D^B_i   (xx, yy, zz, xy, xz, yz)
//   Dpart[t][B][6..8] = sum_{i in t} a_i E^{Bgr}_i
// for B > A only (zero for B < A), from which the assembly builds E_{gr,gr}
// and the grid part of the gradient: summed over the tiles of A, both are
// (anti)symmetric in the atom pair (a_i a_j Phi (2 S d d^T - T I) is
// symmetric in i, j; a_i e_ij is symmetric and d_ij = -d_ji), so the
// (B, A) sums give the B < A ones.  For B < A the pass therefore forms
// E^{Bgr} + c_i U^{Bgr} as one vector (and E^{Bgr} only for Ze).  The
// own-atom slot B = O(i) follows from translational invariance and is
// filled by the assembly.
//
// The same pass also accumulates the pair integrals E, U, W, A, B, C of the
// Hessian call (over every j, the outer point's own atom included), so the
// pair geometry and its reciprocal are evaluated once per pair.  The self
// pair j = i is left out of the loops and added in FP64 (from the FP64
// point data Pd) by the workgroup whose atom group holds the own atom.
//
// One wave per (tile of 64 outer points, group of atoms B); tiles never
// straddle atoms, so the D sums are plain wave reductions in a fixed order.
// FP64 mode evaluates and accumulates in FP64; the mixed modes evaluate each
// pair in FP32, accumulate one 64-point chunk in FP32 and add the chunk sums
// into FP64 accumulators.
#pragma once

#include "dev_common.h"
#include "vv10_internal.h"

namespace vv10 {

namespace {

constexpr int TG = kGridTile;

// Shared geometry of one (i, j) pair: with r = 1/(g g' s), p = a_j r
// (a_j Phi = -3/2 p), 1/g = g' s r, 1/g' = g s r, 1/s = g g' r.
template <typename T>
struct PairGeo {
    T R2, p, ig, igp, is, h;
};

template <typename T, typename T4>
__device__ __forceinline__ PairGeo<T> pair_geo(const T4 a0, const T4 a1, const T4 b0, const T4 b1) {
    PairGeo<T> q;
    const T dx = b0.x - a0.x, dy = b0.y - a0.y, dz = b0.z - a0.z;
    q.R2 = dx * dx + dy * dy + dz * dz;
    const T g = a0.w * q.R2 + a1.x;
    const T gp = b0.w * q.R2 + b1.x;
    const T s = g + gp;
    const T tt = g * gp;
    T r;
    if constexpr (sizeof(T) == 8) r = rcp64(tt * s); else r = rcp32(tt * s);
    q.p = b1.y * r;
    const T sr = s * r;
    q.ig = gp * sr;
    q.igp = g * sr;
    q.is = tt * r;
    q.h = q.ig + q.is;
    return q;
}

// Pair-integral sums, scaled: c[0] += p, c[1] += p h, c[2] += p h R^2,
// c[3..5] += p m (R^2)^{0,1,2} with m = 1/s^2 + 1/(s g) + 1/g^2 = h^2 - (1/s)(1/g).
// Then E = -3/2 c0, U = 3/2 c1, W = 3/2 c2, (A, B, C) = -3 (c3, c4, c5).
template <typename T>
__device__ __forceinline__ void add_pair_integrals(const PairGeo<T> &q, T *c) {
    const T ph = q.p * q.h;
    const T pm = q.p * (q.h * q.h - q.is * q.ig);
    const T pmR2 = pm * q.R2;
    c[0] += q.p;
    c[1] += ph;
    c[2] += ph * q.R2;
    c[3] += pm;
    c[4] += pmR2;
    c[5] += pmR2 * q.R2;
}

// One LDS chunk of points j of atom B != A: pair integrals into pc (when
// INTS), grid sums into c (see k_grid); the D sums only when DSUM.  The
// first six sums (SUMS): kEU, c[0..2] = sum e d and c[3..5] = sum u d
// (B > A, where the tile sums need E^{Bgr} on its own); kZ, c[0..2] =
// sum (e - c_i u) d, the combination the Z channel needs (B < A); kZE, kZ
// and c[3..5] = sum e d (B < A with Ze).
enum { kEU = 0, kZ = 1, kZE = 2 };
template <bool DSUM, bool INTS, int SUMS, typename T, typename T4>
__device__ __forceinline__ void grid_chunk(const T4 a0, const T4 a1, const T4 *sA, const T4 *sB,
                                           int cnt, T *pc, T *c) {
    const T oi = a0.w, ci = a1.z;
#pragma unroll 4
    for (int jj = 0; jj < cnt; ++jj) {
        const T4 b0 = sA[jj];
        const PairGeo<T> q = pair_geo<T>(a0, a1, b0, sB[jj]);
        if (INTS) add_pair_integrals(q, pc);
        const T dx = b0.x - a0.x, dy = b0.y - a0.y, dz = b0.z - a0.z;
        const T Ti = oi * q.ig, Tj = b0.w * q.igp, Ts = (oi + b0.w) * q.is;
        const T T_ = Ti + Tj + Ts;
        const T TQ = T_ * q.h + Ti * q.ig + Ts * q.is;
        const T e = q.p * T_;
        const T v = q.p * (q.R2 * TQ - q.h);
        if (SUMS == kEU) {
            const T u = q.p * TQ;
            c[0] += e * dx; c[1] += e * dy; c[2] += e * dz;
            c[3] += u * dx; c[4] += u * dy; c[5] += u * dz;
        } else {
            const T z = q.p * (T_ - ci * TQ);
            c[0] += z * dx; c[1] += z * dy; c[2] += z * dz;
            if (SUMS == kZE) {
                c[3] += e * dx; c[4] += e * dy; c[5] += e * dz;
            }
        }
        c[6] += v * dx; c[7] += v * dy; c[8] += v * dz;
        if (DSUM) {
            const T S = T_ * T_ + Ti * Ti + Tj * Tj + Ts * Ts;
            const T ps = q.p * S;
            const T psx = ps * dx, psy = ps * dy, psz = ps * dz;
            c[9] += psx * dx;
            c[10] += psy * dy;
            c[11] += psz * dz;
            c[12] += psx * dy;
            c[13] += psx * dz;
            c[14] += psy * dz;
            c[15] += e;
        }
    }
}


// LDS hand-off between the lanes of one wave (the chunk buffers are private
// to the wave): the writes complete before any lane reads, and no lane
// overwrites a chunk before every lane has read it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One (tile t, atom group grp) unit of the grid pass, run by one wave (lane
// = its lane) on its own LDS chunk buffers sA, sB of TG points each.
// Fused with the pair integrals of the Hessian call (INTS): the group of
// atoms B of a workgroup also covers the outer point's own atom for
// E, U, W, A, B, C, whose per-group partial sums go to Ipart[group][6][npad].
// Without INTS (the plan already holds the six integrals) the own atom is
// skipped and only the grid sums are formed.
//
// Per pair (B != A), with Ti = omega_i/g, Tj = omega_j/g', Ts = (omega_i + omega_j)/s,
// T = Ti + Tj + Ts, TQ = T h + Ti/g + Ts/s, S = T^2 + Ti^2 + Tj^2 + Ts^2, the
// scaled sums
//   g[0..2] = sum p T d,  g[3..5] = sum p TQ d,  g[6..8] = sum p (R^2 TQ - h) d,
//   g[9..14] = sum p S d d^T (xx, yy, zz, xy, xz, yz),  g[15] = sum p T
// give e d, u d, v d and D through e = 3 p T, u = -3 p TQ, v = -3 p (R^2 TQ - h),
// D = 6 sum p S d d^T - 3 (sum p T) I.  The D sums and the tile sums of
// a_i E^{Bgr}_i are formed for B > A only (see above); for B < A
// g[0..2] = sum p (T - c_i TQ) d gives E^{Bgr} + c_i U^{Bgr} = 3 g[0..2],
// and g[3..5] = sum p T d only for Ze.
template <typename T, typename T4, bool INTS, bool ZE>
__device__ __forceinline__ void grid_unit(
    int32_t n_atom, int32_t Pp, int32_t bgroups, int64_t npad, const int64_t *__restrict__ seg,
    const int32_t *__restrict__ tile_i0, const int32_t *__restrict__ tile_n,
    const int32_t *__restrict__ tile_atom, const T4 *__restrict__ P0,
    const T4 *__restrict__ P1, const double4 *__restrict__ Pd, double *__restrict__ Z,
    double *__restrict__ Ze, double *__restrict__ Dpart, double *__restrict__ Ipart, int t,
    int grp, int lane, T4 *__restrict__ sA, T4 *__restrict__ sB) {
    const int A = tile_atom[t];
    const int nt = tile_n[t];
    const bool live = lane < nt;
    const int64_t i = (int64_t)tile_i0[t] + (live ? lane : 0);
    const T4 a0 = P0[i], a1 = P1[i];
    const double ai = live ? (double)a1.y : 0.0, ci = (double)a1.z;
    double pint[6] = {};
    for (int B = grp; B < n_atom; B += bgroups) {
        if (!INTS && B == A) continue;
        const int64_t jb = seg[B], je = seg[B + 1];
        const bool dsum = B > A;
        double acc[16] = {};
        for (int64_t j0 = jb; j0 < je; j0 += TG) {
            wave_lds_sync();
            const int64_t j = j0 + lane;
            sA[lane] = P0[j < je ? j : jb];
            sB[lane] = P1[j < je ? j : jb];
            wave_lds_sync();
            const int cnt = (int)min((int64_t)TG, je - j0);
            T pc[6] = {};
            if (B == A) {
                // own atom: pair integrals only (grid-position terms vanish);
                // the chunk of the tile's own points leaves out the self pair
                if (j0 == tile_i0[t]) {
#pragma unroll 4
                    for (int jj = 0; jj < cnt; ++jj) {
                        PairGeo<T> q = pair_geo<T>(a0, a1, sA[jj], sB[jj]);
                        q.p = jj == lane ? T(0) : q.p;
                        add_pair_integrals(q, pc);
                    }
                } else {
#pragma unroll 4
                    for (int jj = 0; jj < cnt; ++jj) {
                        const PairGeo<T> q = pair_geo<T>(a0, a1, sA[jj], sB[jj]);
                        add_pair_integrals(q, pc);
                    }
                }
            } else {
                T c[16] = {};
                if (dsum) grid_chunk<true, INTS, kEU, T, T4>(a0, a1, sA, sB, cnt, pc, c);
                else grid_chunk<false, INTS, ZE ? kZE : kZ, T, T4>(a0, a1, sA, sB, cnt, pc, c);
#pragma unroll
                for (int k = 0; k < 16; ++k) acc[k] += (double)c[k];
            }
            if (INTS)
#pragma unroll
                for (int k = 0; k < 6; ++k) pint[k] += (double)pc[k];
        }
        if (B == A) continue;
        // B > A: E^{Bgr} = 3 acc[0..2], U^{Bgr} = -3 acc[3..5]; B < A:
        // E^{Bgr} + c_i U^{Bgr} = 3 acc[0..2] (and E^{Bgr} = 3 acc[3..5] with
        // Ze); W^{Bgr} = -3 acc[6..8]
        if (live) {
            double *z0 = Z + (i * 2 + 0) * Pp + 3 * B;
            double *z1 = Z + (i * 2 + 1) * Pp + 3 * B;
            z0[0] = 3.0 * (dsum ? acc[0] - ci * acc[3] : acc[0]);
            z0[1] = 3.0 * (dsum ? acc[1] - ci * acc[4] : acc[1]);
            z0[2] = 3.0 * (dsum ? acc[2] - ci * acc[5] : acc[2]);
            z1[0] = -3.0 * acc[6];
            z1[1] = -3.0 * acc[7];
            z1[2] = -3.0 * acc[8];
            if (ZE) {
                double *ze = Ze + i * Pp + 3 * B;
                ze[0] = 3.0 * (dsum ? acc[0] : acc[3]);
                ze[1] = 3.0 * (dsum ? acc[1] : acc[4]);
                ze[2] = 3.0 * (dsum ? acc[2] : acc[5]);
            }
        }
        const double di = -3.0 * acc[15];
        const double red[9] = {ai * (6.0 * acc[9] + di), ai * (6.0 * acc[10] + di),
                               ai * (6.0 * acc[11] + di), ai * 6.0 * acc[12],
                               ai * 6.0 * acc[13], ai * 6.0 * acc[14],
                               ai * 3.0 * acc[0], ai * 3.0 * acc[1], ai * 3.0 * acc[2]};
        double *dp = Dpart + ((int64_t)t * n_atom + B) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            if (!dsum) {   // B < A: the assembly reads both parts from the (B, A) sums
                if (lane == 0) dp[k] = 0.0;
                continue;
            }
            const double tot = wave_sum(red[k]);
            if (lane == 0) dp[k] = tot;
        }
    }
    if (INTS && live) {
        // the group that holds the own atom adds the self pair in FP64:
        // E += a Phi, U += -a Phi h, A += 2 a Phi m (W, B, C get none)
        double self[6] = {0, 0, 0, 0, 0, 0};
        if (A % bgroups == grp) {
            const double4 pd = Pd[i];
            const SelfPair q = self_pair(pd.x);
            self[0] = pd.y * q.phi;
            self[1] = -pd.y * q.phi * q.h;
            self[3] = 2.0 * pd.y * q.phi * q.m;
        }
        const double sc[6] = {-1.5, 1.5, 1.5, -3.0, -3.0, -3.0};
#pragma unroll
        for (int k = 0; k < 6; ++k)
            Ipart[((int64_t)grp * NI + k) * npad + i] = sc[k] * pint[k] + self[k];
    }
}

}  // namespace

}  // namespace vv10
