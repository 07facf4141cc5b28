// The grid pass (Section II.B grid-position intermediates) and the gradient
// pass's grid sums; the per-wave unit of the grid pass is in grid_tile.h.
#include "grid_tile.h"

namespace vv10 {

namespace {

// The grid pass as one wave per (tile, atom group): blockIdx = (tile, group).
template <typename T, typename T4, bool INTS, bool ZE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_grid(
    int32_t n_atom, int32_t Pp, int32_t bgroups, int64_t npad, const int64_t *__restrict__ seg,
    const int32_t *__restrict__ tile_i0, const int32_t *__restrict__ tile_n,
    const int32_t *__restrict__ tile_atom, const T4 *__restrict__ P0,
    const T4 *__restrict__ P1, const double4 *__restrict__ Pd, double *__restrict__ Z,
    double *__restrict__ Ze, double *__restrict__ Dpart, double *__restrict__ Ipart) {
    __shared__ T4 sA[TG], sB[TG];
    grid_unit<T, T4, INTS, ZE>(n_atom, Pp, bgroups, npad, seg, tile_i0, tile_n, tile_atom, P0, P1,
                               Pd, Z, Ze, Dpart, Ipart, blockIdx.x, blockIdx.y, threadIdx.x, sA,
                               sB);
}

// I[k][i] = sum over atom groups of Ipart[grp][k][i] (group order),
// k0 <= k < nrows, i < n.
__global__ __launch_bounds__(256) void k_sum_groups(int64_t n, int64_t npad, int G, int nrows, int k0,
                                                    const double *__restrict__ Ipart,
                                                    double *__restrict__ I) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x + (int64_t)k0 * n;
    if (e >= (int64_t)nrows * n) return;
    const int k = (int)(e / n);
    const int64_t i = e - (int64_t)k * n;
    double a = 0.0;
#pragma unroll 8
    for (int gidx = 0; gidx < G; ++gidx) a += Ipart[((int64_t)gidx * nrows + k) * npad + i];
    I[k * npad + i] = a;
}

// Gradient pass (Section II.A): the pair integrals E, U, W of every outer
// point (over all j) and, per tile t of outer points (atom A) and atom
// B > A, Gpart[t][B][a] = sum_{i in t} a_i E^{Bgr}_{i,a} (zero for B <= A),
// from which the grid part of the gradient follows,
// E_gr = -sum_{B != A} sum_{i in A} a_i E^{Bgr}_i (translational invariance),
// the B < A terms being minus the (B, A) ones.
// The layout and the scaled sums are those of k_grid: E^{Bgr}_i = 3 sum_j p T d.
// Without INTS (the plan already holds E, U, W) only the grid sums are formed.
template <typename T, typename T4, bool INTS>
__global__ __launch_bounds__(64) void k_grid_grad(
    int32_t n_atom, int32_t bgroups, int64_t npad, const int64_t *__restrict__ seg,
    const int32_t *__restrict__ tile_i0, const int32_t *__restrict__ tile_n,
    const int32_t *__restrict__ tile_atom, const T4 *__restrict__ P0,
    const T4 *__restrict__ P1, const double4 *__restrict__ Pd, double *__restrict__ Gpart,
    double *__restrict__ Ipart) {
    __shared__ T4 sA[TG], sB[TG];
    const int t = blockIdx.x, grp = blockIdx.y, lane = threadIdx.x;
    const int A = tile_atom[t];
    const int nt = tile_n[t];
    const bool live = lane < nt;
    const int64_t i = (int64_t)tile_i0[t] + (live ? lane : 0);
    const T4 a0 = P0[i], a1 = P1[i];
    const double ai = live ? (double)a1.y : 0.0;
    const T oi = a0.w;
    double pint[3] = {};
    for (int B = grp; B < n_atom; B += bgroups) {
        const int64_t jb = seg[B], je = seg[B + 1];
        double acc[3] = {};
        // the tile sums are antisymmetric in (A, B) (a_i e_ij symmetric,
        // d_ij = -d_ji): formed for B > A only, the assembly takes the B < A
        // ones from the (B, A) sums; B <= A still adds to the pair integrals
        const bool gsum = B > A;
        if (!INTS && !gsum) {
            if (lane == 0)
                for (int k = 0; k < 3; ++k) Gpart[((int64_t)t * n_atom + B) * 3 + k] = 0.0;
            continue;
        }
        for (int64_t j0 = jb; j0 < je; j0 += TG) {
            __syncthreads();
            const int64_t j = j0 + lane;
            sA[lane] = P0[j < je ? j : jb];
            sB[lane] = P1[j < je ? j : jb];
            __syncthreads();
            const int cnt = (int)min((int64_t)TG, je - j0);
            T pc[3] = {}, c[3] = {};
            if (!gsum) {
                // the chunk of the tile's own points leaves out the self pair
                const int jself = (B == A && j0 == tile_i0[t]) ? lane : -1;
#pragma unroll 4
                for (int jj = 0; jj < cnt; ++jj) {
                    const PairGeo<T> q = pair_geo<T>(a0, a1, sA[jj], sB[jj]);
                    const T pj = jj == jself ? T(0) : q.p;
                    const T ph = pj * q.h;
                    pc[0] += pj;
                    pc[1] += ph;
                    pc[2] += ph * q.R2;
                }
            } else {
#pragma unroll 4
                for (int jj = 0; jj < cnt; ++jj) {
                    const T4 b0 = sA[jj];
                    const PairGeo<T> q = pair_geo<T>(a0, a1, b0, sB[jj]);
                    if (INTS) {
                        const T ph = q.p * q.h;
                        pc[0] += q.p;
                        pc[1] += ph;
                        pc[2] += ph * q.R2;
                    }
                    const T e = q.p * (oi * q.ig + b0.w * q.igp + (oi + b0.w) * q.is);
                    c[0] += e * (b0.x - a0.x);
                    c[1] += e * (b0.y - a0.y);
                    c[2] += e * (b0.z - a0.z);
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) acc[k] += (double)c[k];
            }
            if (INTS)
#pragma unroll
                for (int k = 0; k < 3; ++k) pint[k] += (double)pc[k];
        }
        double *gp = Gpart + ((int64_t)t * n_atom + B) * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double tot = gsum ? wave_sum(ai * 3.0 * acc[k]) : 0.0;
            if (lane == 0) gp[k] = tot;
        }
    }
    if (INTS && live) {
        // self pair in FP64 (group of the own atom): E += a Phi, U += -a Phi h
        double self[3] = {0, 0, 0};
        if (A % bgroups == grp) {
            const double4 pd = Pd[i];
            const SelfPair q = self_pair(pd.x);
            self[0] = pd.y * q.phi;
            self[1] = -pd.y * q.phi * q.h;
        }
        const double sc[3] = {-1.5, 1.5, 1.5};
#pragma unroll
        for (int k = 0; k < 3; ++k) Ipart[((int64_t)grp * 3 + k) * npad + i] = sc[k] * pint[k] + self[k];
    }
}

}  // namespace

template <bool INTS, bool ZE>
void grid_terms_launch(vv10_plan *p, double *Ze) {
    const Workspace &ws = p->ws;
    dim3 grid((unsigned)p->ntiles, (unsigned)ws.bgroups);
    if (p->prec == VV10_FP64)
        k_grid<double, double4, INTS, ZE><<<grid, TG, 0, p->stream>>>(
            p->n_atom, ws.Pp, ws.bgroups, p->npad, p->d_seg, p->d_tile_i0, p->d_tile_n,
            p->d_tile_atom, p->P0, p->P1, p->P1, ws.Z, Ze, ws.Dpart, ws.Igrp);
    else
        k_grid<float, float4, INTS, ZE><<<grid, TG, 0, p->stream>>>(
            p->n_atom, ws.Pp, ws.bgroups, p->npad, p->d_seg, p->d_tile_i0, p->d_tile_n,
            p->d_tile_atom, p->P0f, p->P1f, p->P1, ws.Z, Ze, ws.Dpart, ws.Igrp);
}

template <bool INTS>
void grid_terms_mode(vv10_plan *p, double *Ze) {
    if (Ze) grid_terms_launch<INTS, true>(p, Ze);
    else grid_terms_launch<INTS, false>(p, Ze);
}

template <bool INTS>
void grid_grad_mode(vv10_plan *p) {
    const GradWork &gw = p->gw;
    dim3 grid((unsigned)p->ntiles, (unsigned)gw.bgroups);
    if (p->prec == VV10_FP64)
        k_grid_grad<double, double4, INTS><<<grid, TG, 0, p->stream>>>(
            p->n_atom, gw.bgroups, p->npad, p->d_seg, p->d_tile_i0, p->d_tile_n, p->d_tile_atom,
            p->P0, p->P1, p->P1, gw.Gpart, gw.Igrp);
    else
        k_grid_grad<float, float4, INTS><<<grid, TG, 0, p->stream>>>(
            p->n_atom, gw.bgroups, p->npad, p->d_seg, p->d_tile_i0, p->d_tile_n, p->d_tile_atom,
            p->P0f, p->P1f, p->P1, gw.Gpart, gw.Igrp);
}

hipError_t launch_grid_terms(vv10_plan *p, double *Ze, int ints_from) {
    if (ints_from >= NI) {
        grid_terms_mode<false>(p, Ze);
        return hipGetLastError();
    }
    grid_terms_mode<true>(p, Ze);
    return launch_sum_groups(p, ints_from);
}

hipError_t launch_sum_groups(vv10_plan *p, int ints_from) {
    const int64_t tot = (int64_t)(NI - ints_from) * p->n;
    if (tot <= 0) return hipSuccess;
    k_sum_groups<<<(unsigned)((tot + 255) / 256), 256, 0, p->stream>>>(
        p->n, p->npad, p->ws.bgroups, NI, ints_from, p->ws.Igrp, p->I);
    return hipGetLastError();
}

hipError_t launch_grid_grad(vv10_plan *p, bool ints) {
    if (!ints) {
        grid_grad_mode<false>(p);
        return hipGetLastError();
    }
    grid_grad_mode<true>(p);
    const int64_t tot = (int64_t)3 * p->n;
    k_sum_groups<<<(unsigned)((tot + 255) / 256), 256, 0, p->stream>>>(p->n, p->npad, p->gw.bgroups,
                                                                       3, 0, p->gw.Igrp, p->I);
    return hipGetLastError();
}

}  // namespace vv10
