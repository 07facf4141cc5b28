/*
 * VV10 oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, obviously-correct FP64 CPU evaluation of the VV10 energy,
 * grid-level potential and nuclear-Hessian grid terms, written from
 * Liang, Feng, Liu & Head-Gordon, "Analytical harmonic vibrational
 * frequencies with VV10-containing density functionals" (arXiv 2208.14639),
 * Section II.  Every function cites the equation it evaluates.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library; the HIP library shares no code with it.
 *
 * Conventions (the readings of the paper this file follows):
 *  - every inner sum over j runs over ALL grid points, j = i included;
 *  - rho^x_i, gamma^x_i are total derivatives with the grid point moving with
 *    its owner atom, and gamma^x = 2 grad(rho) . grad(rho)^x;
 *  - f^{xy}_{ij} is normalised so that d2E/dx_i dy_j = w_i w_j f^{xy}_{ij};
 *  - the weight-derivative terms (E_w, E_{w,w}, E_{G,w}, E_{w,gr}) are zero
 *    for weights that depend only on the distance to the owner atom; for
 *    position-dependent weights the C functions here provide the
 *    weight-perturbed inner integrals E^{Bw}, U^{Bw}, W^{Bw}, and the
 *    Python wrapper composes the terms from them;
 *  - the returned "Hessian terms" exclude the caller's
 *    sum_i w_i (f^rho_i rho^{AB}_i + f^gamma_i gamma^{AB}_i).
 *  - No density cutoff and no screening.
 *
 * Parity status: every function here is pinned by the CPU tests (closed
 * forms, brute force, uniform-gas limit, finite differences, invariances).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Per-point quantities (Section II.A: omega, kappa, beta and their    */
/* partial derivatives with respect to rho and gamma).                 */
/* ------------------------------------------------------------------ */

/* beta = (1/32) (3/b^2)^{3/4}  (Section II.A, uniform-density condition) */
double oracle_beta(double b) { return pow(3.0 / (b * b), 0.75) / 32.0; }

enum { PT_OMEGA, PT_KAPPA, PT_OMEGA_R, PT_OMEGA_G, PT_KAPPA_R, PT_OMEGA_RR,
       PT_OMEGA_RG, PT_OMEGA_GG, PT_KAPPA_RR, PT_N };

/* omega = sqrt(C gamma^2/rho^4 + 4 pi rho/3), kappa = b (3 pi/2) (rho/9pi)^{1/6}
 * (Section II.A).  The paper names but does not print the first and second
 * partials used in the potential and in f^{rho rho} ... f^{gamma gamma}; they
 * are obtained here by differentiating S = omega^2:
 *   S_r = -4 C gamma^2/rho^5 + 4 pi/3,  S_g = 2 C gamma/rho^4,
 *   S_rr = 20 C gamma^2/rho^6, S_rg = -8 C gamma/rho^5, S_gg = 2 C/rho^4,
 *   omega_x = S_x/(2 omega), omega_xy = S_xy/(2 omega) - S_x S_y/(4 omega^3),
 *   kappa_r = kappa/(6 rho), kappa_rr = -5 kappa/(36 rho^2).             */
void oracle_point(double b, double C, double rho, double gamma, double *out)
{
    double t = gamma / (rho * rho);              /* gamma/rho^2 */
    double S = C * t * t + 4.0 * PI * rho / 3.0;
    double om = sqrt(S);
    double ka = b * 1.5 * PI * pow(rho / (9.0 * PI), 1.0 / 6.0);
    double Sr = -4.0 * C * t * t / rho + 4.0 * PI / 3.0;
    double Sg = 2.0 * C * gamma / (rho * rho * rho * rho);
    double Srr = 20.0 * C * t * t / (rho * rho);
    double Srg = -8.0 * C * gamma / (rho * rho * rho * rho * rho);
    double Sgg = 2.0 * C / (rho * rho * rho * rho);
    out[PT_OMEGA] = om;
    out[PT_KAPPA] = ka;
    out[PT_OMEGA_R] = Sr / (2.0 * om);
    out[PT_OMEGA_G] = Sg / (2.0 * om);
    out[PT_KAPPA_R] = ka / (6.0 * rho);
    out[PT_OMEGA_RR] = Srr / (2.0 * om) - Sr * Sr / (4.0 * om * om * om);
    out[PT_OMEGA_RG] = Srg / (2.0 * om) - Sr * Sg / (4.0 * om * om * om);
    out[PT_OMEGA_GG] = Sgg / (2.0 * om) - Sg * Sg / (4.0 * om * om * om);
    out[PT_KAPPA_RR] = -5.0 * ka / (36.0 * rho * rho);
}

/* atom_of must be nondecreasing; seg[A]..seg[A+1] are atom A's points. */
static int atom_segments(int64_t n, int32_t n_atom, const int32_t *atom_of, int64_t *seg)
{
    for (int64_t i = 1; i < n; ++i) if (atom_of[i] < atom_of[i - 1]) return -3;
    for (int32_t A = 0; A <= n_atom; ++A) seg[A] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (atom_of[i] < 0 || atom_of[i] >= n_atom) return -1;
        seg[atom_of[i] + 1] += 1;
    }
    for (int32_t A = 0; A < n_atom; ++A) seg[A + 1] += seg[A];
    return 0;
}

static double *all_points(int64_t n, const double *rho, const double *gamma,
                          double b, double C)
{
    double *pt = (double *)malloc(sizeof(double) * PT_N * (size_t)n);
    for (int64_t i = 0; i < n; ++i) oracle_point(b, C, rho[i], gamma[i], pt + PT_N * i);
    return pt;
}

/* gamma = |grad rho|^2 */
void oracle_gamma(int64_t n, const double *grad_rho, double *gamma)
{
    for (int64_t i = 0; i < n; ++i) {
        const double *g = grad_rho + 3 * i;
        gamma[i] = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    }
}

/* gamma^x_i = 2 grad(rho)_i . grad(rho)^x_i  (total derivative of |grad rho|^2) */
void oracle_gamma_x(int64_t n, int32_t n_pert, const double *grad_rho,
                    const double *grad_rho_x, double *gamma_x)
{
    for (int32_t x = 0; x < n_pert; ++x)
        for (int64_t i = 0; i < n; ++i) {
            const double *g = grad_rho + 3 * i;
            const double *gx = grad_rho_x + ((size_t)x * n + i) * 3;
            gamma_x[(size_t)x * n + i] = 2.0 * (g[0] * gx[0] + g[1] * gx[1] + g[2] * gx[2]);
        }
}

/* ------------------------------------------------------------------ */
/* Pair geometry: R^2_ij, g_ij = omega_i R^2 + kappa_i,                */
/* g'_ij = omega_j R^2 + kappa_j, Phi_ij = -3/(2 g g' (g + g'))        */
/* (Section II.A, kernel and its quadrature form).                     */
/* ------------------------------------------------------------------ */
typedef struct { double R2, g, gp, s, phi; } pair_t;

static pair_t pair_terms(const double *ri, const double *rj, const double *pti,
                         const double *ptj)
{
    pair_t p;
    double dx = ri[0] - rj[0], dy = ri[1] - rj[1], dz = ri[2] - rj[2];
    p.R2 = dx * dx + dy * dy + dz * dz;
    p.g = pti[PT_OMEGA] * p.R2 + pti[PT_KAPPA];
    p.gp = ptj[PT_OMEGA] * p.R2 + ptj[PT_KAPPA];
    p.s = p.g + p.gp;
    p.phi = -3.0 / (2.0 * p.g * p.gp * p.s);
    return p;
}

/* ------------------------------------------------------------------ */
/* Inner integrals E_i, U_i, W_i (Section II.A) and A_i, B_i, C_i      */
/* (Section II.B), all six as plain sums over every j.                 */
/* out is [6][n] in the order E, U, W, A, B, C.                        */
/* ------------------------------------------------------------------ */
static void pair_integrals_rows(int64_t i0, int64_t i1, int64_t n, const double *coords,
                                const double *w, const double *rho, const double *pt,
                                double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = i0; i < i1; ++i) {
        double E = 0, U = 0, W = 0, A = 0, B = 0, Cc = 0;
        for (int64_t j = 0; j < n; ++j) {
            pair_t p = pair_terms(coords + 3 * i, coords + 3 * j, pt + PT_N * i, pt + PT_N * j);
            double wr = w[j] * rho[j];
            double h = 1.0 / p.s + 1.0 / p.g;
            double m = 1.0 / (p.s * p.s) + 1.0 / (p.s * p.g) + 1.0 / (p.g * p.g);
            E += wr * p.phi;
            U += -wr * p.phi * h;
            W += -wr * p.phi * p.R2 * h;
            A += 2.0 * wr * p.phi * m;
            B += 2.0 * wr * p.phi * p.R2 * m;
            Cc += 2.0 * wr * p.phi * p.R2 * p.R2 * m;
        }
        out[0 * n + i] = E; out[1 * n + i] = U; out[2 * n + i] = W;
        out[3 * n + i] = A; out[4 * n + i] = B; out[5 * n + i] = Cc;
    }
}

static void pair_integrals_pt(int64_t n, const double *coords, const double *w,
                              const double *rho, const double *pt, double *out)
{
    pair_integrals_rows(0, n, n, coords, w, rho, pt, out);
}

void oracle_pair_integrals(int64_t n, const double *coords, const double *w,
                           const double *rho, const double *gamma, double b,
                           double C, double *out)
{
    double *pt = all_points(n, rho, gamma, b, C);
    pair_integrals_pt(n, coords, w, rho, pt, out);
    free(pt);
}

/* ------------------------------------------------------------------ */
/* Energy and potential (Section II.A):                                 */
/*   E = sum_i w_i rho_i (beta + E_i/2)                                  */
/*   f^rho_i = beta + E_i + rho_i (kappa_r U_i + omega_r W_i)            */
/*   f^gamma_i = rho_i omega_g W_i                                       */
/* ints (optional) receives [6][n] E, U, W, A, B, C.                     */
/* ------------------------------------------------------------------ */
void oracle_energy_potential(int64_t n, const double *coords, const double *w,
                             const double *rho, const double *gamma, double b,
                             double C, double *energy, double *f_rho,
                             double *f_gamma, double *ints)
{
    double *pt = all_points(n, rho, gamma, b, C);
    double *I = ints ? ints : (double *)malloc(sizeof(double) * 6 * (size_t)n);
    pair_integrals_pt(n, coords, w, rho, pt, I);
    double beta = oracle_beta(b);
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double Ei = I[i], Ui = I[n + i], Wi = I[2 * n + i];
        const double *q = pt + PT_N * i;
        e += w[i] * rho[i] * (beta + 0.5 * Ei);
        if (f_rho) f_rho[i] = beta + Ei + rho[i] * (q[PT_KAPPA_R] * Ui + q[PT_OMEGA_R] * Wi);
        if (f_gamma) f_gamma[i] = rho[i] * q[PT_OMEGA_G] * Wi;
    }
    *energy = e;
    if (!ints) free(I);
    free(pt);
}

/* The potential of rows i in [i0, i1) only (each row needs its own     */
/* inner integrals, a sum over every j): f^rho_i, f^gamma_i and the      */
/* integrals [6][n], those rows set.                                     */
void oracle_potential_rows(int64_t i0, int64_t i1, int64_t n, const double *coords,
                           const double *w, const double *rho, const double *gamma, double b,
                           double C, double *ints, double *f_rho, double *f_gamma)
{
    double *pt = all_points(n, rho, gamma, b, C);
    pair_integrals_rows(i0, i1, n, coords, w, rho, pt, ints);
    double beta = oracle_beta(b);
    for (int64_t i = i0; i < i1; ++i) {
        double Ei = ints[i], Ui = ints[n + i], Wi = ints[2 * n + i];
        const double *q = pt + PT_N * i;
        f_rho[i] = beta + Ei + rho[i] * (q[PT_KAPPA_R] * Ui + q[PT_OMEGA_R] * Wi);
        f_gamma[i] = rho[i] * q[PT_OMEGA_G] * Wi;
    }
    free(pt);
}

/* ------------------------------------------------------------------ */
/* One row i of the four second-derivative matrices (Section II.B):     */
/* f^{rho rho}_{ij}, f^{gamma rho}_{ij}, f^{rho gamma}_{ij},              */
/* f^{gamma gamma}_{ij}: the pair expression for every j (j = i too),    */
/* plus delta_ij/w_i times the local bracket built from U, W, A, B, C.   */
/* I is [6][n] from pair_integrals_pt.  The bracket of the delta_ij/w_i  */
/* term goes to loc[3] = (rho rho, gamma rho = rho gamma, gamma gamma)  */
/* when loc is given (the caller then multiplies it by w_i itself, so a  */
/* zero weight needs no division), else it is added over w_i.            */
/* ------------------------------------------------------------------ */
static void second_row(int64_t i, int64_t n, const double *coords, const double *w,
                       const double *rho, const double *pt, const double *I,
                       double *frr, double *fgr, double *frg, double *fgg, double *loc)
{
    const double *pi_ = pt + PT_N * i;
    const double wkr_i = pi_[PT_KAPPA_R], wor_i = pi_[PT_OMEGA_R], wog_i = pi_[PT_OMEGA_G];
    for (int64_t j = 0; j < n; ++j) {
        const double *pj = pt + PT_N * j;
        pair_t p = pair_terms(coords + 3 * i, coords + 3 * j, pi_, pj);
        double ai = rho[i] * (p.R2 * wor_i + wkr_i);
        double aj = rho[j] * (p.R2 * pj[PT_OMEGA_R] + pj[PT_KAPPA_R]);
        double two = 2.0 / (p.s * p.s) + 2.0 / (p.g * p.gp);
        double hi = 1.0 / p.s + 1.0 / p.g;
        double hj = 1.0 / p.s + 1.0 / p.gp;
        frr[j] = p.phi * (ai * aj * two - ai * hi - aj * hj + 1.0);
        fgr[j] = rho[i] * wog_i * p.R2 * p.phi * (aj * two - hi);
        frg[j] = rho[j] * pj[PT_OMEGA_G] * p.R2 * p.phi * (ai * two - hj);
        fgg[j] = rho[i] * rho[j] * wog_i * pj[PT_OMEGA_G] * p.R2 * p.R2 * p.phi * two;
    }
    double U = I[n + i], W = I[2 * n + i], A = I[3 * n + i], B = I[4 * n + i], Cc = I[5 * n + i];
    double r = rho[i];
    double loc_rr = 2.0 * wor_i * W + 2.0 * wkr_i * U
        + r * (pi_[PT_OMEGA_RR] * W + pi_[PT_KAPPA_RR] * U + wkr_i * wkr_i * A
               + wor_i * wor_i * Cc + 2.0 * wor_i * wkr_i * B);
    double loc_gr = wog_i * W + r * pi_[PT_OMEGA_RG] * W + r * wog_i * wkr_i * B
        + r * wog_i * wor_i * Cc;
    double loc_gg = r * (pi_[PT_OMEGA_GG] * W + wog_i * wog_i * Cc);
    if (loc) {
        loc[0] = loc_rr; loc[1] = loc_gr; loc[2] = loc_gg;
        return;
    }
    frr[i] += loc_rr / w[i];
    fgr[i] += loc_gr / w[i];
    frg[i] += loc_gr / w[i];
    fgg[i] += loc_gg / w[i];
}

/* Full n x n matrices (tiny n only; used by the finite-difference pins). */
void oracle_second_matrices(int64_t n, const double *coords, const double *w,
                            const double *rho, const double *gamma, double b, double C,
                            double *frr, double *fgr, double *frg, double *fgg)
{
    double *pt = all_points(n, rho, gamma, b, C);
    double *I = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    pair_integrals_pt(n, coords, w, rho, pt, I);
    for (int64_t i = 0; i < n; ++i)
        second_row(i, n, coords, w, rho, pt, I, frr + i * n, fgr + i * n, frg + i * n, fgg + i * n,
                   NULL);
    free(I);
    free(pt);
}

/* ------------------------------------------------------------------ */
/* Response rows (Section II.B, the inner sums of E^{AB}_{G,G}):        */
/*   Yr_{x i} = sum_j w_j (f^{rho rho}_{ij} rho^x_j + f^{rho gamma}_{ij} gamma^x_j) */
/*   Yg_{x i} = sum_j w_j (f^{gamma rho}_{ij} rho^x_j + f^{gamma gamma}_{ij} gamma^x_j) */
/* for rows i in [i0, i1); Yr, Yg are [n_pert][n] (only those rows set). */
/* The j = i term w_i (delta_ii/w_i) loc is taken as loc itself (exact   */
/* cancellation), which keeps points of zero weight finite.             */
/* This is the dominant O(N^2 P) step of the oracle.                     */
/* ------------------------------------------------------------------ */
static void response_rows(int64_t i0, int64_t i1, int64_t n, const double *coords,
                          const double *w, const double *rho, const double *pt,
                          const double *I, int32_t n_pert, const double *rho_x,
                          const double *gamma_x, double *Yr, double *Yg)
{
#pragma omp parallel
    {
        double *frr = (double *)malloc(sizeof(double) * 4 * (size_t)n);
        double *fgr = frr + n, *frg = frr + 2 * n, *fgg = frr + 3 * n;
#pragma omp for schedule(static)
        for (int64_t i = i0; i < i1; ++i) {
            double loc[3];
            second_row(i, n, coords, w, rho, pt, I, frr, fgr, frg, fgg, loc);
            for (int32_t x = 0; x < n_pert; ++x) {
                const double *rx = rho_x + (size_t)x * n, *gx = gamma_x + (size_t)x * n;
                double yr = 0.0, yg = 0.0;
                for (int64_t j = 0; j < n; ++j) {
                    yr += w[j] * (frr[j] * rx[j] + frg[j] * gx[j]);
                    yg += w[j] * (fgr[j] * rx[j] + fgg[j] * gx[j]);
                }
                yr += loc[0] * rx[i] + loc[1] * gx[i];
                yg += loc[1] * rx[i] + loc[2] * gx[i];
                Yr[(size_t)x * n + i] = yr;
                Yg[(size_t)x * n + i] = yg;
            }
        }
        free(frr);
    }
}

void oracle_response_rows(int64_t i0, int64_t i1, int64_t n, const double *coords,
                          const double *w, const double *rho, const double *gamma,
                          double b, double C, int32_t n_pert, const double *rho_x,
                          const double *gamma_x, double *Yr, double *Yg)
{
    double *pt = all_points(n, rho, gamma, b, C);
    double *I = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    /* the local bracket of row i needs row i's integrals only */
    pair_integrals_rows(i0, i1, n, coords, w, rho, pt, I);
    response_rows(i0, i1, n, coords, w, rho, pt, I, n_pert, rho_x, gamma_x, Yr, Yg);
    free(I);
    free(pt);
}

/* ------------------------------------------------------------------ */
/* Grid-position intermediates (Section II.B):                          */
/*   E^{Bgr}_i, U^{Bgr}_i, W^{Bgr}_i (3-vectors) for i not in B as sums   */
/*   over j in B; for i in B, minus the sum over the other atoms         */
/*   (translational invariance).  Egr, Ugr, Wgr are [n][n_atom][3].      */
/* T = omega_i/g + omega_j/g' + (omega_i + omega_j)/(g + g').            */
/* ------------------------------------------------------------------ */
static void grid_vectors(int64_t n, int32_t n_atom, const int32_t *atom_of,
                         const double *coords, const double *w, const double *rho,
                         const double *pt, double *Egr, double *Ugr, double *Wgr)
{
    size_t tot = (size_t)n * n_atom * 3;
    memset(Egr, 0, sizeof(double) * tot);
    memset(Ugr, 0, sizeof(double) * tot);
    memset(Wgr, 0, sizeof(double) * tot);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double *pi_ = pt + PT_N * i;
        double oi = pi_[PT_OMEGA];
        for (int64_t j = 0; j < n; ++j) {
            int32_t B = atom_of[j];
            if (B == atom_of[i]) continue;
            const double *pj = pt + PT_N * j;
            double oj = pj[PT_OMEGA];
            pair_t p = pair_terms(coords + 3 * i, coords + 3 * j, pi_, pj);
            double T = oi / p.g + oj / p.gp + (oi + oj) / p.s;
            double h = 1.0 / p.s + 1.0 / p.g;
            double Q = oi / (p.g * p.g) + (oi + oj) / (p.s * p.s);
            double wr = w[j] * rho[j];
            double e = -2.0 * wr * p.phi * T;
            double u = 2.0 * wr * p.phi * (T * h + Q);
            double v = 2.0 * wr * p.phi * (p.R2 * T * h + p.R2 * Q - h);
            for (int a = 0; a < 3; ++a) {
                double d = coords[3 * j + a] - coords[3 * i + a];     /* r_j - r_i */
                size_t k = ((size_t)i * n_atom + B) * 3 + a;
                Egr[k] += e * d;
                Ugr[k] += u * d;
                Wgr[k] += v * d;
            }
        }
        /* i in B = O(i): minus the sum over every other atom C */
        int32_t Oi = atom_of[i];
        for (int a = 0; a < 3; ++a) {
            double se = 0, su = 0, sw = 0;
            for (int32_t C = 0; C < n_atom; ++C) {
                if (C == Oi) continue;
                size_t k = ((size_t)i * n_atom + C) * 3 + a;
                se += Egr[k]; su += Ugr[k]; sw += Wgr[k];
            }
            size_t k = ((size_t)i * n_atom + Oi) * 3 + a;
            Egr[k] = -se; Ugr[k] = -su; Wgr[k] = -sw;
        }
    }
}

void oracle_grid_vectors(int64_t n, int32_t n_atom, const int32_t *atom_of,
                         const double *coords, const double *w, const double *rho,
                         const double *gamma, double b, double C, double *Egr,
                         double *Ugr, double *Wgr)
{
    double *pt = all_points(n, rho, gamma, b, C);
    grid_vectors(n, n_atom, atom_of, coords, w, rho, pt, Egr, Ugr, Wgr);
    free(pt);
}

/* D^B_i (3x3) for i not in B (Section II.B):
 *   D^B_i = -2 sum_{j in B} w_j rho_j Phi_ij [2 S (r_j - r_i)(r_j - r_i)^T - T I]
 * with S = T^2 + (omega_i/g)^2 + (omega_j/g')^2 + ((omega_i+omega_j)/(g+g'))^2. */
static void grid_D(int64_t i, int64_t j0, int64_t j1, const double *coords,
                   const double *w, const double *rho, const double *pt, double *D)
{
    for (int k = 0; k < 9; ++k) D[k] = 0.0;
    const double *pi_ = pt + PT_N * i;
    double oi = pi_[PT_OMEGA];
    for (int64_t j = j0; j < j1; ++j) {
        const double *pj = pt + PT_N * j;
        double oj = pj[PT_OMEGA];
        pair_t p = pair_terms(coords + 3 * i, coords + 3 * j, pi_, pj);
        double T = oi / p.g + oj / p.gp + (oi + oj) / p.s;
        double S = T * T + (oi / p.g) * (oi / p.g) + (oj / p.gp) * (oj / p.gp)
                 + ((oi + oj) / p.s) * ((oi + oj) / p.s);
        double f = -2.0 * w[j] * rho[j] * p.phi;
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = coords[3 * j + a] - coords[3 * i + a];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                D[3 * a + c] += f * (2.0 * S * d[a] * d[c] - (a == c ? T : 0.0));
    }
}

int oracle_grid_D(int64_t i, int32_t B, int64_t n, int32_t n_atom, const int32_t *atom_of,
                  const double *coords, const double *w, const double *rho,
                  const double *gamma, double b, double C, double *D)
{
    int64_t *seg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_atom + 1));
    int rc = atom_segments(n, n_atom, atom_of, seg);
    if (rc == 0) {
        double *pt = all_points(n, rho, gamma, b, C);
        grid_D(i, seg[B], seg[B + 1], coords, w, rho, pt, D);
        free(pt);
    }
    free(seg);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Nuclear gradient (Section II.A), weight term identically zero:       */
/*   E^A_G = sum_i w_i (f^rho_i rho^A_i + f^gamma_i gamma^A_i)             */
/*   E^A_gr, first (two-sum) form:                                        */
/*     - sum_{i in A} sum_{j notin A} w_i w_j rho_i rho_j Phi T (r_i - r_j) */
/*     - sum_{i notin A} sum_{j in A} w_i w_j rho_i rho_j Phi T (r_j - r_i) */
/* grad is [3 n_atom]; parts (optional) [2][3 n_atom] = (E_G, E_gr).      */
/* ------------------------------------------------------------------ */
int oracle_gradient(int64_t n, int32_t n_atom, const int32_t *atom_of,
                     const double *coords, const double *w, const double *rho,
                     const double *gamma, double b, double C, const double *rho_x,
                     const double *gamma_x, double *grad, double *parts)
{
    int32_t P = 3 * n_atom;
    double *pt = all_points(n, rho, gamma, b, C);
    double *I = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    pair_integrals_pt(n, coords, w, rho, pt, I);
    double beta = oracle_beta(b);
    double *fr = (double *)malloc(sizeof(double) * (size_t)n);
    double *fg = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const double *q = pt + PT_N * i;
        fr[i] = beta + I[i] + rho[i] * (q[PT_KAPPA_R] * I[n + i] + q[PT_OMEGA_R] * I[2 * n + i]);
        fg[i] = rho[i] * q[PT_OMEGA_G] * I[2 * n + i];
    }
    double *gG = (double *)calloc((size_t)P, sizeof(double));
    double *gr = (double *)calloc((size_t)P, sizeof(double));
    for (int32_t x = 0; x < P; ++x) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i)
            s += w[i] * (fr[i] * rho_x[(size_t)x * n + i] + fg[i] * gamma_x[(size_t)x * n + i]);
        gG[x] = s;
    }
    int64_t *seg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_atom + 1));
    int rc = atom_segments(n, n_atom, atom_of, seg);
#pragma omp parallel for schedule(dynamic)
    for (int32_t A = 0; A < n_atom; ++A) {
        if (rc) continue;
        double acc[3] = {0, 0, 0};
        /* first sum: i in A, j not in A, direction r_i - r_j */
        for (int64_t i = seg[A]; i < seg[A + 1]; ++i)
            for (int64_t j = 0; j < n; ++j) {
                if (atom_of[j] == A) continue;
                const double *pi_ = pt + PT_N * i, *pj = pt + PT_N * j;
                pair_t p = pair_terms(coords + 3 * i, coords + 3 * j, pi_, pj);
                double oi = pi_[PT_OMEGA], oj = pj[PT_OMEGA];
                double T = oi / p.g + oj / p.gp + (oi + oj) / p.s;
                double f = w[i] * w[j] * rho[i] * rho[j] * p.phi * T;
                for (int a = 0; a < 3; ++a) acc[a] -= f * (coords[3 * i + a] - coords[3 * j + a]);
            }
        /* second sum: i not in A, j in A, direction r_j - r_i */
        for (int64_t i = 0; i < n; ++i) {
            if (atom_of[i] == A) continue;
            for (int64_t j = seg[A]; j < seg[A + 1]; ++j) {
                const double *pi_ = pt + PT_N * i, *pj = pt + PT_N * j;
                pair_t p = pair_terms(coords + 3 * i, coords + 3 * j, pi_, pj);
                double oi = pi_[PT_OMEGA], oj = pj[PT_OMEGA];
                double T = oi / p.g + oj / p.gp + (oi + oj) / p.s;
                double f = w[i] * w[j] * rho[i] * rho[j] * p.phi * T;
                for (int a = 0; a < 3; ++a) acc[a] -= f * (coords[3 * j + a] - coords[3 * i + a]);
            }
        }
        for (int a = 0; a < 3; ++a) gr[3 * A + a] = acc[a];
    }
    free(seg);
    for (int32_t x = 0; x < P; ++x) {
        grad[x] = gG[x] + gr[x];
        if (parts) { parts[x] = gG[x]; parts[P + x] = gr[x]; }
    }
    free(gG); free(gr); free(fr); free(fg); free(I); free(pt);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Nuclear-Hessian grid terms (Section II.B, nine-term split with the  */
/* weight terms identically zero):                                      */
/*   H = E_{G,G} (without the caller's f^rho rho^{AB} + f^gamma gamma^{AB}) */
/*     + E_{G,gr} + (E_{G,gr})^T + E_{gr,gr}                              */
/* returned symmetrised, (H + H^T)/2, with the pre-symmetrisation        */
/* max |H - H^T| in *asym.  parts (optional) [3][P][P] = GG, Ggr, grgr.  */
/* resp_rho/resp_gamma (optional) [P][n] = Yr, Yg of response_rows.      */
/* ------------------------------------------------------------------ */
int oracle_hessian_terms(int64_t n, int32_t n_atom, const int32_t *atom_of,
                         const double *coords, const double *w, const double *rho,
                         const double *gamma, double b, double C, int32_t n_pert,
                         const double *rho_x, const double *gamma_x, double *hess,
                         double *parts, double *resp_rho, double *resp_gamma,
                         double *asym)
{
    if (n_pert != 3 * n_atom) return -1;
    int64_t *seg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_atom + 1));
    int rc = atom_segments(n, n_atom, atom_of, seg);
    if (rc) { free(seg); return rc; }
    const int32_t P = n_pert;
    double *pt = all_points(n, rho, gamma, b, C);
    double *I = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    pair_integrals_pt(n, coords, w, rho, pt, I);

    /* E_{G,G}: sum_i w_i (rho^A_i Yr_{B i} + gamma^A_i Yg_{B i}) */
    double *Yr = resp_rho ? resp_rho : (double *)malloc(sizeof(double) * (size_t)P * n);
    double *Yg = resp_gamma ? resp_gamma : (double *)malloc(sizeof(double) * (size_t)P * n);
    response_rows(0, n, n, coords, w, rho, pt, I, P, rho_x, gamma_x, Yr, Yg);
    double *HGG = (double *)calloc((size_t)P * P, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int32_t A = 0; A < P; ++A)
        for (int32_t B = 0; B < P; ++B) {
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i)
                s += w[i] * (rho_x[(size_t)A * n + i] * Yr[(size_t)B * n + i]
                             + gamma_x[(size_t)A * n + i] * Yg[(size_t)B * n + i]);
            HGG[(size_t)A * P + B] = s;
        }

    /* E_{G,gr}[A][(B,b)] = sum_i w_i rho^A_i [E^{Bgr} + rho_i (kappa_r U^{Bgr} + omega_r W^{Bgr})]_b
     *                    + sum_i w_i gamma^A_i rho_i omega_g W^{Bgr}_b                      */
    size_t tot = (size_t)n * n_atom * 3;
    double *Egr = (double *)malloc(sizeof(double) * tot);
    double *Ugr = (double *)malloc(sizeof(double) * tot);
    double *Wgr = (double *)malloc(sizeof(double) * tot);
    grid_vectors(n, n_atom, atom_of, coords, w, rho, pt, Egr, Ugr, Wgr);
    double *HGgr = (double *)calloc((size_t)P * P, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int32_t A = 0; A < P; ++A)
        for (int32_t Bb = 0; Bb < P; ++Bb) {
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                const double *q = pt + PT_N * i;
                size_t k = (size_t)i * n_atom * 3 + Bb;   /* (i, B, b) with Bb = 3B + b */
                s += w[i] * rho_x[(size_t)A * n + i]
                       * (Egr[k] + rho[i] * (q[PT_KAPPA_R] * Ugr[k] + q[PT_OMEGA_R] * Wgr[k]))
                   + w[i] * gamma_x[(size_t)A * n + i] * rho[i] * q[PT_OMEGA_G] * Wgr[k];
            }
            HGgr[(size_t)A * P + Bb] = s;
        }

    /* E_{gr,gr}: for atoms A != B, sum_{i in A} w_i rho_i D^B_i;
     * E^{AA}_{gr,gr} = -sum_{B != A} E^{AB}_{gr,gr}. */
    double *Hgg = (double *)calloc((size_t)P * P, sizeof(double));
#pragma omp parallel for schedule(dynamic)
    for (int64_t AB = 0; AB < (int64_t)n_atom * n_atom; ++AB) {
        int32_t A = (int32_t)(AB / n_atom), B = (int32_t)(AB % n_atom);
        if (A == B) continue;
        double blk[9] = {0}, D[9];
        for (int64_t i = seg[A]; i < seg[A + 1]; ++i) {
            grid_D(i, seg[B], seg[B + 1], coords, w, rho, pt, D);
            for (int k = 0; k < 9; ++k) blk[k] += w[i] * rho[i] * D[k];
        }
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                Hgg[(size_t)(3 * A + a) * P + 3 * B + c] = blk[3 * a + c];
    }
    for (int32_t A = 0; A < n_atom; ++A)
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int32_t B = 0; B < n_atom; ++B)
                    if (B != A) s += Hgg[(size_t)(3 * A + a) * P + 3 * B + c];
                Hgg[(size_t)(3 * A + a) * P + 3 * A + c] = -s;
            }

    double amax = 0.0;
    for (int32_t A = 0; A < P; ++A)
        for (int32_t B = 0; B < P; ++B) {
            size_t ab = (size_t)A * P + B, ba = (size_t)B * P + A;
            double hab = HGG[ab] + HGgr[ab] + HGgr[ba] + Hgg[ab];
            double hba = HGG[ba] + HGgr[ba] + HGgr[ab] + Hgg[ba];
            double d = fabs(hab - hba);
            if (d > amax) amax = d;
            hess[ab] = 0.5 * (hab + hba);
        }
    if (asym) *asym = amax;
    if (parts) {
        size_t PP = (size_t)P * P;
        memcpy(parts, HGG, sizeof(double) * PP);
        for (size_t k = 0; k < PP; ++k) {
            size_t A = k / P, B = k % P;
            parts[PP + k] = HGgr[k] + HGgr[B * P + A];
        }
        memcpy(parts + 2 * PP, Hgg, sizeof(double) * PP);
    }
    free(Hgg); free(HGgr); free(Egr); free(Ugr); free(Wgr); free(HGG);
    if (!resp_rho) free(Yr);
    if (!resp_gamma) free(Yg);
    free(I); free(pt); free(seg);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Weight-perturbed inner integrals (Section II.B), for every column x   */
/* of w_x (the nuclear derivatives of the weights, [P][n]):             */
/*   E^{xw}_i = sum_j w^x_j rho_j Phi_ij                                 */
/*   U^{xw}_i = -sum_j w^x_j rho_j Phi_ij (1/(g + g') + 1/g)              */
/*   W^{xw}_i = -sum_j w^x_j rho_j Phi_ij R^2 (1/(g + g') + 1/g)          */
/* Rows i0 <= i < i1 only; Ew, Uw, Ww are [P][i1 - i0].                */
/* ------------------------------------------------------------------ */
void oracle_weight_integrals(int64_t i0, int64_t i1, int64_t n, const double *coords,
                             const double *rho, const double *gamma, double b, double C,
                             int32_t n_pert, const double *w_x, double *Ew, double *Uw,
                             double *Ww)
{
    double *pt = all_points(n, rho, gamma, b, C);
    int64_t m = i1 - i0;
#pragma omp parallel
    {
        double *e = (double *)malloc(sizeof(double) * (size_t)n_pert * 3);
#pragma omp for schedule(static)
        for (int64_t i = i0; i < i1; ++i) {
            memset(e, 0, sizeof(double) * (size_t)n_pert * 3);
            for (int64_t j = 0; j < n; ++j) {
                pair_t p = pair_terms(coords + 3 * i, coords + 3 * j, pt + PT_N * i, pt + PT_N * j);
                double h = 1.0 / p.s + 1.0 / p.g;
                for (int32_t x = 0; x < n_pert; ++x) {
                    double wr = w_x[(size_t)x * n + j] * rho[j];
                    e[3 * x + 0] += wr * p.phi;
                    e[3 * x + 1] += -wr * p.phi * h;
                    e[3 * x + 2] += -wr * p.phi * p.R2 * h;
                }
            }
            for (int32_t x = 0; x < n_pert; ++x) {
                Ew[(size_t)x * m + (i - i0)] = e[3 * x + 0];
                Uw[(size_t)x * m + (i - i0)] = e[3 * x + 1];
                Ww[(size_t)x * m + (i - i0)] = e[3 * x + 2];
            }
        }
        free(e);
    }
    free(pt);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
