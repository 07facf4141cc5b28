/*
 * vv10.h -- C ABI of the MI355X VV10 double-grid engine.
 *
 * The library evaluates, on one GPU, the O(N_grid^2) double sums of the VV10
 * nonlocal correlation kernel
 *     Phi_ij = -3 / (2 g g' (g + g')),  g = omega_i R_ij^2 + kappa_i,
 *     g' = omega_j R_ij^2 + kappa_j
 * that give the VV10 energy, its grid-level potential and the nuclear
 * Hessian grid terms (Liang, Feng, Liu & Head-Gordon, arXiv 2208.14639,
 * Section II).  Atomic units throughout.
 *
 * Conventions shared by every entry point:
 *  - Every array argument is a DEVICE pointer, FP64 (int32 for atom_of),
 *    row-major, owned by the caller.  The library reads inputs only during
 *    the call that receives them and packs what it keeps into memory the
 *    plan owns.
 *  - Every call is asynchronous on the plan's HIP stream (the stream given
 *    to vv10_prepare), except vv10_prepare, which synchronises that stream
 *    once to read back its validation result.  Outputs are valid once the
 *    caller has synchronised the stream.
 *  - Errors are status codes; nothing throws across the ABI.  A call that
 *    returns VV10_E_ARG, VV10_E_STATE, VV10_E_DENSITY, VV10_E_GRID_ORDER or
 *    VV10_E_OOM has written no output.  After VV10_E_HIP (a failed launch or
 *    runtime call) the outputs are undefined and the plan refuses further
 *    work (VV10_E_STATE).  Any plan, failed or not, is safe to destroy.
 *  - A plan is used from one host thread and one stream at a time; distinct
 *    plans may run concurrently on distinct streams.
 *  - All inner sums run over every grid point, the self pair j = i included.
 *  - Unless a call receives the weights' nuclear derivatives, quadrature
 *    weights are taken as independent of nuclear positions (they move
 *    rigidly with their owner atom), so the weight-derivative terms of the
 *    paper's gradient and nine-term Hessian split vanish.  vv10_nuclear_terms
 *    and vv10_gradient accept w^x (weights that depend on every nucleus, as
 *    for an atom-partitioned grid) and then add those terms.
 */
#ifndef VV10_H
#define VV10_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VV10_OK = 0,
    VV10_E_ARG = -1,        /* bad size, null pointer, atom index out of range, n_pert != 3 n_atom */
    VV10_E_DENSITY = -2,    /* some rho <= 0, or a non-finite rho, grad rho, weight or coordinate */
    VV10_E_GRID_ORDER = -3, /* atom_of is not nondecreasing */
    VV10_E_OOM = -4,        /* device allocation failed */
    VV10_E_HIP = -5,        /* a HIP runtime call failed */
    VV10_E_STATE = -6       /* call out of order (e.g. a destroyed or failed plan) */
} vv10_status;

/* Arithmetic of the O(N^2) parts.  Per-point preparation, every
 * cross-tile accumulation, the energy and Hessian reductions and the
 * symmetrisation are FP64 in all modes. */
typedef enum {
    VV10_FP64 = 0,          /* all pair arithmetic and the contraction in FP64 */
    VV10_MIXED_FP32 = 1,    /* pair arithmetic FP32; contraction on FP32 MFMA */
    VV10_MIXED_BF16X3 = 2   /* pair arithmetic FP32; contraction as split-BF16 (hi*hi + hi*lo + lo*hi) MFMA */
} vv10_precision;

/* VV10 parameters b and C (Section II.A: kappa = b (3 pi/2)(rho/9pi)^{1/6},
 * omega = sqrt(C gamma^2/rho^4 + 4 pi rho/3), beta = (1/32)(3/b^2)^{3/4}). */
typedef struct {
    double b;
    double C;
} vv10_params;

typedef struct vv10_plan vv10_plan; /* opaque; owns its device workspace */

/*
 * vv10_prepare -- validate and pack one grid (Section II.A, per-point
 * intermediates omega, kappa and their first and second partials).
 *
 *  params    b, C.
 *  n_grid    N >= 1 grid points.  n_atom >= 1 atoms.
 *  coords    [N][3] point positions (bohr).
 *  weights   [N] quadrature weights (> 0 not required, finite).
 *  atom_of   [N] owner atom of each point, 0 <= atom_of[i] < n_atom, nondecreasing
 *            (points grouped by atom; the grid moves rigidly with its atom).
 *  rho       [N] density, every value > 0 and finite.
 *  grad_rho  [N][3] density gradient.
 *  prec      arithmetic mode for the O(N^2) work of later calls.
 *  stream    HIP stream every later call of this plan runs on (0 = null stream).
 *  out       receives the plan; set to NULL on error.
 * Errors: VV10_E_ARG, VV10_E_DENSITY, VV10_E_GRID_ORDER, VV10_E_OOM, VV10_E_HIP.
 * Synchronises `stream` once to read its validation flag.
 */
vv10_status vv10_prepare(const vv10_params *params, int64_t n_grid, int32_t n_atom,
                         const double *coords, const double *weights,
                         const int32_t *atom_of, const double *rho,
                         const double *grad_rho, vv10_precision prec,
                         hipStream_t stream, vv10_plan **out);

/*
 * vv10_energy_potential -- VV10 energy and grid-level potential
 * (Section II.A):
 *   E_i = sum_j w_j rho_j Phi_ij,
 *   U_i = -sum_j w_j rho_j Phi_ij (1/(g+g') + 1/g),
 *   W_i = -sum_j w_j rho_j Phi_ij R_ij^2 (1/(g+g') + 1/g),
 *   energy  = sum_i w_i rho_i (beta + E_i/2),
 *   f_rho_i = beta + E_i + rho_i (dkappa/drho U_i + domega/drho W_i),
 *   f_gamma_i = rho_i domega/dgamma W_i
 * (so dE/drho_i = w_i f_rho_i and dE/dgamma_i = w_i f_gamma_i).
 *  energy   [1] device scalar.  f_rho, f_gamma [N]; either may be NULL.
 * The pair integrals depend only on the plan's grid and density, so a plan
 * forms each of them once and keeps it: this call's pair pass computes E, U,
 * W unless an earlier call on the plan formed them (vv10_nuclear_terms adds
 * A, B, C in its grid pass; vv10_gradient forms E, U, W in its own).
 * Errors: VV10_E_ARG (energy NULL), VV10_E_STATE, VV10_E_HIP.
 */
vv10_status vv10_energy_potential(vv10_plan *plan, double *energy, double *f_rho,
                                  double *f_gamma);

/* Outputs of vv10_nuclear_terms: each is DEVICE memory, FP64, or NULL (not
 * formed); P = 3 n_atom, perturbation x = 3 A + alpha.  The bracketed terms
 * are present only when weight derivatives w_x are passed. */
typedef struct {
    double *hess;        /* [P][P] E_{G,G} + E_{G,gr} + E_{G,gr}^T + E_{gr,gr}
                            [+ E_{w,w} (its second sum) + E_{G,w} + E_{G,w}^T
                             + E_{w,gr} + E_{w,gr}^T], symmetrised */
    double *grad;        /* [P] nuclear gradient E_G + E_gr [+ E_w] (Section II.A) */
    double *resp_rho;    /* [P][N] sum_j w_j (f^{rho rho}_ij rho^x_j + f^{rho gamma}_ij gamma^x_j) */
    double *resp_gamma;  /* [P][N] sum_j w_j (f^{gamma rho}_ij rho^x_j + f^{gamma gamma}_ij gamma^x_j) */
    double *fock_rho;    /* [P][N] resp_rho + E^{Agr}_i + rho_i (kappa_r U^{Agr}_i + omega_r W^{Agr}_i)
                            [+ E^{Aw}_i + rho_i (kappa_r U^{Aw}_i + omega_r W^{Aw}_i)] */
    double *fock_gamma;  /* [P][N] resp_gamma + rho_i omega_g W^{Agr}_i [+ rho_i omega_g W^{Aw}_i] */
    double *w_coef;      /* [N] rho_i (beta + E_i): the coefficient of w^A_i in E^A_w and of
                            w^{AB}_i in the first sum of E^{AB}_{w,w}, which the caller forms
                            from its weights' second derivatives */
    double *energy;      /* [1] the VV10 energy (Section II.A), from the same pair pass */
    double *f_rho;       /* [N] potential f^rho_i, as vv10_energy_potential */
    double *f_gamma;     /* [N] potential f^gamma_i */
} vv10_nuclear_outputs;

/*
 * vv10_nuclear_terms -- every nuclear-perturbation output of one pass over
 * the pairs (Section II.B): the Hessian terms (below), the gradient, the
 * response rows, and the grid-level coefficients of the Fock nuclear
 * derivative F^A_{mu nu} = F^A_G + F^A_w + F^A_gr: fock_rho multiplies
 * w_i phi_mu phi_nu and fock_gamma multiplies 2 w_i grad rho . grad(phi_mu phi_nu)
 * in the second line of F^A_G, in F^A_gr and in the second and third lines
 * of F^A_w; the first lines of F^A_G and F^A_w (f^rho, f^gamma times
 * basis-function or weight derivatives) belong to the caller.
 * fock_rho/fock_gamma equal the derivative of the potential f^rho, f^gamma
 * when nucleus A moves with its grid points (and, with w_x, its weights).
 * energy, f_rho and f_gamma come from the pair integrals that the grid-term
 * pass forms anyway, so one call gives energy, potential and Hessian with a
 * single pass over the pairs (vv10_energy_potential first would add its own).
 * Outputs set to NULL are not formed (no output: no work).
 *  n_pert, rho_x, grad_rho_x as for vv10_hessian_terms.
 *  w_x   [n_pert][N] DEVICE, or NULL for weights that do not depend on the
 *        nuclear positions: w^x_i = dw_i/dX_x with grid points moving with
 *        their owner atoms (Section II.A, w^A_i; Becke-partitioned weights,
 *        for example).  The entries of the owner atom (x/3 == atom_of[i]) are
 *        not read: the library takes them from translational invariance,
 *        w^{(O(i),b)}_i = -sum_{B != O(i)} w^{(B,b)}_i.  With w_x the Hessian
 *        adds the weight terms of the nine-term split except
 *        sum_i w^{AB}_i rho_i (beta + E_i), which needs the weights' second
 *        derivatives (w_coef is its coefficient).  The first call with w_x
 *        adds a weight workspace of about (5 + 3 jsplit) N P doubles.
 *  out   non-NULL.
 * Errors: VV10_E_ARG, VV10_E_OOM (workspace), VV10_E_STATE, VV10_E_HIP.
 */
vv10_status vv10_nuclear_terms(vv10_plan *plan, int32_t n_pert, const double *rho_x,
                               const double *grad_rho_x, const double *w_x,
                               const vv10_nuclear_outputs *out);

/*
 * vv10_hessian_terms -- nuclear-Hessian grid terms for all 3 n_atom
 * perturbations at once (Section II.B, nine-term split with the weight
 * terms zero):
 *   hess = E_{G,G} + E_{G,gr} + E_{G,gr}^T + E_{gr,gr}
 * where E_{G,G} excludes sum_i w_i (f^rho_i rho^{AB}_i + f^gamma_i gamma^{AB}_i)
 * (that term needs second density derivatives, which belong to the caller).
 *
 *  n_pert      must equal 3 n_atom; perturbation x = 3 A + alpha moves
 *              nucleus A along axis alpha.
 *  rho_x       [n_pert][N] total derivative of rho at each point when the
 *              nucleus moves and the point moves with its owner atom.
 *  grad_rho_x  [n_pert][N][3] the same for grad rho; gamma^x = 2 grad rho . grad rho^x.
 *  hess        [n_pert][n_pert] output, symmetrised as (H + H^T)/2.
 *  grad        [n_pert] or NULL: nuclear gradient E_G + E_gr (Section II.A).
 *  resp_rho    [n_pert][N] or NULL: sum_j w_j (f^{rho rho}_ij rho^x_j + f^{rho gamma}_ij gamma^x_j).
 *  resp_gamma  [n_pert][N] or NULL: sum_j w_j (f^{gamma rho}_ij rho^x_j + f^{gamma gamma}_ij gamma^x_j).
 * (vv10_nuclear_terms with these outputs.)
 * Errors: VV10_E_ARG, VV10_E_OOM (workspace), VV10_E_STATE, VV10_E_HIP.
 */
vv10_status vv10_hessian_terms(vv10_plan *plan, int32_t n_pert, const double *rho_x,
                               const double *grad_rho_x, double *hess, double *grad,
                               double *resp_rho, double *resp_gamma);

/*
 * vv10_gradient -- VV10 nuclear gradient alone (Section II.A):
 *   grad[x] = E^x_G + E^x_gr [+ E^x_w],
 *   E^x_G  = sum_i w_i (f^rho_i rho^x_i + f^gamma_i gamma^x_i),  gamma^x = 2 grad rho . grad rho^x,
 *   E^A_gr = sum_{i in A} w_i rho_i E^{Agr}_i = -sum_{B != A} sum_{i in A} w_i rho_i E^{Bgr}_i,
 *   E^x_w  = sum_i w^x_i rho_i (beta + E_i)   (only with w_x).
 * Costs one pass over the pairs for E, U, W and the E^{Bgr} sums, without
 * the Hessian contraction; the same value as the grad output of
 * vv10_nuclear_terms.
 *  n_pert      must equal 3 n_atom.
 *  rho_x       [n_pert][N] DEVICE, FP64 (as for vv10_hessian_terms).
 *  grad_rho_x  [n_pert][N][3] DEVICE, FP64.
 *  w_x         [n_pert][N] DEVICE, FP64, or NULL: weight derivatives as for
 *              vv10_nuclear_terms (owner-atom entries not read).
 *  grad        [n_pert] DEVICE, FP64 output.
 * Errors: VV10_E_ARG, VV10_E_OOM, VV10_E_STATE, VV10_E_HIP.
 */
vv10_status vv10_gradient(vv10_plan *plan, int32_t n_pert, const double *rho_x,
                          const double *grad_rho_x, const double *w_x, double *grad);

/*
 * vv10_energy_potential_noalloc -- for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): vv10_prepare + vv10_energy_potential + vv10_destroy as
 * one call that allocates nothing and never synchronises.  Same inputs as
 * vv10_prepare, same outputs as vv10_energy_potential (bitwise: the same
 * kernels and launch shapes run).
 *
 * Its working memory (packed point data, per-point fields, pair integrals,
 * reduction scratch, validation flag) is one library-owned device array of
 * VV10_NOALLOC_SCRATCH_BYTES on each device the call runs on, held until the
 * process ends.  Grids that need more (vv10_noalloc_bytes) are rejected with
 * VV10_E_ARG before any work; the limit is about 250000 points.  All calls on
 * one device share that array: calls that overlap in time on one device
 * (several streams, several host threads) race and must be ordered by the
 * caller.  The first call on a device resolves the array's address (a HIP
 * symbol query, not an allocation).
 *
 *  params, n_grid, n_atom, coords, weights, atom_of, rho, grad_rho, prec,
 *  stream     as vv10_prepare (DEVICE inputs; the call is asynchronous on
 *             `stream`).
 *  energy     [1] DEVICE output (required); f_rho, f_gamma [N] DEVICE or NULL.
 *  status     [1] DEVICE int32 or NULL: receives VV10_OK, or the status
 *             vv10_prepare would return for invalid inputs (VV10_E_DENSITY,
 *             VV10_E_GRID_ORDER, VV10_E_ARG), in which case nothing was
 *             written to energy, f_rho, f_gamma.
 * Errors (returned): VV10_E_ARG (null pointer, bad size or parameters, grid
 * larger than the scratch), VV10_E_HIP (launch or symbol query failed).
 */
#define VV10_NOALLOC_SCRATCH_BYTES (64u << 20)
vv10_status vv10_energy_potential_noalloc(const vv10_params *params, int64_t n_grid,
                                          int32_t n_atom, const double *coords,
                                          const double *weights, const int32_t *atom_of,
                                          const double *rho, const double *grad_rho,
                                          vv10_precision prec, hipStream_t stream,
                                          double *energy, double *f_rho, double *f_gamma,
                                          int32_t *status);

/* Bytes of the scratch array vv10_energy_potential_noalloc needs for a grid
 * (at most VV10_NOALLOC_SCRATCH_BYTES is available); 0 for invalid sizes. */
size_t vv10_noalloc_bytes(int64_t n_grid, int32_t n_atom);

/* Device bytes that vv10_gradient adds to a plan (its tile sums and
 * per-group pair integrals, and the owner slots of w^x), an upper bound
 * over devices; 0 for invalid sizes. */
size_t vv10_gradient_footprint_bytes(int64_t n_grid, int32_t n_atom);

/* Largest n_t accepted by vv10_trial_response. */
#define VV10_MAX_TRIAL 65536

/*
 * vv10_trial_response -- VV10 part of the contracted orbital Hessian for
 * n_t trial densities (Section II.B, the f^{rho,t}, f^{gamma,t} equations
 * that enter G^t_{mu nu}; the same quantities drive CPSCF and TDDFT):
 *   f^{rho,t}_i   = sum_j w_j (f^{rho rho}_ij rho^t_j + 2 f^{rho gamma}_ij gamma^t_j)
 *   f^{gamma,t}_i = sum_j w_j (f^{gamma rho}_ij rho^t_j + 2 f^{gamma gamma}_ij gamma^t_j)
 * with gamma^t_j = grad rho_j . grad rho^t_j and the second-derivative
 * matrices including their delta_ij (same-point) terms; that is, the
 * derivative of the potential (f^rho, f^gamma of vv10_energy_potential)
 * along rho + t rho^t.
 *
 *  n_t         number of trial densities, 0 <= n_t <= VV10_MAX_TRIAL (0: no-op).
 *  rho_t       [n_t][N] DEVICE, FP64: trial densities on the grid.
 *  grad_rho_t  [n_t][N][3] DEVICE, FP64: their gradients.
 *  f_rho_t     [n_t][N] DEVICE, FP64 output.
 *  f_gamma_t   [n_t][N] DEVICE, FP64 output.
 * The pair integrals the same-point terms need are computed by the plan's
 * first call and kept; the workspace for n_t columns is kept and rebuilt
 * when n_t changes.  Asynchronous on the plan's stream.
 * Errors: VV10_E_ARG, VV10_E_OOM (workspace), VV10_E_STATE, VV10_E_HIP.
 */
vv10_status vv10_trial_response(vv10_plan *plan, int32_t n_t, const double *rho_t,
                                const double *grad_rho_t, double *f_rho_t, double *f_gamma_t);

/* Device bytes that vv10_trial_response adds to a plan for n_t trial
 * densities (an upper bound for automatic tiles and for tiles whose j-split
 * count is at most twice the automatic one); 0 for invalid sizes. */
size_t vv10_response_footprint_bytes(int64_t n_grid, int32_t n_t, vv10_precision prec);

/* Stages of the library's launch sequence, for vv10_stage_times. */
typedef enum {
    VV10_STAGE_PAIR = 0,      /* pair integrals E, U, W of vv10_energy_potential */
    VV10_STAGE_POTENTIAL = 1, /* f^rho, f^gamma and the energy reduction */
    VV10_STAGE_PERT_PREP = 2, /* packing of the perturbation channels */
    VV10_STAGE_CONTRACT = 3,  /* perturbation-batched contraction (MFMA) */
    VV10_STAGE_GRID = 4,      /* grid-position intermediates fused with the pair
                                 integrals E, U, W, A, B, C of vv10_hessian_terms */
    VV10_STAGE_ASSEMBLE = 5,  /* Hessian assembly (and gradient) */
    VV10_STAGE_WEIGHTS = 6,   /* weight-derivative packing and contraction */
    VV10_NUM_STAGES = 7
} vv10_stage;

/* Rebind the plan to another HIP stream: later calls enqueue on `stream`.
 * The caller orders the new stream after the plan's earlier work (for
 * example with an event); the plan must not have calls in flight on two
 * streams at once.  Errors: VV10_E_STATE (NULL plan). */
vv10_status vv10_set_stream(vv10_plan *plan, hipStream_t stream);

/* Enable (1) or disable (0) per-stage timing: while enabled, every call
 * records a HIP event pair on the plan's stream around each stage it runs.
 * The events come from a per-device pool; vv10_destroy returns them.
 * Errors: VV10_E_STATE (NULL plan), VV10_E_HIP (event creation failed). */
vv10_status vv10_set_timing(vv10_plan *plan, int32_t enable);

/* Per-stage timing for the chosen stages only: bit k of mask (1 << k, k a
 * vv10_stage) brackets stage k with the event pair above; 0 disables timing
 * (vv10_set_timing(plan, 1) equals the mask of every stage).  Each timed
 * stage adds two event records to the stream, so timing only the stages
 * that are read disturbs the launch sequence least.
 * Errors: VV10_E_STATE (NULL plan), VV10_E_ARG (bits beyond the stages),
 * VV10_E_HIP (event creation failed). */
vv10_status vv10_set_timing_stages(vv10_plan *plan, uint32_t mask);

/* Device time in milliseconds of each stage's most recent timed run, from
 * the events above; ms has VV10_NUM_STAGES entries (HOST memory), stages
 * never timed report 0.  Waits for the recorded events to complete.
 * Errors: VV10_E_STATE (NULL plan or timing never enabled), VV10_E_ARG
 * (ms NULL), VV10_E_HIP. */
vv10_status vv10_stage_times(vv10_plan *plan, double *ms);

/* Tile-shape overrides for a plan (0 = the library's automatic choice):
 *  jsplit   number of j splits of the perturbation contraction;
 *  bgroups  number of atom groups the grid-term pass splits its sums into.
 * Set before the plan's first vv10_hessian_terms (the workspace is sized by
 * them); values are clamped to the valid range.  Used by the autotuner.
 * Errors: VV10_E_STATE (NULL plan, or workspace already built), VV10_E_ARG. */
typedef struct {
    int32_t jsplit;
    int32_t bgroups;
} vv10_tiles;
vv10_status vv10_set_tiles(vv10_plan *plan, const vv10_tiles *tiles);

/* The tile shape a plan uses (after the overrides and clamping); builds the
 * workspace if it does not exist yet.  tiles is HOST memory.
 * Errors: VV10_E_STATE (NULL plan), VV10_E_ARG (tiles NULL), VV10_E_OOM. */
vv10_status vv10_get_tiles(vv10_plan *plan, vv10_tiles *tiles);

/*
 * vv10_set_screening -- grid screening of the perturbation contraction
 * (Section II.B, last paragraph: sums over a batch of j are skipped where the
 * perturbed densities are below a precision threshold; the paper gives no
 * threshold).  With tau > 0, later vv10_nuclear_terms, vv10_hessian_terms
 * and vv10_trial_response calls on this plan skip the MFMA work of every
 * (16-point j block, 16-column block) whose channels all satisfy
 *   max_{j in block} max(|p^x_j|, |q^x_j|) <= tau * max_j max(|p^x_j|, |q^x_j|)
 * for each column x of the block (p = w rho^x, q = w rho (omega_r rho^x +
 * omega_g gamma^x), the contraction's two channels).  The skipped terms are
 * dropped: each is below tau of its column's largest block, and their sum
 * over a row changes the contraction's outputs by a few tens of tau relative
 * to the column's largest (4e-7 at tau = 1e-8 on a 5400-point water
 * hexamer); tau = 0 (the default) computes every block and gives bitwise the
 * unscreened results.  The saving is largest when the points of
 * each atom are stored in radial-shell order.  Batches (vv10_batch_*) do not
 * screen.  Adds (N/16) P bytes plus (N/16 + 1) P floats per workspace.
 * Errors: VV10_E_STATE (NULL plan), VV10_E_ARG (tau negative or not finite).
 */
vv10_status vv10_set_screening(vv10_plan *plan, double tau);

/* Active and total (16-point, 16-column) blocks of the plan's most recent
 * screened contraction (waits for the plan's stream).  active, total HOST.
 * Errors: VV10_E_STATE (NULL plan or no screened contraction yet),
 * VV10_E_ARG (NULL outputs), VV10_E_HIP. */
vv10_status vv10_screening_stats(vv10_plan *plan, int64_t *active, int64_t *total);

/* ------------------------------------------------------------------------ */
/* Batches: many molecules (grids) of uneven size evaluated together.        */
/* ------------------------------------------------------------------------ */
typedef struct vv10_batch vv10_batch;

/*
 * vv10_batch_create -- prepare n_mol grids stored back to back.
 *  grid_off  HOST [n_mol + 1], nondecreasing, grid_off[0] = 0: molecule m owns
 *            points [grid_off[m], grid_off[m+1]) of coords, weights, atom_of,
 *            rho and grad_rho (each laid out as for vv10_prepare).
 *  atom_off  HOST [n_mol + 1]: molecule m has atom_off[m+1] - atom_off[m] >= 1
 *            atoms; atom_of holds molecule-local atom indices.
 *  tiles     HOST [n_mol] tile overrides, or NULL for automatic choices.
 * Validates every molecule as vv10_prepare does (one stream synchronisation
 * per molecule) and allocates every workspace.  Errors as vv10_prepare.
 */
vv10_status vv10_batch_create(const vv10_params *params, int32_t n_mol, const int64_t *grid_off,
                              const int32_t *atom_off, const double *coords,
                              const double *weights, const int32_t *atom_of, const double *rho,
                              const double *grad_rho, vv10_precision prec,
                              const vv10_tiles *tiles, hipStream_t stream, vv10_batch **out);

/*
 * vv10_batch_run -- energies and Hessian terms of every molecule.
 *  rho_x       molecule m's [3 n_atom_m][N_m] block, blocks back to back.
 *  grad_rho_x  molecule m's [3 n_atom_m][N_m][3] block, blocks back to back.
 *  energy      [n_mol] VV10 energies.
 *  hess        molecule m's [3 n_atom_m][3 n_atom_m] block, blocks back to back.
 * The whole evaluation is one HIP graph: the perturbation packing of every
 * molecule; then persistent kernels, each pulling the items of all
 * molecules from a list of its own, largest first: in split-BF16 an
 * eight-wave kernel over the contraction items (molecule, tile, column
 * group, j split) of the molecules with eight or more 16-column blocks per
 * column group (the standalone contraction's form for them), a four-wave
 * kernel over the other contraction items, and a kernel over the grid-pass
 * items (molecule, grid tile, atom group); then each molecule's
 * pair-integral sums, energy and assembly as independent branches.
 * The graph is captured on the first call and replayed while the four
 * pointers stay the same.  Asynchronous on the batch's stream.
 * Each molecule's results equal those of vv10_hessian_terms on the same
 * grid with the same tiles (same kernels, same reduction order).
 * Errors: VV10_E_ARG, VV10_E_STATE, VV10_E_HIP.
 */
vv10_status vv10_batch_run(vv10_batch *batch, const double *rho_x, const double *grad_rho_x,
                           double *energy, double *hess);

/* Work items of the batch (contraction and grid-pass items of all its
 * persistent kernels) and workgroups of its four-wave contraction kernel. */
vv10_status vv10_batch_info(const vv10_batch *batch, int64_t *n_items, int32_t *n_workgroups);

/* Destroy a batch (waits for its stream); NULL is accepted. */
void vv10_batch_destroy(vv10_batch *batch);

/* Device bytes a plan for this size holds once vv10_hessian_terms has run
 * (an upper bound for automatic tiles and for tiles whose j-split count is at
 * most twice the automatic one, as the autotuner's are; the contraction
 * partials are FP64, one [N][2][P] block per j split; vv10_energy_potential
 * alone needs less). */
size_t vv10_footprint_bytes(int64_t n_grid, int32_t n_atom, vv10_precision prec);

/* Destroy a plan (NULL is accepted).  Waits for the plan's stream to finish
 * the plan's work, then returns its device memory to the library's
 * per-device cache, from which later plans of similar sizes are served. */
void vv10_destroy(vv10_plan *plan);

/* Bytes of device memory held in the library's cache (freed plans' blocks
 * kept for reuse), summed over devices. */
size_t vv10_cached_bytes(void);

/* Return every cached block to the HIP runtime (hipFree).  Blocks still
 * owned by live plans are not affected.  Call with no library work in flight. */
void vv10_release_cached(void);

/* Static description of a status code. */
const char *vv10_status_string(vv10_status s);

/* Library build identifier (compile-time arch and version string). */
const char *vv10_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VV10_H */
