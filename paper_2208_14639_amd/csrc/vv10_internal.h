// Internal declarations of the VV10 HIP library: the plan, its device
// layout and the kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/vv10.h"

namespace vv10 {

// Rows of the per-point FP64 table F[NF][npad] (structure of arrays).
enum Field {
    F_W = 0,     // quadrature weight
    F_RHO,       // density
    F_GX, F_GY, F_GZ,  // density gradient
    F_OMR,       // d omega / d rho
    F_OMG,       // d omega / d gamma
    F_KAR,       // d kappa / d rho
    F_OMRR,      // d2 omega / d rho2
    F_OMRG,      // d2 omega / d rho d gamma
    F_OMGG,      // d2 omega / d gamma2
    F_KARR,      // d2 kappa / d rho2
    F_FR,        // potential f^rho (filled by the pair-integral finalisation)
    F_FG,        // potential f^gamma
    F_F0,        // rho (beta + E): coefficient of the weight derivatives
    NF
};

// Rows of the pair-integral table I[6][npad].
enum Integral { I_E = 0, I_U, I_W, I_A, I_B, I_C, NI };

constexpr int kPad = 256;        // npad is a multiple of this
constexpr int kGridTile = 64;    // i points per grid-term tile (one wave)
// The mixed contractions sum at most kFp32Run consecutive j points of a tile
// in FP32 (the MFMA accumulators) and then add those sums into the tile's
// rows of the split's FP64 partials: FP32 within a tile, FP64 across tiles.
// Each addition after the first re-reads the rows (about 32 N^2 P / kFp32Run
// bytes over a contraction), which sets the length.
constexpr int kFp32Run = 8192;

struct Workspace {
    int32_t P = 0, Pp = 0;       // perturbations and padded column count
    int32_t ncb = 0, ngroups = 0;  // 16-column blocks per contraction group, groups
    int32_t jsplit = 1;          // j splits of the contraction
    int64_t jlen = 0;            // j points per split (multiple of 32)
    int32_t gsplit = 1;          // point slices of the assembly GEMM
    int32_t bgroups = 1;         // atom groups of the grid-term kernel
    void *X = nullptr;           // (p, q) channels: FP64 or FP32 [npad][2][Pp];
                                 // BF16X3: hi then lo, each [npad/16][Pp][32] bf16
    double *L = nullptr;         // [npad][2][Pp] (rho^x, gamma^x)
    void *Ypart = nullptr;       // [jsplit][npad][2][Pp] contraction partials (FP64; Y itself with one split)
    double *Y = nullptr;         // [npad][2][Pp] summed contraction, then R in place
    double *Z = nullptr;         // [npad][2][Pp] grid-position channels
    double *Dpart = nullptr;     // [ntiles][n_atom][9] tile sums of a_i D^B_i (6) and a_i E^{Bgr}_i (3)
    double *Igrp = nullptr;      // [bgroups][6][npad] pair integrals per atom group
    double *Hpart = nullptr;     // [gsplit][Pp + 1][Pp] GEMM slices; row Pp: gradient
    double *Hsum = nullptr;      // [Pp + 1][Pp] the slices summed
    double *DS = nullptr;        // [n_atom][n_atom][9] Dpart summed over each atom's tiles
    // screening of the contraction (allocated when the plan screens)
    float *bmax = nullptr;       // [npad/16][Pp] block maxima of max(|p|, |q|)
    float *colmax = nullptr;     // [Pp] column maxima
    uint32_t *mask = nullptr;    // [npad/16][ngroups] bit cb: (16-point, 16-column) block active
    int32_t *screen_count = nullptr;  // number of active blocks of the last screened contraction
    bool screened = false;       // the last contraction used the mask
    size_t bytes = 0;
};

// Buffers of the gradient-only pass (vv10_gradient).
struct GradWork {
    int32_t bgroups = 0;
    double *Gpart = nullptr;     // [ntiles][n_atom][3] tile sums of a_i E^{Bgr}_i
    double *Igrp = nullptr;      // [bgroups][3][npad] E, U, W per atom group
};

// Buffers of the weight-derivative terms (allocated by the first call with
// weight derivatives).
struct WeightWork {
    int32_t ncb = 0, groups = 0; // 16-column blocks per weight-contraction group, groups
    double *Wown = nullptr;      // [npad][3] owner-atom slot of w^x
    void *Xv = nullptr;          // v = w^x rho: FP64/FP32 [npad][Pp]; BF16X3 hi, lo [npad/32][Pp][32]
    double *Lw = nullptr;        // [npad][Pp] w^x with the owner slot filled
    void *Ypart = nullptr;       // [jsplit][npad][3][Pp] (Y_pv, Y_qv, Y_vv) partials, FP64
    double *Ze = nullptr;        // [npad][Pp] E^{Bgr}_i (grid pass)
    double *Rw = nullptr;        // [npad][Pp] right factor of the w^x rows of the GEMM
    double *Hpart = nullptr;     // [gsplit][Pp + 1][Pp] GEMM slices of the w^x rows
    size_t bytes = 0;
};

}  // namespace vv10

struct vv10_plan {
    vv10_params prm{};
    double beta = 0.0;
    int64_t n = 0, npad = 0;
    int32_t n_atom = 0;
    vv10_precision prec = VV10_FP64;
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cu = 256;
    bool failed = false;
    // pair integrals held in I: 0 none, 3 (E, U, W), 6 (E..C).  Each is
    // formed once, by the first call that needs it, and never overwritten
    // (the inputs never change), so later calls do not depend on which
    // call formed them.
    int ints_level = 0;

    std::vector<int64_t> seg;       // host: atom segments, seg[A]..seg[A+1]
    std::vector<int32_t> tile_i0, tile_n, tile_atom, tile_first;  // grid-term tiles
    int32_t ntiles = 0;

    // device memory owned by the plan
    double4 *P0 = nullptr;   // [npad] (x, y, z, omega), coordinates shifted by the grid centroid
    double4 *P1 = nullptr;   // [npad] (kappa, a = w rho, c = rho dkappa/drho, 0)
    float4 *P0f = nullptr;   // FP32 copies for the mixed modes
    float4 *P1f = nullptr;
    double *F = nullptr;     // [NF][npad]
    double *I = nullptr;     // [6][npad]
    double *Ipart = nullptr; // [pair_splits][6][npad] partial pair integrals
    int32_t *atom_of = nullptr;   // [npad], padding rows hold n_atom
    // grid metadata, one device block (d_meta) holding the views below
    char *d_meta = nullptr;
    std::vector<char> h_meta;     // host image of d_meta (lives as long as the plan)
    int64_t *d_seg = nullptr;     // [n_atom + 1]
    int32_t *d_tile_i0 = nullptr, *d_tile_n = nullptr, *d_tile_atom = nullptr, *d_tile_first = nullptr;
    double *red = nullptr;   // reduction scratch
    int32_t *flag = nullptr; // [1 + n_atom + 1] validation flag and segment starts
    size_t base_bytes = 0;

    // tile overrides (vv10_set_tiles); 0 = automatic
    int32_t tiles_jsplit = 0, tiles_bgroups = 0;

    // screening threshold of the contraction (vv10_set_screening); 0 = off
    double screen_tau = 0.0;

    // per-stage timing (vv10_set_timing, vv10_set_timing_stages): bit k
    // set = stage k is bracketed by events
    uint32_t timing = 0;
    hipEvent_t ev[2 * VV10_NUM_STAGES] = {};
    bool ran[VV10_NUM_STAGES] = {};

    vv10::Workspace ws;

    // trial-density response (vv10_trial_response): a workspace for its n_t
    // columns (X, L, partials only) and the Hessian-mode pair integrals
    // E..C, computed by its first call and kept
    vv10::Workspace rws;
    double *Ir = nullptr;    // [6][npad]
    bool ir_ready = false;

    // gradient-only pass (vv10_gradient)
    vv10::GradWork gw;

    // weight-derivative terms (vv10_nuclear_terms / vv10_gradient with w_x)
    vv10::WeightWork ww;
    double *wown = nullptr;  // [npad][3] owner slot of w^x for the gradient-only pass
};

namespace vv10 {

// Operands of one molecule of a batch (device copy): the contraction's and
// the grid pass's (grid-position intermediates with the pair integrals).
struct BatchMol {
    int64_t npad, jlen;
    int32_t Pp, ncb;
    const void *P0, *P1;   // double4 (FP64) or float4 (mixed) point data
    const void *X;         // (p, q) channels in the plan's layout
    void *Ypart;           // [jsplit][npad][2][Pp] partial outputs
    int32_t n_atom, bgroups, ntiles, pad0;
    const int64_t *seg;    // [n_atom + 1] atom segments
    const int32_t *tile_i0, *tile_n, *tile_atom;   // grid-pass tiles
    const double4 *Pd;     // FP64 point data (the self pair)
    double *Z, *Dpart, *Igrp;   // grid-pass outputs, as the plan's workspace holds them
};
// One unit of work of a persistent kernel: with split >= 0 a contraction
// item (molecule, column group grp, j split, i tile itile of 16 W points,
// where W = persistent_waves(prec), or 8 for the wide kernel); with
// split = -1 a grid item (molecule, atom group grp, grid-pass tile itile).
struct BatchItem {
    int32_t mol, grp, split, itile;
};
int persistent_waves(vv10_precision prec);
int persistent_blocks_per_cu(vv10_precision prec);
hipError_t launch_contract_persistent(vv10_precision prec, const BatchMol *mols,
                                      const BatchItem *items, int32_t n_items, int32_t *counter,
                                      int n_blocks, hipStream_t stream);
// Split-BF16 molecules with at least kWideMinNcb column blocks per group run
// their contraction items in a second persistent kernel of eight waves
// (i tiles of 128 points), the standalone kernel's form for these counts.
constexpr int kWideMinNcb = 8;
// The grid items (one grid tile of one molecule and atom group each) run in
// a persistent kernel of their own, one wave per workgroup.
int persistent_grid_blocks_per_cu(vv10_precision prec);
hipError_t launch_grid_persistent(vv10_precision prec, const BatchMol *mols,
                                  const BatchItem *items, int32_t n_items, int32_t *counter,
                                  int n_blocks, hipStream_t stream);
int persistent_wide_blocks_per_cu();
hipError_t launch_contract_persistent_wide(const BatchMol *mols, const BatchItem *items,
                                           int32_t n_items, int32_t *counter, int n_blocks,
                                           hipStream_t stream);

// Device allocations of the library (per-device caching allocator).
hipError_t dev_alloc(void **ptr, size_t bytes);
void dev_free(void *ptr);
size_t dev_cached_bytes();
void dev_release_cached();

// j splits of the pair-integral kernel for a padded grid size.
int pair_splits(int64_t npad);
// Doubles of a plan's reduction scratch (centroid partials, energy partials).
size_t reduction_doubles(int64_t npad);

// Kernel launchers (each enqueues on plan->stream and returns hipGetLastError()).
hipError_t launch_prepare(vv10_plan *p, const double *coords, const double *w,
                          const int32_t *atom_of, const double *rho,
                          const double *grad_rho);
hipError_t launch_pair_integrals(vv10_plan *p, bool hessian_mode, double *I_out);
// valid (device, or null): when *valid != 0 (a failed input validation)
// nothing is written to energy, f_rho, f_gamma.
hipError_t launch_potential(vv10_plan *p, double *energy, double *f_rho, double *f_gamma,
                            const int32_t *valid = nullptr);
// screen: also the block maxima and the contraction mask (ws.bmax etc. allocated).
hipError_t launch_pert_prep(vv10_plan *p, const Workspace &ws, const double *rho_x,
                            const double *grad_rho_x, bool screen = false);
// screen: skip the (16-point, 16-column) blocks that ws.mask marks inactive.
hipError_t launch_contract(vv10_plan *p, const Workspace &ws, bool screen = false);
// ints_from: the pair integrals I[k] for ints_from <= k < 6 are formed in the
// same pass and written to p->I (0: all six; 6: none, the plan holds them).
hipError_t launch_grid_terms(vv10_plan *p, double *Ze, int ints_from = 0);
// The second half of launch_grid_terms: I[k] for ints_from <= k < 6 from the
// per-group partials the grid pass left in ws.Igrp.
hipError_t launch_sum_groups(vv10_plan *p, int ints_from = 0);
// ints: also E, U, W into p->I (else the plan holds them).
hipError_t launch_grid_grad(vv10_plan *p, bool ints = true);
hipError_t launch_gradient(vv10_plan *p, const double *rho_x, const double *grad_rho_x,
                           const double *w_x, double *grad);
// Weight-derivative terms: owner slots, packing, contraction.
void weight_shape(int32_t Pp, vv10_precision prec, WeightWork &ww);
hipError_t launch_weight_own(vv10_plan *p, const double *w_x, double *Wown);
hipError_t launch_weight_prep(vv10_plan *p, const double *w_x);
hipError_t launch_weight_contract(vv10_plan *p);
// The fused split-BF16 contraction (main and weight rows in one pass over the
// pairs) applies when the columns form one group of at most four blocks.
bool fused_weighted_contract(const vv10_plan *p, const Workspace &ws);
hipError_t launch_contract_weighted(vv10_plan *p, const Workspace &ws, const WeightWork &ww);
hipError_t launch_trial_response(vv10_plan *p, double *f_rho_t, double *f_gamma_t);
// weighted: also the weight-derivative terms (p->ww filled by the weight stages)
hipError_t launch_assemble(vv10_plan *p, const vv10_nuclear_outputs &out, bool weighted);

// Layout decisions shared by the host code.
// n_cols: contraction columns (0 = the 3 n_atom nuclear perturbations).
void plan_workspace_shape(int64_t npad, int32_t n_atom, int32_t ntiles, int num_cu,
                          vv10_precision prec, Workspace &ws, int32_t jsplit_override = 0,
                          int32_t bgroups_override = 0, int32_t n_cols = 0);
// Bytes of the trial-response workspace (X, L and partials for n_t columns)
// plus its pair-integral table.
size_t response_bytes(int64_t npad, vv10_precision prec, const Workspace &ws);
// Allocate the Hessian workspace of a plan (no-op when it exists).
vv10_status ensure_workspace(vv10_plan *p);
size_t workspace_bytes(int64_t npad, int32_t n_atom, int32_t ntiles, vv10_precision prec,
                       const Workspace &ws);
// Resident workgroups per CU of the contraction kernel for this shape (0 if unknown).
int contract_blocks_per_cu(vv10_precision prec, int ncb);
// Max 16-column blocks per contraction workgroup.
inline int max_ncb(vv10_precision prec) { return prec == VV10_FP64 ? 8 : 12; }
// Max 16-column blocks per weight-contraction workgroup (three outputs).
inline int max_wncb(vv10_precision prec) { return prec == VV10_FP64 ? 4 : 8; }
// Bytes of one element of the contraction partials: FP64 in every mode (the
// mixed modes add their FP32 tile sums into them).
inline size_t partial_elem(vv10_precision) { return sizeof(double); }

}  // namespace vv10
