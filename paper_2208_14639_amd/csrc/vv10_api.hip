// Host side of the C ABI declared in include/vv10.h: argument validation,
// plan and workspace ownership, launch sequencing and error mapping.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "vv10_internal.h"

using vv10::Workspace;

namespace vv10 {

void plan_workspace_shape(int64_t npad, int32_t n_atom, int32_t ntiles, int num_cu,
                          vv10_precision prec, Workspace &ws, int32_t jsplit_override,
                          int32_t bgroups_override, int32_t n_cols) {
    ws.P = n_cols > 0 ? n_cols : 3 * n_atom;
    const int ncb_total = (ws.P + 15) / 16;
    const int cap = max_ncb(prec);
    ws.ngroups = (ncb_total + cap - 1) / cap;
    ws.ncb = (ncb_total + ws.ngroups - 1) / ws.ngroups;
    ws.Pp = 16 * ws.ncb * ws.ngroups;

    // j splits of the contraction: fill the last round of resident
    // workgroups (every mode keeps FP64 partials per split; the mixed modes
    // sum at most kFp32Run points in FP32 before adding into them, so a
    // split may be as long as the grid).
    int per_cu = contract_blocks_per_cu(prec, ws.ncb);
    if (per_cu <= 0) per_cu = 2;
    const int64_t units = (npad / 64) * ws.ngroups;
    const int64_t slots = (int64_t)per_cu * num_cu;
    const int min_split = 1;
    double best = -1.0;
    ws.jsplit = min_split;
    for (int S = min_split; S <= min_split + 15; ++S) {
        if (S > 1 && npad / S < 256) break;
        const int64_t u = units * S;
        const double eff = (double)u / (double)(((u + slots - 1) / slots) * slots);
        const double score = eff - 0.01 * (S - min_split);
        if (score > best + 1e-12) {
            best = score;
            ws.jsplit = S;
        }
    }
    if (jsplit_override > 0) {
        const int max_split = (int)std::max<int64_t>(1, npad / 256);
        ws.jsplit = std::max(min_split, std::min(jsplit_override, max_split));
    }
    ws.jlen = ((npad / ws.jsplit + 31) / 32) * 32;
    while ((ws.jsplit - 1) * ws.jlen >= npad) --ws.jsplit;   // no empty split
    // assembly GEMM: about one workgroup per CU over (64 x 64 tiles) x slices
    const int tiles = (ws.Pp + 63) / 64;
    ws.gsplit = (int)std::max<int64_t>(1, std::min<int64_t>((num_cu + tiles * tiles - 1) / (tiles * tiles),
                                                             std::max<int64_t>(1, npad / 64)));
    ws.bgroups = std::max(1, std::min<int>(n_atom, (8192 + std::max(ntiles, 1) - 1) / std::max(ntiles, 1)));
    if (bgroups_override > 0) ws.bgroups = std::min<int>(n_atom, bgroups_override);
}

size_t workspace_bytes(int64_t npad, int32_t n_atom, int32_t ntiles, vv10_precision prec,
                       const Workspace &ws) {
    const size_t ch = (size_t)npad * 2 * ws.Pp;
    size_t b = 3 * ch * sizeof(double);                       // L, Y, Z
    b += ch * (prec == VV10_FP64 ? 8 : 4);                    // X (FP64, FP32, or BF16 hi + lo)
    const bool alias = ws.jsplit == 1;   // partials written straight into Y
    if (!alias) b += (size_t)ws.jsplit * ch * partial_elem(prec);
    b += (size_t)ntiles * n_atom * 9 * sizeof(double);
    b += (size_t)ws.bgroups * NI * npad * sizeof(double);
    b += (size_t)(ws.gsplit + 1) * (ws.Pp + 1) * ws.Pp * sizeof(double);
    b += (size_t)n_atom * n_atom * 9 * sizeof(double);
    return b;
}

size_t reduction_doubles(int64_t npad) {
    // the coordinate partial sums of 64 blocks and the centroid, or the
    // energy's block partials and the energy
    return std::max<size_t>((size_t)(npad / 256) + 2, 3 * 64 + 3);
}

size_t response_bytes(int64_t npad, vv10_precision prec, const Workspace &ws) {
    const size_t ch = (size_t)npad * 2 * ws.Pp;
    size_t b = ch * sizeof(double);                           // L
    b += ch * (prec == VV10_FP64 ? 8 : 4);                    // X
    b += (size_t)ws.jsplit * ch * partial_elem(prec);         // partials
    b += (size_t)NI * npad * sizeof(double);                  // pair integrals
    return b;
}

}  // namespace vv10

namespace {


size_t base_bytes(int64_t npad, int32_t n_atom, int64_t ntiles_bound) {
    size_t b = 2 * (size_t)npad * sizeof(double4) + 2 * (size_t)npad * sizeof(float4);
    b += (size_t)vv10::NF * npad * sizeof(double) + (size_t)vv10::NI * npad * sizeof(double);
    if (vv10::pair_splits(npad) > 1)
        b += (size_t)vv10::pair_splits(npad) * vv10::NI * npad * sizeof(double);
    b += (size_t)npad * sizeof(int32_t) + (size_t)(n_atom + 1) * sizeof(int64_t);
    b += (size_t)(3 * ntiles_bound + n_atom + 1) * sizeof(int32_t);
    b += vv10::reduction_doubles(npad) * sizeof(double) + (size_t)(n_atom + 2) * sizeof(int32_t);
    return b;
}

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return vv10::dev_alloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

void dfree(void *ptr) { vv10::dev_free(ptr); }

// Timing events are kept in a per-device pool: plans take them when timing
// is switched on and give them back when destroyed (after their stream has
// been synchronised), so short-lived timed plans create no events.
std::mutex g_ev_mutex;
std::map<int, std::vector<hipEvent_t>> g_ev_pool;

hipError_t take_event(int device, hipEvent_t *ev) {
    {
        std::lock_guard<std::mutex> lock(g_ev_mutex);
        auto &v = g_ev_pool[device];
        if (!v.empty()) {
            *ev = v.back();
            v.pop_back();
            return hipSuccess;
        }
    }
    return hipEventCreate(ev);
}

void give_event(int device, hipEvent_t ev) {
    std::lock_guard<std::mutex> lock(g_ev_mutex);
    g_ev_pool[device].push_back(ev);
}

void free_workspace(Workspace &ws) {
    dfree(ws.bmax);
    dfree(ws.colmax);
    dfree(ws.mask);
    dfree(ws.screen_count);
    dfree(ws.X);
    dfree(ws.L);
    if (ws.Ypart != ws.Y) dfree(ws.Ypart);
    dfree(ws.Y);
    dfree(ws.Z);
    dfree(ws.Dpart);
    dfree(ws.Igrp);
    dfree(ws.Hpart);
    dfree(ws.Hsum);
    dfree(ws.DS);
    ws = Workspace{};
}

void free_weight_work(vv10::WeightWork &ww) {
    dfree(ww.Wown);
    dfree(ww.Xv);
    dfree(ww.Lw);
    dfree(ww.Ypart);
    dfree(ww.Ze);
    dfree(ww.Rw);
    dfree(ww.Hpart);
    ww = vv10::WeightWork{};
}

void free_plan(vv10_plan *p) {
    if (!p) return;
    free_weight_work(p->ww);
    dfree(p->wown);
    for (auto &ev : p->ev)
        if (ev) give_event(p->device, ev);
    free_workspace(p->ws);
    free_workspace(p->rws);
    dfree(p->Ir);
    dfree(p->gw.Gpart);
    dfree(p->gw.Igrp);
    dfree(p->P0);
    dfree(p->P1);
    dfree(p->P0f);
    dfree(p->P1f);
    dfree(p->F);
    dfree(p->I);
    dfree(p->Ipart);
    dfree(p->atom_of);
    dfree(p->d_meta);
    dfree(p->red);
    dfree(p->flag);
    delete p;
}

vv10_status hip_status(hipError_t e) {
    if (e == hipSuccess) return VV10_OK;
    if (e == hipErrorOutOfMemory) return VV10_E_OOM;
    return VV10_E_HIP;
}

// Test hook: VV10_FAIL_ALLOC=<n> makes the n-th workspace allocation of the
// process report out-of-memory (used to exercise the error path on the host).
bool injected_alloc_failure() {
    static int countdown = [] {
        const char *s = std::getenv("VV10_FAIL_ALLOC");
        return s ? std::atoi(s) : 0;
    }();
    if (countdown <= 0) return false;
    return --countdown == 0;
}

}  // namespace

vv10_status vv10::ensure_workspace(vv10_plan *p) {
    if (p->ws.X) return VV10_OK;
    Workspace ws;
    vv10::plan_workspace_shape(p->npad, p->n_atom, p->ntiles, p->num_cu, p->prec, ws,
                               p->tiles_jsplit, p->tiles_bgroups);
    if (injected_alloc_failure()) return VV10_E_OOM;
    const size_t ch = (size_t)p->npad * 2 * ws.Pp;
    hipError_t e = hipSuccess;
    char *xb = nullptr, *yp = nullptr;
    if (e == hipSuccess) e = dalloc(&xb, ch * (p->prec == VV10_FP64 ? 8 : 4));
    ws.X = xb;
    if (e == hipSuccess) e = dalloc(&ws.L, ch);
    if (e == hipSuccess) e = dalloc(&ws.Y, ch);
    if (e == hipSuccess) {
        if (ws.jsplit == 1) {
            ws.Ypart = ws.Y;
        } else {
            e = dalloc(&yp, ch * ws.jsplit * vv10::partial_elem(p->prec));
            ws.Ypart = yp;
        }
    }
    if (e == hipSuccess) e = dalloc(&ws.Z, ch);
    if (e == hipSuccess) e = dalloc(&ws.Dpart, (size_t)p->ntiles * p->n_atom * 9);
    if (e == hipSuccess) e = dalloc(&ws.Igrp, (size_t)ws.bgroups * vv10::NI * p->npad);
    if (e == hipSuccess) e = dalloc(&ws.Hpart, (size_t)ws.gsplit * (ws.Pp + 1) * ws.Pp);
    if (e == hipSuccess) e = dalloc(&ws.Hsum, (size_t)(ws.Pp + 1) * ws.Pp);
    if (e == hipSuccess) e = dalloc(&ws.DS, (size_t)p->n_atom * p->n_atom * 9);
    if (e != hipSuccess) {
        free_workspace(ws);
        (void)hipGetLastError();
        return hip_status(e);
    }
    ws.bytes = vv10::workspace_bytes(p->npad, p->n_atom, p->ntiles, p->prec, ws);
    p->ws = ws;
    return VV10_OK;
}

// Allocate the trial-response workspace for n_t columns (rebuilt when n_t
// changes) and the response's pair-integral table.
static vv10_status ensure_response_workspace(vv10_plan *p, int32_t n_t) {
    if (!p->Ir) {
        if (dalloc(&p->Ir, (size_t)vv10::NI * p->npad) != hipSuccess) {
            (void)hipGetLastError();
            return VV10_E_OOM;
        }
        p->ir_ready = false;
    }
    if (p->rws.X && p->rws.P == n_t) return VV10_OK;
    free_workspace(p->rws);
    Workspace ws;
    vv10::plan_workspace_shape(p->npad, p->n_atom, p->ntiles, p->num_cu, p->prec, ws, 0, 0, n_t);
    if (injected_alloc_failure()) return VV10_E_OOM;
    const size_t ch = (size_t)p->npad * 2 * ws.Pp;
    hipError_t e = hipSuccess;
    char *xb = nullptr, *yp = nullptr;
    e = dalloc(&xb, ch * (p->prec == VV10_FP64 ? 8 : 4));
    ws.X = xb;
    if (e == hipSuccess) e = dalloc(&ws.L, ch);
    if (e == hipSuccess) e = dalloc(&yp, ch * ws.jsplit * vv10::partial_elem(p->prec));
    ws.Ypart = yp;
    if (e != hipSuccess) {
        free_workspace(ws);
        (void)hipGetLastError();
        return hip_status(e);
    }
    ws.bytes = vv10::response_bytes(p->npad, p->prec, ws);
    p->rws = ws;
    return VV10_OK;
}

// Allocate the gradient-only pass's buffers (once per plan).
static vv10_status ensure_gradient_work(vv10_plan *p) {
    if (p->gw.Gpart) return VV10_OK;
    Workspace ws;
    vv10::plan_workspace_shape(p->npad, p->n_atom, p->ntiles, p->num_cu, p->prec, ws,
                               p->tiles_jsplit, p->tiles_bgroups);
    vv10::GradWork gw;
    gw.bgroups = ws.bgroups;
    hipError_t e = dalloc(&gw.Gpart, (size_t)p->ntiles * p->n_atom * 3);
    if (e == hipSuccess) e = dalloc(&gw.Igrp, (size_t)gw.bgroups * 3 * p->npad);
    if (e != hipSuccess) {
        dfree(gw.Gpart);
        dfree(gw.Igrp);
        (void)hipGetLastError();
        return hip_status(e);
    }
    p->gw = gw;
    return VV10_OK;
}

// Allocate the screening buffers of a workspace (once).
static vv10_status ensure_screen(vv10_plan *p, Workspace &ws) {
    if (ws.mask) return VV10_OK;
    const size_t nblk = (size_t)p->npad / 16;
    hipError_t e = dalloc(&ws.bmax, nblk * ws.Pp);
    if (e == hipSuccess) e = dalloc(&ws.colmax, (size_t)ws.Pp);
    if (e == hipSuccess) e = dalloc(&ws.mask, nblk * ws.ngroups);
    if (e == hipSuccess) e = dalloc(&ws.screen_count, 1);
    if (e != hipSuccess) {
        dfree(ws.bmax);
        dfree(ws.colmax);
        dfree(ws.mask);
        dfree(ws.screen_count);
        ws.bmax = nullptr;
        ws.colmax = nullptr;
        ws.mask = nullptr;
        ws.screen_count = nullptr;
        (void)hipGetLastError();
        return hip_status(e);
    }
    ws.bytes += nblk * ws.Pp * sizeof(float) + ws.Pp * sizeof(float) +
                nblk * ws.ngroups * sizeof(uint32_t) + 4;
    return VV10_OK;
}

// Allocate the weight-derivative buffers (once per plan, after the Hessian
// workspace whose shape they follow).
static vv10_status ensure_weight_work(vv10_plan *p) {
    if (p->ww.Xv) return VV10_OK;
    const Workspace &ws = p->ws;
    vv10::WeightWork ww;
    vv10::weight_shape(ws.Pp, p->prec, ww);
    if (injected_alloc_failure()) return VV10_E_OOM;
    const size_t ch = (size_t)p->npad * ws.Pp;
    char *xv = nullptr, *yp = nullptr;
    hipError_t e = dalloc(&ww.Wown, (size_t)p->npad * 3);
    if (e == hipSuccess) e = dalloc(&xv, ch * (p->prec == VV10_FP64 ? 8 : 4));
    ww.Xv = xv;
    if (e == hipSuccess) e = dalloc(&ww.Lw, ch);
    if (e == hipSuccess) e = dalloc(&yp, ch * 3 * ws.jsplit * vv10::partial_elem(p->prec));
    ww.Ypart = yp;
    if (e == hipSuccess) e = dalloc(&ww.Ze, ch);
    if (e == hipSuccess) e = dalloc(&ww.Rw, ch);
    if (e == hipSuccess) e = dalloc(&ww.Hpart, (size_t)ws.gsplit * (ws.Pp + 1) * ws.Pp);
    if (e != hipSuccess) {
        free_weight_work(ww);
        (void)hipGetLastError();
        return hip_status(e);
    }
    ww.bytes = (size_t)p->npad * 3 * sizeof(double)                    // Wown
             + ch * (p->prec == VV10_FP64 ? 8 : 4)                      // Xv
             + 3 * ch * sizeof(double)                                  // Lw, Ze, Rw
             + ch * 3 * ws.jsplit * vv10::partial_elem(p->prec)         // partials
             + (size_t)ws.gsplit * (ws.Pp + 1) * ws.Pp * sizeof(double); // GEMM slices
    p->ww = ww;
    return VV10_OK;
}

namespace {

// Run one stage, bracketed by timing events when timing is enabled for it.
template <typename Fn>
hipError_t stage(vv10_plan *p, int k, Fn &&fn) {
    const bool timed = (p->timing >> k) & 1u;
    hipError_t e = hipSuccess;
    if (timed) e = hipEventRecord(p->ev[2 * k], p->stream);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess && timed) e = hipEventRecord(p->ev[2 * k + 1], p->stream);
    if (e == hipSuccess && timed) p->ran[k] = true;
    return e;
}

}  // namespace

extern "C" {

const char *vv10_status_string(vv10_status s) {
    switch (s) {
        case VV10_OK: return "ok";
        case VV10_E_ARG: return "invalid argument";
        case VV10_E_DENSITY: return "density not positive or input not finite";
        case VV10_E_GRID_ORDER: return "atom_of is not nondecreasing";
        case VV10_E_OOM: return "device allocation failed";
        case VV10_E_HIP: return "HIP runtime error";
        case VV10_E_STATE: return "plan in invalid state";
    }
    return "unknown status";
}

const char *vv10_version(void) { return "vv10-mi355x 0.1 (gfx950)"; }

size_t vv10_footprint_bytes(int64_t n_grid, int32_t n_atom, vv10_precision prec) {
    if (n_grid < 1 || n_atom < 1) return 0;
    const int64_t npad = ((n_grid + vv10::kPad - 1) / vv10::kPad) * vv10::kPad;
    const int64_t ntiles = (n_grid + vv10::kGridTile - 1) / vv10::kGridTile + n_atom;
    Workspace ws;
    vv10::plan_workspace_shape(npad, n_atom, (int32_t)ntiles, 256, prec, ws);
    // tuned tiles take at most twice the automatic j-split count (the
    // autotuner's candidates); one split writes the partials into Y itself
    ws.jsplit = (int32_t)std::min<int64_t>(2 * (int64_t)ws.jsplit, std::max<int64_t>(1, npad / 256));
    return base_bytes(npad, n_atom, ntiles) +
           vv10::workspace_bytes(npad, n_atom, (int32_t)ntiles, prec, ws);
}

vv10_status vv10_prepare(const vv10_params *params, int64_t n_grid, int32_t n_atom,
                         const double *coords, const double *weights, const int32_t *atom_of,
                         const double *rho, const double *grad_rho, vv10_precision prec,
                         hipStream_t stream, vv10_plan **out) {
    if (!out) return VV10_E_ARG;
    *out = nullptr;
    if (!params || !coords || !weights || !atom_of || !rho || !grad_rho) return VV10_E_ARG;
    if (n_grid < 1 || n_atom < 1 || n_grid > (int64_t)INT32_MAX - vv10::kPad) return VV10_E_ARG;
    if (!(params->b > 0.0) || !std::isfinite(params->b) || !(params->C >= 0.0) ||
        !std::isfinite(params->C))
        return VV10_E_ARG;
    if (prec != VV10_FP64 && prec != VV10_MIXED_FP32 && prec != VV10_MIXED_BF16X3) return VV10_E_ARG;

    vv10_plan *p = new (std::nothrow) vv10_plan();
    if (!p) return VV10_E_OOM;
    p->prm = *params;
    p->beta = std::pow(3.0 / (params->b * params->b), 0.75) / 32.0;
    p->n = n_grid;
    p->npad = ((n_grid + vv10::kPad - 1) / vv10::kPad) * vv10::kPad;
    p->n_atom = n_atom;
    p->prec = prec;
    p->stream = stream;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cu > 0)
            p->num_cu = cu;
    }
    const int64_t npad = p->npad;
    if (e == hipSuccess) e = dalloc(&p->P0, npad);
    if (e == hipSuccess) e = dalloc(&p->P1, npad);
    if (e == hipSuccess) e = dalloc(&p->P0f, npad);
    if (e == hipSuccess) e = dalloc(&p->P1f, npad);
    if (e == hipSuccess) e = dalloc(&p->F, (size_t)vv10::NF * npad);
    if (e == hipSuccess) e = dalloc(&p->I, (size_t)vv10::NI * npad);
    if (e == hipSuccess && vv10::pair_splits(npad) > 1)
        e = dalloc(&p->Ipart, (size_t)vv10::pair_splits(npad) * vv10::NI * npad);
    if (e == hipSuccess) e = dalloc(&p->atom_of, npad);
    if (e == hipSuccess) e = dalloc(&p->red, vv10::reduction_doubles(npad));
    if (e == hipSuccess) e = dalloc(&p->flag, (size_t)n_atom + 2);
    if (e != hipSuccess) {
        vv10_status st = hip_status(e);
        (void)hipGetLastError();
        free_plan(p);
        return st;
    }
    e = vv10::launch_prepare(p, coords, weights, atom_of, rho, grad_rho);
    std::vector<int32_t> flag((size_t)n_atom + 2);
    if (e == hipSuccess)
        e = hipMemcpyAsync(flag.data(), p->flag, flag.size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        return VV10_E_HIP;
    }
    if (flag[0] != 0) {
        free_plan(p);
        if (flag[0] & 4) return VV10_E_ARG;
        if (flag[0] & 1) return VV10_E_DENSITY;
        return VV10_E_GRID_ORDER;
    }
    // atom segments (empty atoms get zero-length segments)
    p->seg.assign((size_t)n_atom + 1, 0);
    p->seg[n_atom] = n_grid;
    for (int32_t A = n_atom - 1; A >= 0; --A)
        p->seg[A] = flag[1 + A] >= 0 ? flag[1 + A] : p->seg[A + 1];
    // grid-term tiles: kGridTile consecutive points of one atom
    p->tile_first.assign((size_t)n_atom + 1, 0);
    for (int32_t A = 0; A < n_atom; ++A) {
        p->tile_first[A] = (int32_t)p->tile_i0.size();
        for (int64_t i0 = p->seg[A]; i0 < p->seg[A + 1]; i0 += vv10::kGridTile) {
            p->tile_i0.push_back((int32_t)i0);
            p->tile_n.push_back((int32_t)std::min<int64_t>(vv10::kGridTile, p->seg[A + 1] - i0));
            p->tile_atom.push_back(A);
        }
    }
    p->ntiles = (int32_t)p->tile_i0.size();
    p->tile_first[n_atom] = p->ntiles;
    // one host image and one copy for all grid metadata (the image lives in
    // the plan, so the copy needs no synchronisation here)
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o_seg = 0;
    const size_t o_i0 = align(o_seg + p->seg.size() * sizeof(int64_t));
    const size_t o_n = align(o_i0 + p->tile_i0.size() * sizeof(int32_t));
    const size_t o_atom = align(o_n + p->tile_n.size() * sizeof(int32_t));
    const size_t o_first = align(o_atom + p->tile_atom.size() * sizeof(int32_t));
    const size_t meta_bytes = align(o_first + p->tile_first.size() * sizeof(int32_t));
    p->h_meta.assign(meta_bytes, 0);
    std::memcpy(p->h_meta.data() + o_seg, p->seg.data(), p->seg.size() * sizeof(int64_t));
    std::memcpy(p->h_meta.data() + o_i0, p->tile_i0.data(), p->tile_i0.size() * sizeof(int32_t));
    std::memcpy(p->h_meta.data() + o_n, p->tile_n.data(), p->tile_n.size() * sizeof(int32_t));
    std::memcpy(p->h_meta.data() + o_atom, p->tile_atom.data(), p->tile_atom.size() * sizeof(int32_t));
    std::memcpy(p->h_meta.data() + o_first, p->tile_first.data(), p->tile_first.size() * sizeof(int32_t));
    if (e == hipSuccess) e = dalloc(&p->d_meta, meta_bytes);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_meta, p->h_meta.data(), meta_bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
        vv10_status st = hip_status(e);
        (void)hipGetLastError();
        free_plan(p);
        return st;
    }
    p->d_seg = reinterpret_cast<int64_t *>(p->d_meta + o_seg);
    p->d_tile_i0 = reinterpret_cast<int32_t *>(p->d_meta + o_i0);
    p->d_tile_n = reinterpret_cast<int32_t *>(p->d_meta + o_n);
    p->d_tile_atom = reinterpret_cast<int32_t *>(p->d_meta + o_atom);
    p->d_tile_first = reinterpret_cast<int32_t *>(p->d_meta + o_first);
    p->base_bytes = base_bytes(npad, n_atom, p->ntiles);
    *out = p;
    return VV10_OK;
}

vv10_status vv10_energy_potential(vv10_plan *p, double *energy, double *f_rho, double *f_gamma) {
    if (!p) return VV10_E_STATE;
    if (p->failed) return VV10_E_STATE;
    if (!energy) return VV10_E_ARG;
    // the pair pass forms E, U, W unless the plan holds them already (a later
    // nuclear-terms call adds A, B, C in its grid pass, which shares the pair
    // arithmetic)
    hipError_t e = hipSuccess;
    if (p->ints_level < 3) {
        e = stage(p, VV10_STAGE_PAIR, [&] { return vv10::launch_pair_integrals(p, false, p->I); });
        if (e == hipSuccess) p->ints_level = 3;
    }
    if (e == hipSuccess)
        e = stage(p, VV10_STAGE_POTENTIAL, [&] { return vv10::launch_potential(p, energy, f_rho, f_gamma); });
    if (e != hipSuccess) {
        p->failed = true;
        (void)hipGetLastError();
        return VV10_E_HIP;
    }
    return VV10_OK;
}

vv10_status vv10_nuclear_terms(vv10_plan *p, int32_t n_pert, const double *rho_x,
                               const double *grad_rho_x, const double *w_x,
                               const vv10_nuclear_outputs *out) {
    if (!p) return VV10_E_STATE;
    if (p->failed) return VV10_E_STATE;
    if (n_pert != 3 * p->n_atom || !rho_x || !grad_rho_x || !out) return VV10_E_ARG;
    if (!out->hess && !out->grad && !out->resp_rho && !out->resp_gamma && !out->fock_rho &&
        !out->fock_gamma && !out->w_coef && !out->energy && !out->f_rho && !out->f_gamma)
        return VV10_OK;
    vv10_status st = vv10::ensure_workspace(p);
    if (st != VV10_OK) return st;
    // weight terms only where an output needs them
    const bool weighted = w_x && (out->hess || out->grad || out->fock_rho || out->fock_gamma);
    if (weighted) {
        st = ensure_weight_work(p);
        if (st != VV10_OK) return st;
    }
    const bool screen = p->screen_tau > 0.0;
    if (screen) {
        st = ensure_screen(p, p->ws);
        if (st != VV10_OK) return st;
    }
    // the grid-term pass also produces the pair integrals E, U, W, A, B, C
    // unless the plan holds them already
    const int ints_from = p->ints_level;    // 0: all six, 3: A, B, C only, 6: none
    hipError_t e = stage(p, VV10_STAGE_GRID, [&] {
        return vv10::launch_grid_terms(p, weighted ? p->ww.Ze : nullptr, ints_from);
    });
    if (e == hipSuccess) p->ints_level = 6;
    if (e == hipSuccess)
        e = stage(p, VV10_STAGE_POTENTIAL, [&] {
            return vv10::launch_potential(p, out->energy, out->f_rho, out->f_gamma);
        });
    if (e == hipSuccess && out->w_coef)
        e = hipMemcpyAsync(out->w_coef, p->F + (size_t)vv10::F_F0 * p->npad,
                           (size_t)p->n * sizeof(double), hipMemcpyDeviceToDevice, p->stream);
    if (e == hipSuccess)
        e = stage(p, VV10_STAGE_PERT_PREP, [&] { return vv10::launch_pert_prep(p, p->ws, rho_x, grad_rho_x, screen); });
    // weighted split-BF16 with one column group of at most four blocks: one
    // fused contraction for the main and the weight rows (timed as the
    // contraction; the weight stage is then the packing alone)
    const bool fused = weighted && !screen && vv10::fused_weighted_contract(p, p->ws);
    if (e == hipSuccess && fused)
        e = stage(p, VV10_STAGE_WEIGHTS, [&] { return vv10::launch_weight_prep(p, w_x); });
    if (e == hipSuccess)
        e = stage(p, VV10_STAGE_CONTRACT, [&] {
            return fused ? vv10::launch_contract_weighted(p, p->ws, p->ww)
                         : vv10::launch_contract(p, p->ws, screen);
        });
    if (e == hipSuccess) {
        p->ws.screened = screen;
        p->rws.screened = false;
    }
    if (e == hipSuccess && weighted && !fused)
        e = stage(p, VV10_STAGE_WEIGHTS, [&] {
            hipError_t r = vv10::launch_weight_prep(p, w_x);
            if (r == hipSuccess) r = vv10::launch_weight_contract(p);
            return r;
        });
    if (e == hipSuccess)
        e = stage(p, VV10_STAGE_ASSEMBLE, [&] { return vv10::launch_assemble(p, *out, weighted); });
    if (e != hipSuccess) {
        p->failed = true;
        (void)hipGetLastError();
        return VV10_E_HIP;
    }
    return VV10_OK;
}

vv10_status vv10_hessian_terms(vv10_plan *p, int32_t n_pert, const double *rho_x,
                               const double *grad_rho_x, double *hess, double *grad,
                               double *resp_rho, double *resp_gamma) {
    if (!p) return VV10_E_STATE;
    if (!hess) return VV10_E_ARG;
    const vv10_nuclear_outputs out = {hess, grad, resp_rho, resp_gamma, nullptr, nullptr,
                                      nullptr, nullptr, nullptr, nullptr};
    return vv10_nuclear_terms(p, n_pert, rho_x, grad_rho_x, nullptr, &out);
}

vv10_status vv10_gradient(vv10_plan *p, int32_t n_pert, const double *rho_x,
                          const double *grad_rho_x, const double *w_x, double *grad) {
    if (!p) return VV10_E_STATE;
    if (p->failed) return VV10_E_STATE;
    if (n_pert != 3 * p->n_atom || !rho_x || !grad_rho_x || !grad) return VV10_E_ARG;
    vv10_status st = ensure_gradient_work(p);
    if (st != VV10_OK) return st;
    if (w_x && !p->wown) {
        if (dalloc(&p->wown, (size_t)p->npad * 3) != hipSuccess) {
            (void)hipGetLastError();
            return VV10_E_OOM;
        }
    }
    const bool ints = p->ints_level < 3;
    hipError_t e = stage(p, VV10_STAGE_GRID, [&] { return vv10::launch_grid_grad(p, ints); });
    if (e == hipSuccess && ints) p->ints_level = 3;
    if (e == hipSuccess)
        e = stage(p, VV10_STAGE_POTENTIAL, [&] { return vv10::launch_potential(p, nullptr, nullptr, nullptr); });
    if (e == hipSuccess)
        e = stage(p, VV10_STAGE_ASSEMBLE, [&] { return vv10::launch_gradient(p, rho_x, grad_rho_x, w_x, grad); });
    if (e != hipSuccess) {
        p->failed = true;
        (void)hipGetLastError();
        return VV10_E_HIP;
    }
    return VV10_OK;
}

vv10_status vv10_trial_response(vv10_plan *p, int32_t n_t, const double *rho_t,
                                const double *grad_rho_t, double *f_rho_t, double *f_gamma_t) {
    if (!p) return VV10_E_STATE;
    if (p->failed) return VV10_E_STATE;
    if (n_t < 0 || n_t > VV10_MAX_TRIAL) return VV10_E_ARG;
    if (n_t == 0) return VV10_OK;
    if (!rho_t || !grad_rho_t || !f_rho_t || !f_gamma_t) return VV10_E_ARG;
    vv10_status st = ensure_response_workspace(p, n_t);
    if (st != VV10_OK) return st;
    const bool screen = p->screen_tau > 0.0;
    if (screen) {
        st = ensure_screen(p, p->rws);
        if (st != VV10_OK) return st;
    }
    hipError_t e = hipSuccess;
    if (!p->ir_ready) {
        e = stage(p, VV10_STAGE_PAIR, [&] { return vv10::launch_pair_integrals(p, true, p->Ir); });
        if (e == hipSuccess) p->ir_ready = true;
    }
    if (e == hipSuccess)
        e = stage(p, VV10_STAGE_PERT_PREP, [&] { return vv10::launch_pert_prep(p, p->rws, rho_t, grad_rho_t, screen); });
    if (e == hipSuccess) e = stage(p, VV10_STAGE_CONTRACT, [&] { return vv10::launch_contract(p, p->rws, screen); });
    if (e == hipSuccess) {
        p->rws.screened = screen;
        p->ws.screened = false;
    }
    if (e == hipSuccess)
        e = stage(p, VV10_STAGE_ASSEMBLE, [&] { return vv10::launch_trial_response(p, f_rho_t, f_gamma_t); });
    if (e != hipSuccess) {
        p->failed = true;
        (void)hipGetLastError();
        return VV10_E_HIP;
    }
    return VV10_OK;
}

size_t vv10_gradient_footprint_bytes(int64_t n_grid, int32_t n_atom) {
    if (n_grid < 1 || n_atom < 1) return 0;
    const int64_t npad = ((n_grid + vv10::kPad - 1) / vv10::kPad) * vv10::kPad;
    const int64_t ntiles = (n_grid + vv10::kGridTile - 1) / vv10::kGridTile + n_atom;
    Workspace ws;
    vv10::plan_workspace_shape(npad, n_atom, (int32_t)ntiles, 256, VV10_FP64, ws);
    // Gpart [tiles][atoms][3] and Igrp [bgroups][3][npad] (ensure_gradient_work)
    return ((size_t)ntiles * n_atom * 3 + (size_t)ws.bgroups * 3 * npad) * sizeof(double) +
           (size_t)npad * 3 * sizeof(double);   // owner slots of w^x (only with weight derivatives)
}

size_t vv10_response_footprint_bytes(int64_t n_grid, int32_t n_t, vv10_precision prec) {
    if (n_grid < 1 || n_t < 1) return 0;
    const int64_t npad = ((n_grid + vv10::kPad - 1) / vv10::kPad) * vv10::kPad;
    Workspace ws;
    vv10::plan_workspace_shape(npad, 1, 1, 256, prec, ws, 0, 0, n_t);
    // tuned tiles take at most twice the automatic j-split count
    ws.jsplit = (int32_t)std::min<int64_t>(2 * (int64_t)ws.jsplit, std::max<int64_t>(1, npad / 256));
    return vv10::response_bytes(npad, prec, ws);
}

vv10_status vv10_set_tiles(vv10_plan *p, const vv10_tiles *t) {
    if (!p || p->ws.X) return VV10_E_STATE;
    if (!t || t->jsplit < 0 || t->bgroups < 0) return VV10_E_ARG;
    p->tiles_jsplit = t->jsplit;
    p->tiles_bgroups = t->bgroups;
    return VV10_OK;
}

vv10_status vv10_set_stream(vv10_plan *p, hipStream_t stream) {
    if (!p) return VV10_E_STATE;
    p->stream = stream;
    return VV10_OK;
}

vv10_status vv10_set_screening(vv10_plan *p, double tau) {
    if (!p) return VV10_E_STATE;
    if (!(tau >= 0.0) || !std::isfinite(tau)) return VV10_E_ARG;
    p->screen_tau = tau;
    return VV10_OK;
}

vv10_status vv10_screening_stats(vv10_plan *p, int64_t *active, int64_t *total) {
    if (!p) return VV10_E_STATE;
    if (!active || !total) return VV10_E_ARG;
    const Workspace *ws = p->ws.screened ? &p->ws : (p->rws.screened ? &p->rws : nullptr);
    if (!ws) return VV10_E_STATE;
    int32_t count = 0;
    hipError_t e = hipMemcpyAsync(&count, ws->screen_count, sizeof(int32_t), hipMemcpyDeviceToHost,
                                  p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return VV10_E_HIP;
    }
    *active = count;
    *total = (p->npad / 16) * (ws->Pp / 16);
    return VV10_OK;
}

vv10_status vv10_get_tiles(vv10_plan *p, vv10_tiles *t) {
    if (!p) return VV10_E_STATE;
    if (!t) return VV10_E_ARG;
    const vv10_status st = vv10::ensure_workspace(p);
    if (st != VV10_OK) return st;
    t->jsplit = p->ws.jsplit;
    t->bgroups = p->ws.bgroups;
    return VV10_OK;
}

vv10_status vv10_set_timing_stages(vv10_plan *p, uint32_t mask) {
    if (!p) return VV10_E_STATE;
    if (mask >> VV10_NUM_STAGES) return VV10_E_ARG;
    if (mask && !p->ev[0]) {
        for (auto &ev : p->ev) {
            if (take_event(p->device, &ev) != hipSuccess) {
                ev = nullptr;
                (void)hipGetLastError();
                return VV10_E_HIP;
            }
        }
    }
    p->timing = mask;
    return VV10_OK;
}

vv10_status vv10_set_timing(vv10_plan *p, int32_t enable) {
    return vv10_set_timing_stages(p, enable ? (1u << VV10_NUM_STAGES) - 1u : 0u);
}

vv10_status vv10_stage_times(vv10_plan *p, double *ms) {
    if (!p || !p->ev[0]) return VV10_E_STATE;
    if (!ms) return VV10_E_ARG;
    for (int k = 0; k < VV10_NUM_STAGES; ++k) {
        ms[k] = 0.0;
        if (!p->ran[k]) continue;
        float t = 0.f;
        if (hipEventSynchronize(p->ev[2 * k + 1]) != hipSuccess ||
            hipEventElapsedTime(&t, p->ev[2 * k], p->ev[2 * k + 1]) != hipSuccess) {
            (void)hipGetLastError();
            return VV10_E_HIP;
        }
        ms[k] = t;
    }
    return VV10_OK;
}

void vv10_destroy(vv10_plan *p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    free_plan(p);
}

}  // extern "C"
