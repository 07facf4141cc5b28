// Batched evaluation of many molecules (host side of vv10_batch_*).
//
// Every molecule keeps its own plan and workspace (prepared and validated
// eagerly).  vv10_batch_run captures, once, one HIP graph:
//   fork -> per molecule: perturbation packing (branches on side streams)
//   join -> persistent kernels over the work lists of all molecules, each
//           list largest first: split-BF16 only, the contraction items of
//           the molecules with eight or more column blocks per group (eight
//           waves, the standalone kernel's form for them); the other
//           contraction items (four waves); the grid-pass items, one grid
//           tile each (grid-position intermediates with the pair integrals)
//   fork -> per molecule: pair integrals summed over atom groups, potential
//           and energy, Hessian assembly -> join
// and replays it while the caller's pointers stay the same.
#include <algorithm>
#include <new>
#include <vector>

#include "vv10_internal.h"

struct vv10_batch {
    vv10_precision prec = VV10_FP64;
    hipStream_t user_stream = nullptr;
    hipStream_t cap = nullptr;                 // capture stream (never the null stream)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;                // fork/join events
    std::vector<vv10_plan *> plans;
    std::vector<int64_t> rx_off, gx_off, h_off;
    vv10::BatchMol *d_mols = nullptr;
    vv10::BatchItem *d_items = nullptr;        // contraction, wide, grid lists
    int32_t *d_counter = nullptr;              // [3]: one per list
    int64_t n_items = 0;                       // contraction items (four waves)
    int64_t n_wide = 0;                        // wide contraction items (split-BF16)
    int64_t n_grid = 0;                        // grid items
    int32_t n_blocks = 0;
    int32_t n_wide_blocks = 0;
    int32_t n_grid_blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *cap_ptr[4] = {nullptr, nullptr, nullptr, nullptr};
    bool failed = false;
};

namespace {

void destroy_batch(vv10_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (vv10_plan *p : b->plans) vv10_destroy(p);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : b->side)
        if (s) (void)hipStreamDestroy(s);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    vv10::dev_free(b->d_mols);
    vv10::dev_free(b->d_items);
    vv10::dev_free(b->d_counter);
    delete b;
}

vv10_status status_of(hipError_t e) {
    if (e == hipSuccess) return VV10_OK;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? VV10_E_OOM : VV10_E_HIP;
}

// Enqueue the whole batch on b->cap (inside stream capture).
hipError_t enqueue_batch(vv10_batch *b, const double *rho_x, const double *grad_rho_x,
                         double *energy, double *hess) {
    const int K = (int)b->side.size();
    const size_t nm = b->plans.size();
    hipError_t e = hipEventRecord(b->ev[0], b->cap);
    for (int k = 0; k < K && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->side[k], b->ev[0], 0);
    // per-molecule stage before the persistent kernel
    for (size_t m = 0; m < nm && e == hipSuccess; ++m) {
        vv10_plan *p = b->plans[m];
        p->stream = b->side[m % K];
        e = vv10::launch_pert_prep(p, p->ws, rho_x + b->rx_off[m], grad_rho_x + b->gx_off[m]);
    }
    for (int k = 0; k < K && e == hipSuccess; ++k) {
        e = hipEventRecord(b->ev[1 + k], b->side[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->ev[1 + k], 0);
    }
    if (e == hipSuccess && b->n_wide > 0)
        e = vv10::launch_contract_persistent_wide(b->d_mols, b->d_items + b->n_items,
                                                  (int32_t)b->n_wide, b->d_counter + 1,
                                                  b->n_wide_blocks, b->cap);
    if (e == hipSuccess && b->n_items > 0)
        e = vv10::launch_contract_persistent(b->prec, b->d_mols, b->d_items, (int32_t)b->n_items,
                                            b->d_counter, b->n_blocks, b->cap);
    if (e == hipSuccess && b->n_grid > 0)
        e = vv10::launch_grid_persistent(b->prec, b->d_mols, b->d_items + b->n_items + b->n_wide,
                                         (int32_t)b->n_grid, b->d_counter + 2, b->n_grid_blocks,
                                         b->cap);
    if (e == hipSuccess) e = hipEventRecord(b->ev[1 + K], b->cap);
    for (int k = 0; k < K && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->side[k], b->ev[1 + K], 0);
    for (size_t m = 0; m < nm && e == hipSuccess; ++m) {
        vv10_plan *p = b->plans[m];
        p->stream = b->side[m % K];
        const vv10_nuclear_outputs out = {hess + b->h_off[m], nullptr, nullptr, nullptr, nullptr,
                                          nullptr, nullptr, nullptr, nullptr, nullptr};
        e = vv10::launch_sum_groups(p, 0);
        if (e == hipSuccess) e = vv10::launch_potential(p, energy + m, nullptr, nullptr);
        if (e == hipSuccess) e = vv10::launch_assemble(p, out, false);
    }
    for (int k = 0; k < K && e == hipSuccess; ++k) {
        e = hipEventRecord(b->ev[2 + K + k], b->side[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->ev[2 + K + k], 0);
    }
    for (vv10_plan *p : b->plans) p->stream = b->user_stream;
    return e;
}

}  // namespace

extern "C" {

vv10_status vv10_batch_create(const vv10_params *params, int32_t n_mol, const int64_t *grid_off,
                              const int32_t *atom_off, const double *coords,
                              const double *weights, const int32_t *atom_of, const double *rho,
                              const double *grad_rho, vv10_precision prec,
                              const vv10_tiles *tiles, hipStream_t stream, vv10_batch **out) {
    if (!out) return VV10_E_ARG;
    *out = nullptr;
    if (!params || n_mol < 1 || !grid_off || !atom_off || !coords || !weights || !atom_of ||
        !rho || !grad_rho)
        return VV10_E_ARG;
    if (grid_off[0] != 0 || atom_off[0] != 0) return VV10_E_ARG;
    for (int32_t m = 0; m < n_mol; ++m)
        if (grid_off[m + 1] <= grid_off[m] || atom_off[m + 1] <= atom_off[m]) return VV10_E_ARG;

    vv10_batch *b = new (std::nothrow) vv10_batch();
    if (!b) return VV10_E_OOM;
    b->prec = prec;
    b->user_stream = stream;
    vv10_status st = VV10_OK;
    int64_t rx = 0, hx = 0;
    for (int32_t m = 0; m < n_mol && st == VV10_OK; ++m) {
        const int64_t g0 = grid_off[m], n = grid_off[m + 1] - g0;
        const int32_t na = atom_off[m + 1] - atom_off[m];
        vv10_plan *p = nullptr;
        st = vv10_prepare(params, n, na, coords + 3 * g0, weights + g0, atom_of + g0, rho + g0,
                          grad_rho + 3 * g0, prec, stream, &p);
        if (st != VV10_OK) break;
        b->plans.push_back(p);
        if (tiles) st = vv10_set_tiles(p, tiles + m);
        if (st == VV10_OK) st = vv10::ensure_workspace(p);
        b->rx_off.push_back(rx);
        b->gx_off.push_back(3 * rx);
        b->h_off.push_back(hx);
        rx += (int64_t)3 * na * n;
        hx += (int64_t)9 * na * na;
    }
    // work lists: contraction items (molecule, column group, j split, i tile)
    // and grid items (molecule, atom group, grid tile)
    std::vector<vv10::BatchMol> mols;
    std::vector<vv10::BatchItem> items, gitems, witems;
    std::vector<int64_t> cost, gcost, wcost;
    const int W = vv10::persistent_waves(prec);   // waves per persistent workgroup
    if (st == VV10_OK) {
        for (size_t m = 0; m < b->plans.size(); ++m) {
            const vv10_plan *p = b->plans[m];
            const vv10::Workspace &ws = p->ws;
            vv10::BatchMol d;
            d.npad = p->npad;
            d.jlen = ws.jlen;
            d.Pp = ws.Pp;
            d.ncb = ws.ncb;
            d.P0 = prec == VV10_FP64 ? (const void *)p->P0 : (const void *)p->P0f;
            d.P1 = prec == VV10_FP64 ? (const void *)p->P1 : (const void *)p->P1f;
            d.X = ws.X;
            d.Ypart = ws.Ypart;
            d.n_atom = p->n_atom;
            d.bgroups = ws.bgroups;
            d.ntiles = p->ntiles;
            d.pad0 = 0;
            d.seg = p->d_seg;
            d.tile_i0 = p->d_tile_i0;
            d.tile_n = p->d_tile_n;
            d.tile_atom = p->d_tile_atom;
            d.Pd = p->P1;
            d.Z = ws.Z;
            d.Dpart = ws.Dpart;
            d.Igrp = ws.Igrp;
            mols.push_back(d);
            // a grid item pairs one grid tile of up to 64 outer points with
            // every point of its atom group
            for (int32_t g = 0; g < ws.bgroups; ++g) {
                int64_t pts = 0;
                for (int32_t B = g; B < p->n_atom; B += ws.bgroups) pts += p->seg[B + 1] - p->seg[B];
                for (int32_t t = 0; t < p->ntiles; ++t) {
                    gitems.push_back({(int32_t)m, g, -1, t});
                    gcost.push_back((int64_t)p->tile_n[t] * pts);
                }
            }
            // split-BF16 with kWideMinNcb or more column blocks: the wide
            // list, i tiles of 128 points (npad is a multiple of 256)
            const bool wide = prec == VV10_MIXED_BF16X3 && ws.ncb >= vv10::kWideMinNcb;
            const int Wc = wide ? 8 : W;
            for (int32_t s = 0; s < ws.jsplit; ++s) {
                const int64_t jl = std::min<int64_t>(ws.jlen, p->npad - (int64_t)s * ws.jlen);
                for (int32_t g = 0; g < ws.ngroups; ++g)
                    for (int64_t t = 0; t < p->npad / (16 * Wc); ++t) {
                        (wide ? witems : items).push_back({(int32_t)m, g, s, (int32_t)t});
                        (wide ? wcost : cost).push_back(jl * ws.ncb * Wc / 4);
                    }
            }
        }
        // one list per kernel, each largest first: run side by side on one
        // CU, grid and contraction items slow each other more than they
        // overlap (measured on the 64-cluster batch: interleaved in
        // proportion to their cost 3.02 s per launch, one kind after the
        // other 2.86 s)
        auto by_cost = [](const std::vector<vv10::BatchItem> &it, const std::vector<int64_t> &c,
                          std::vector<vv10::BatchItem> &out) {
            std::vector<size_t> order(it.size());
            for (size_t k = 0; k < order.size(); ++k) order[k] = k;
            std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t d) { return c[a] > c[d]; });
            for (size_t k : order) out.push_back(it[k]);
        };
        std::vector<vv10::BatchItem> all;
        by_cost(items, cost, all);
        b->n_items = (int64_t)all.size();
        by_cost(witems, wcost, all);
        b->n_wide = (int64_t)all.size() - b->n_items;
        by_cost(gitems, gcost, all);
        b->n_grid = (int64_t)all.size() - b->n_items - b->n_wide;
        items.swap(all);
        if (b->n_items > INT32_MAX || b->n_wide > INT32_MAX || b->n_grid > INT32_MAX)
            st = VV10_E_ARG;
    }
    if (st == VV10_OK) {
        hipError_t e = vv10::dev_alloc(reinterpret_cast<void **>(&b->d_mols),
                                       mols.size() * sizeof(vv10::BatchMol));
        if (e == hipSuccess)
            e = vv10::dev_alloc(reinterpret_cast<void **>(&b->d_items),
                                std::max<size_t>(1, items.size()) * sizeof(vv10::BatchItem));
        if (e == hipSuccess) e = vv10::dev_alloc(reinterpret_cast<void **>(&b->d_counter), 3 * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(b->d_mols, mols.data(), mols.size() * sizeof(vv10::BatchMol), hipMemcpyHostToDevice);
        if (e == hipSuccess && !items.empty())
            e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(vv10::BatchItem), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipStreamCreate(&b->cap);
        const int K = (int)std::min<size_t>(4, b->plans.size());
        for (int k = 0; k < K && e == hipSuccess; ++k) {
            hipStream_t s = nullptr;
            e = hipStreamCreate(&s);
            b->side.push_back(s);
        }
        for (int k = 0; k < 2 + 2 * K && e == hipSuccess; ++k) {
            hipEvent_t ev = nullptr;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            b->ev.push_back(ev);
        }
        if (e == hipSuccess) {
            int per_cu = vv10::persistent_blocks_per_cu(prec);
            if (per_cu <= 0) per_cu = 1;
            b->n_blocks = (int32_t)std::min<int64_t>((int64_t)per_cu * b->plans[0]->num_cu,
                                                     std::max<int64_t>(1, b->n_items));
            int per_cu_g = vv10::persistent_grid_blocks_per_cu(prec);
            if (per_cu_g <= 0) per_cu_g = 1;
            b->n_grid_blocks = (int32_t)std::min<int64_t>((int64_t)per_cu_g * b->plans[0]->num_cu,
                                                          std::max<int64_t>(1, b->n_grid));
            if (b->n_wide > 0) {
                int per_cu_w = vv10::persistent_wide_blocks_per_cu();
                if (per_cu_w <= 0) per_cu_w = 1;
                b->n_wide_blocks = (int32_t)std::min<int64_t>(
                    (int64_t)per_cu_w * b->plans[0]->num_cu, b->n_wide);
            }
        }
        st = status_of(e);
    }
    if (st != VV10_OK) {
        destroy_batch(b);
        return st;
    }
    *out = b;
    return VV10_OK;
}

vv10_status vv10_batch_run(vv10_batch *b, const double *rho_x, const double *grad_rho_x,
                           double *energy, double *hess) {
    if (!b || b->failed) return VV10_E_STATE;
    if (!rho_x || !grad_rho_x || !energy || !hess) return VV10_E_ARG;
    const void *ptr[4] = {rho_x, grad_rho_x, energy, hess};
    hipError_t e = hipSuccess;
    if (!b->exec || !std::equal(ptr, ptr + 4, b->cap_ptr)) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = enqueue_batch(b, rho_x, grad_rho_x, energy, hess);
            e = hipStreamEndCapture(b->cap, &b->graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            b->failed = true;
            (void)hipGetLastError();
            return VV10_E_HIP;
        }
        std::copy(ptr, ptr + 4, b->cap_ptr);
    }
    e = hipGraphLaunch(b->exec, b->user_stream);
    if (e != hipSuccess) {
        b->failed = true;
        (void)hipGetLastError();
        return VV10_E_HIP;
    }
    return VV10_OK;
}

vv10_status vv10_batch_info(const vv10_batch *b, int64_t *n_items, int32_t *n_workgroups) {
    if (!b) return VV10_E_STATE;
    if (n_items) *n_items = b->n_items + b->n_wide + b->n_grid;
    if (n_workgroups) *n_workgroups = b->n_blocks;
    return VV10_OK;
}

void vv10_batch_destroy(vv10_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->user_stream);
    destroy_batch(b);
}

}  // extern "C"
