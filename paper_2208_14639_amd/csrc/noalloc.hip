// vv10_energy_potential_noalloc: vv10_prepare, vv10_energy_potential and
// vv10_destroy as one call that allocates no device memory, for callers
// that cannot allocate (code under HIP graph capture, tight loops, harnesses
// that forbid hipMalloc).  Everything the plan would allocate (packed point
// data, per-point fields, pair integrals and their split partials, the
// reduction scratch and the validation flag) lives in one file-scope device
// array, `scratch`, of VV10_NOALLOC_SCRATCH_BYTES per device.  The same
// kernels and launch shapes as the plan path run, so the results are
// bitwise those of vv10_prepare + vv10_energy_potential.
//
// Host code never uses the array's name as an address: the first call on a
// device (that device current) resolves its device address with
// hipGetSymbolAddress and keeps it per device; kernels receive that pointer.
// Calls that overlap on one device share the array and race; the caller
// orders them (one stream, or events between streams).
#include <cmath>
#include <mutex>

#include "vv10_internal.h"

namespace {

static __device__ __align__(256) char scratch[VV10_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
char *g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device (resolved once per
// device), or nullptr with the HIP error in *err.
char *device_scratch(int device, hipError_t *err) {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch[device] = static_cast<char *>(ptr);
    }
    *err = hipSuccess;
    return g_scratch[device];
}

// Byte offsets of the plan's buffers inside the scratch array.
struct Layout {
    size_t P0, P1, P0f, P1f, F, I, Ipart, atom_of, red, flag, end;
};

size_t up(size_t x) { return (x + 255) / 256 * 256; }

Layout layout(int64_t npad, int32_t n_atom) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = up(o + bytes);
        return at;
    };
    L.P0 = take((size_t)npad * sizeof(double4));
    L.P1 = take((size_t)npad * sizeof(double4));
    L.P0f = take((size_t)npad * sizeof(float4));
    L.P1f = take((size_t)npad * sizeof(float4));
    L.F = take((size_t)vv10::NF * npad * sizeof(double));
    L.I = take((size_t)vv10::NI * npad * sizeof(double));
    const int S = vv10::pair_splits(npad);
    L.Ipart = S > 1 ? take((size_t)S * vv10::NI * npad * sizeof(double)) : 0;
    L.atom_of = take((size_t)npad * sizeof(int32_t));
    L.red = take(vv10::reduction_doubles(npad) * sizeof(double));
    L.flag = take(((size_t)n_atom + 2) * sizeof(int32_t));
    L.end = o;
    return L;
}

// *status = the vv10_status of the input validation (flag bits of k_prep:
// 4 atom index out of range, 1 density or input not finite/positive, 2
// atom_of decreasing), as vv10_prepare maps them.
__global__ void k_status(const int32_t *__restrict__ flag, int32_t *__restrict__ status) {
    const int32_t f = flag[0];
    status[0] = f == 0 ? VV10_OK : ((f & 4) ? VV10_E_ARG : ((f & 1) ? VV10_E_DENSITY : VV10_E_GRID_ORDER));
}

}  // namespace

extern "C" size_t vv10_noalloc_bytes(int64_t n_grid, int32_t n_atom) {
    if (n_grid < 1 || n_atom < 1 || n_grid > (int64_t)INT32_MAX - vv10::kPad) return 0;
    const int64_t npad = ((n_grid + vv10::kPad - 1) / vv10::kPad) * vv10::kPad;
    return layout(npad, n_atom).end;
}

extern "C" vv10_status vv10_energy_potential_noalloc(
    const vv10_params *params, int64_t n_grid, int32_t n_atom, const double *coords,
    const double *weights, const int32_t *atom_of, const double *rho, const double *grad_rho,
    vv10_precision prec, hipStream_t stream, double *energy, double *f_rho, double *f_gamma,
    int32_t *status) {
    if (!params || !coords || !weights || !atom_of || !rho || !grad_rho || !energy) return VV10_E_ARG;
    if (n_grid < 1 || n_atom < 1 || n_grid > (int64_t)INT32_MAX - vv10::kPad) return VV10_E_ARG;
    if (!(params->b > 0.0) || !std::isfinite(params->b) || !(params->C >= 0.0) ||
        !std::isfinite(params->C))
        return VV10_E_ARG;
    if (prec != VV10_FP64 && prec != VV10_MIXED_FP32 && prec != VV10_MIXED_BF16X3) return VV10_E_ARG;
    const size_t need = vv10_noalloc_bytes(n_grid, n_atom);
    if (need == 0 || need > (size_t)VV10_NOALLOC_SCRATCH_BYTES) return VV10_E_ARG;

    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess || device < 0 || device >= kMaxDevices) {
        (void)hipGetLastError();
        return VV10_E_HIP;
    }
    char *base = device_scratch(device, &e);
    if (!base) {
        (void)hipGetLastError();
        return VV10_E_HIP;
    }

    // a plan whose buffers are views of the scratch array (host object on
    // the stack; its containers stay empty, nothing is allocated)
    vv10_plan p;
    p.prm = *params;
    p.beta = std::pow(3.0 / (params->b * params->b), 0.75) / 32.0;
    p.n = n_grid;
    p.npad = ((n_grid + vv10::kPad - 1) / vv10::kPad) * vv10::kPad;
    p.n_atom = n_atom;
    p.prec = prec;
    p.stream = stream;
    p.device = device;
    const Layout L = layout(p.npad, n_atom);
    p.P0 = reinterpret_cast<double4 *>(base + L.P0);
    p.P1 = reinterpret_cast<double4 *>(base + L.P1);
    p.P0f = reinterpret_cast<float4 *>(base + L.P0f);
    p.P1f = reinterpret_cast<float4 *>(base + L.P1f);
    p.F = reinterpret_cast<double *>(base + L.F);
    p.I = reinterpret_cast<double *>(base + L.I);
    p.Ipart = L.Ipart ? reinterpret_cast<double *>(base + L.Ipart) : nullptr;
    p.atom_of = reinterpret_cast<int32_t *>(base + L.atom_of);
    p.red = reinterpret_cast<double *>(base + L.red);
    p.flag = reinterpret_cast<int32_t *>(base + L.flag);

    // every scratch word a kernel reads is written earlier in this call
    // (k_fill_i32 sets the flag; k_prep every padded point; the pair pass
    // every partial), so nothing carries over from a previous call
    e = vv10::launch_prepare(&p, coords, weights, atom_of, rho, grad_rho);
    if (e == hipSuccess) e = vv10::launch_pair_integrals(&p, false, p.I);
    if (e == hipSuccess) e = vv10::launch_potential(&p, energy, f_rho, f_gamma, p.flag);
    if (e == hipSuccess && status) {
        k_status<<<1, 1, 0, stream>>>(p.flag, status);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return VV10_E_HIP;
    }
    return VV10_OK;
}
