"""Python binding of the VV10 C ABI (include/vv10.h).

Argument marshalling only: every step of the computation runs in the HIP
library ``libvv10.so``.  Functions keep the C names; array arguments are
torch tensors on the GPU (or raw device addresses as ints) and are passed
as plain pointers.  PyTorch is used for device memory and streams only.

The library is loaded from this directory; if it is missing the import of
any entry point raises -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# VV10_LIBRARY selects another build of the same sources (the host-sanitized
# libvv10_san.so, for example)
LIB_PATH = os.environ.get("VV10_LIBRARY") or os.path.join(HERE, "libvv10.so")

VV10_OK = 0
VV10_E_ARG = -1
VV10_E_DENSITY = -2
VV10_E_GRID_ORDER = -3
VV10_E_OOM = -4
VV10_E_HIP = -5
VV10_E_STATE = -6

VV10_NOALLOC_SCRATCH_BYTES = 64 << 20   # static scratch of vv10_energy_potential_noalloc

VV10_FP64 = 0
VV10_MIXED_FP32 = 1
VV10_MIXED_BF16X3 = 2
PRECISIONS = {"fp64": VV10_FP64, "fp32": VV10_MIXED_FP32, "bf16x3": VV10_MIXED_BF16X3}

STAGES = ("pair", "potential", "pert_prep", "contract", "grid", "assemble", "weights")


class vv10_params(ctypes.Structure):
    _fields_ = [("b", ctypes.c_double), ("C", ctypes.c_double)]


class vv10_tiles(ctypes.Structure):
    _fields_ = [("jsplit", ctypes.c_int32), ("bgroups", ctypes.c_int32)]


class vv10_nuclear_outputs(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in
                ("hess", "grad", "resp_rho", "resp_gamma", "fock_rho", "fock_gamma", "w_coef",
                 "energy", "f_rho", "f_gamma")]


class VV10Error(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {vv10_status_string(status)} ({status})")


_lib = None


def load() -> ctypes.CDLL:
    """Load libvv10.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with paper_2208_14639_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    lib.vv10_prepare.restype = st
    lib.vv10_prepare.argtypes = [ctypes.POINTER(vv10_params), i64, i32, P, P, P, P, P, st, P,
                                 ctypes.POINTER(P)]
    lib.vv10_energy_potential.restype = st
    lib.vv10_energy_potential.argtypes = [P, P, P, P]
    lib.vv10_hessian_terms.restype = st
    lib.vv10_hessian_terms.argtypes = [P, i32, P, P, P, P, P, P]
    lib.vv10_footprint_bytes.restype = ctypes.c_size_t
    lib.vv10_footprint_bytes.argtypes = [i64, i32, st]
    lib.vv10_nuclear_terms.restype = st
    lib.vv10_nuclear_terms.argtypes = [P, i32, P, P, P, ctypes.POINTER(vv10_nuclear_outputs)]
    lib.vv10_gradient.restype = st
    lib.vv10_gradient.argtypes = [P, i32, P, P, P, P]
    lib.vv10_trial_response.restype = st
    lib.vv10_trial_response.argtypes = [P, i32, P, P, P, P]
    lib.vv10_response_footprint_bytes.restype = ctypes.c_size_t
    lib.vv10_response_footprint_bytes.argtypes = [i64, i32, st]
    lib.vv10_gradient_footprint_bytes.restype = ctypes.c_size_t
    lib.vv10_gradient_footprint_bytes.argtypes = [i64, i32]
    lib.vv10_destroy.restype = None
    lib.vv10_destroy.argtypes = [P]
    lib.vv10_status_string.restype = ctypes.c_char_p
    lib.vv10_status_string.argtypes = [st]
    lib.vv10_version.restype = ctypes.c_char_p
    lib.vv10_version.argtypes = []
    lib.vv10_set_tiles.restype = st
    lib.vv10_set_tiles.argtypes = [P, ctypes.POINTER(vv10_tiles)]
    lib.vv10_set_screening.restype = st
    lib.vv10_set_screening.argtypes = [P, ctypes.c_double]
    lib.vv10_screening_stats.restype = st
    lib.vv10_screening_stats.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.vv10_cached_bytes.restype = ctypes.c_size_t
    lib.vv10_cached_bytes.argtypes = []
    lib.vv10_release_cached.restype = None
    lib.vv10_release_cached.argtypes = []
    lib.vv10_set_stream.restype = st
    lib.vv10_set_stream.argtypes = [P, P]
    lib.vv10_get_tiles.restype = st
    lib.vv10_get_tiles.argtypes = [P, ctypes.POINTER(vv10_tiles)]
    lib.vv10_batch_create.restype = st
    lib.vv10_batch_create.argtypes = [ctypes.POINTER(vv10_params), i32, P, P, P, P, P, P, P, st, P, P,
                                      ctypes.POINTER(P)]
    lib.vv10_batch_run.restype = st
    lib.vv10_batch_run.argtypes = [P, P, P, P, P]
    lib.vv10_batch_info.restype = st
    lib.vv10_batch_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.vv10_batch_destroy.restype = None
    lib.vv10_batch_destroy.argtypes = [P]
    lib.vv10_set_timing.restype = st
    lib.vv10_set_timing.argtypes = [P, i32]
    lib.vv10_set_timing_stages.restype = st
    lib.vv10_set_timing_stages.argtypes = [P, ctypes.c_uint32]
    lib.vv10_stage_times.restype = st
    lib.vv10_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    lib.vv10_energy_potential_noalloc.restype = st
    lib.vv10_energy_potential_noalloc.argtypes = [ctypes.POINTER(vv10_params), i64, i32, P, P, P,
                                                  P, P, st, P, P, P, P, P]
    lib.vv10_noalloc_bytes.restype = ctypes.c_size_t
    lib.vv10_noalloc_bytes.argtypes = [i64, i32]
    _lib = lib
    return lib


def _prec_name(prec: int) -> str:
    return {v: k for k, v in PRECISIONS.items()}[prec]


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def vv10_status_string(status: int) -> str:
    return load().vv10_status_string(status).decode()


def vv10_version() -> str:
    return load().vv10_version().decode()


def vv10_footprint_bytes(n_grid: int, n_atom: int, prec: int = VV10_FP64) -> int:
    return int(load().vv10_footprint_bytes(n_grid, n_atom, prec))


def vv10_prepare(b: float, C: float, n_grid: int, n_atom: int, coords, weights, atom_of, rho,
                 grad_rho, prec: int = VV10_FP64, stream=None) -> int:
    """Returns the plan handle (an int); raises VV10Error on failure."""
    lib = load()
    prm = vv10_params(b, C)
    out = ctypes.c_void_p()
    st = lib.vv10_prepare(ctypes.byref(prm), n_grid, n_atom, _ptr(coords), _ptr(weights),
                          _ptr(atom_of), _ptr(rho), _ptr(grad_rho), prec, _stream(stream),
                          ctypes.byref(out))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_prepare")
    return out.value


def vv10_energy_potential(plan: int, energy, f_rho=None, f_gamma=None) -> None:
    st = load().vv10_energy_potential(plan, _ptr(energy), _ptr(f_rho), _ptr(f_gamma))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_energy_potential")


def vv10_energy_potential_noalloc(b: float, C: float, n_grid: int, n_atom: int, coords, weights,
                                  atom_of, rho, grad_rho, prec: int, stream, energy, f_rho=None,
                                  f_gamma=None, status=None) -> None:
    """vv10_prepare + vv10_energy_potential without device allocation (the
    library's static scratch array); status: device int32 [1] or None."""
    prm = vv10_params(b, C)
    st = load().vv10_energy_potential_noalloc(ctypes.byref(prm), n_grid, n_atom, _ptr(coords),
                                              _ptr(weights), _ptr(atom_of), _ptr(rho),
                                              _ptr(grad_rho), prec, _stream(stream), _ptr(energy),
                                              _ptr(f_rho), _ptr(f_gamma), _ptr(status))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_energy_potential_noalloc")


def vv10_noalloc_bytes(n_grid: int, n_atom: int) -> int:
    return int(load().vv10_noalloc_bytes(n_grid, n_atom))


def vv10_hessian_terms(plan: int, n_pert: int, rho_x, grad_rho_x, hess, grad=None,
                       resp_rho=None, resp_gamma=None) -> None:
    st = load().vv10_hessian_terms(plan, n_pert, _ptr(rho_x), _ptr(grad_rho_x), _ptr(hess),
                                   _ptr(grad), _ptr(resp_rho), _ptr(resp_gamma))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_hessian_terms")


def vv10_nuclear_terms(plan: int, n_pert: int, rho_x, grad_rho_x, hess=None, grad=None,
                       resp_rho=None, resp_gamma=None, fock_rho=None, fock_gamma=None,
                       w_x=None, w_coef=None, energy=None, f_rho=None, f_gamma=None) -> None:
    out = vv10_nuclear_outputs(*(_ptr(t) for t in (hess, grad, resp_rho, resp_gamma, fock_rho,
                                                    fock_gamma, w_coef, energy, f_rho, f_gamma)))
    st = load().vv10_nuclear_terms(plan, n_pert, _ptr(rho_x), _ptr(grad_rho_x), _ptr(w_x),
                                   ctypes.byref(out))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_nuclear_terms")


def vv10_gradient(plan: int, n_pert: int, rho_x, grad_rho_x, grad, w_x=None) -> None:
    st = load().vv10_gradient(plan, n_pert, _ptr(rho_x), _ptr(grad_rho_x), _ptr(w_x), _ptr(grad))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_gradient")


def vv10_trial_response(plan: int, n_t: int, rho_t, grad_rho_t, f_rho_t, f_gamma_t) -> None:
    st = load().vv10_trial_response(plan, n_t, _ptr(rho_t), _ptr(grad_rho_t), _ptr(f_rho_t),
                                    _ptr(f_gamma_t))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_trial_response")


def vv10_response_footprint_bytes(n_grid: int, n_t: int, prec: int = VV10_FP64) -> int:
    return int(load().vv10_response_footprint_bytes(n_grid, n_t, prec))


def vv10_gradient_footprint_bytes(n_grid: int, n_atom: int) -> int:
    return int(load().vv10_gradient_footprint_bytes(n_grid, n_atom))


def vv10_set_tiles(plan: int, jsplit: int = 0, bgroups: int = 0) -> None:
    t = vv10_tiles(jsplit, bgroups)
    st = load().vv10_set_tiles(plan, ctypes.byref(t))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_set_tiles")


def vv10_cached_bytes() -> int:
    return int(load().vv10_cached_bytes())


def vv10_release_cached() -> None:
    load().vv10_release_cached()


def vv10_set_stream(plan: int, stream) -> None:
    st = load().vv10_set_stream(plan, _stream(stream))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_set_stream")


def vv10_set_screening(plan: int, tau: float) -> None:
    st = load().vv10_set_screening(plan, float(tau))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_set_screening")


def vv10_screening_stats(plan: int):
    """(active, total) (16-point, 16-column) blocks of the last screened contraction."""
    a, t = ctypes.c_int64(0), ctypes.c_int64(0)
    st = load().vv10_screening_stats(plan, ctypes.byref(a), ctypes.byref(t))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_screening_stats")
    return a.value, t.value


def vv10_get_tiles(plan: int):
    t = vv10_tiles()
    st = load().vv10_get_tiles(plan, ctypes.byref(t))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_get_tiles")
    return int(t.jsplit), int(t.bgroups)


def vv10_batch_create(b: float, C: float, grid_off, atom_off, coords, weights, atom_of, rho,
                      grad_rho, prec: int = VV10_FP64, tiles=None, stream=None) -> int:
    """grid_off / atom_off: host int sequences of length n_mol + 1; tiles: a
    list of (jsplit, bgroups) per molecule or None.  Returns the batch handle."""
    import numpy as np
    lib = load()
    go = np.ascontiguousarray(grid_off, dtype=np.int64)
    ao = np.ascontiguousarray(atom_off, dtype=np.int32)
    n_mol = len(go) - 1
    tl = None
    if tiles is not None:
        tl = (vv10_tiles * n_mol)(*[vv10_tiles(int(j), int(g)) for j, g in tiles])
    prm = vv10_params(b, C)
    out = ctypes.c_void_p()
    st = lib.vv10_batch_create(ctypes.byref(prm), n_mol, go.ctypes.data, ao.ctypes.data,
                               _ptr(coords), _ptr(weights), _ptr(atom_of), _ptr(rho),
                               _ptr(grad_rho), prec, ctypes.cast(tl, ctypes.c_void_p) if tl else None,
                               _stream(stream), ctypes.byref(out))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_batch_create")
    return out.value


def vv10_batch_run(batch: int, rho_x, grad_rho_x, energy, hess) -> None:
    st = load().vv10_batch_run(batch, _ptr(rho_x), _ptr(grad_rho_x), _ptr(energy), _ptr(hess))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_batch_run")


def vv10_batch_info(batch: int):
    n_items = ctypes.c_int64()
    n_wg = ctypes.c_int32()
    st = load().vv10_batch_info(batch, ctypes.byref(n_items), ctypes.byref(n_wg))
    if st != VV10_OK:
        raise VV10Error(st, "vv10_batch_info")
    return n_items.value, n_wg.value


def vv10_batch_destroy(batch: int) -> None:
    if batch:
        load().vv10_batch_destroy(batch)


def vv10_set_timing(plan: int, enable: bool = True) -> None:
    st = load().vv10_set_timing(plan, 1 if enable else 0)
    if st != VV10_OK:
        raise VV10Error(st, "vv10_set_timing")


def vv10_set_timing_stages(plan: int, stages) -> None:
    """Time only the named stages (names of STAGES) or a bit mask of them."""
    mask = stages if isinstance(stages, int) else sum(1 << STAGES.index(s) for s in set(stages))
    st = load().vv10_set_timing_stages(plan, mask)
    if st != VV10_OK:
        raise VV10Error(st, "vv10_set_timing_stages")


def vv10_stage_times(plan: int) -> dict:
    """Milliseconds per stage of the most recent runs (host dict)."""
    buf = (ctypes.c_double * len(STAGES))()
    st = load().vv10_stage_times(plan, buf)
    if st != VV10_OK:
        raise VV10Error(st, "vv10_stage_times")
    return dict(zip(STAGES, list(buf)))


def vv10_destroy(plan: int) -> None:
    if plan:
        load().vv10_destroy(plan)


class Plan:
    """A prepared grid on the current device (owns a vv10_plan).

    ``problem`` is anything with coords, weights, atom_of, rho, grad_rho,
    n_grid, n_atom, b, C (e.g. inputs.Problem); arrays are copied to the
    device as FP64/int32 tensors."""

    def __init__(self, problem, prec="fp64", device="cuda", stream=None, tiles=None,
                 screening=0.0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        self.n = int(problem.n_grid)
        self.n_atom = int(problem.n_atom)
        d = self._dev
        self.coords = d(problem.coords)
        self.weights = d(problem.weights)
        self.atom_of = torch.as_tensor(problem.atom_of, dtype=torch.int32).to(self.device).contiguous()
        self.rho = d(problem.rho)
        self.grad_rho = d(problem.grad_rho)
        self.stream = stream
        self.handle = vv10_prepare(problem.b, problem.C, self.n, self.n_atom, self.coords,
                                   self.weights, self.atom_of, self.rho, self.grad_rho,
                                   self.prec, stream)
        if tiles == "auto":
            from . import autotune
            tiles = autotune.lookup(self.n, self.n_atom, _prec_name(self.prec))
        if tiles is not None:
            vv10_set_tiles(self.handle, *tiles)
        self.tiles = tiles
        if screening:
            vv10_set_screening(self.handle, screening)

    def _dev(self, a):
        return self.torch.as_tensor(a, dtype=self.torch.float64).to(self.device).contiguous()

    def energy_potential(self):
        t = self.torch
        e = t.empty(1, dtype=t.float64, device=self.device)
        fr = t.empty(self.n, dtype=t.float64, device=self.device)
        fg = t.empty(self.n, dtype=t.float64, device=self.device)
        vv10_energy_potential(self.handle, e, fr, fg)
        return e, fr, fg

    def hessian_terms(self, rho_x, grad_rho_x, grad=False, resp=False):
        t = self.torch
        P = 3 * self.n_atom
        rx = rho_x if isinstance(rho_x, t.Tensor) and rho_x.is_cuda else self._dev(rho_x)
        gx = grad_rho_x if isinstance(grad_rho_x, t.Tensor) and grad_rho_x.is_cuda else self._dev(grad_rho_x)
        H = t.empty((P, P), dtype=t.float64, device=self.device)
        g = t.empty(P, dtype=t.float64, device=self.device) if grad else None
        rr = t.empty((P, self.n), dtype=t.float64, device=self.device) if resp else None
        rg = t.empty((P, self.n), dtype=t.float64, device=self.device) if resp else None
        vv10_hessian_terms(self.handle, P, rx, gx, H, g, rr, rg)
        out = {"hess": H}
        if grad:
            out["grad"] = g
        if resp:
            out["resp_rho"], out["resp_gamma"] = rr, rg
        return out

    def _in(self, a):
        t = self.torch
        if a is None:
            return None
        return a if isinstance(a, t.Tensor) and a.is_cuda else self._dev(a)

    def nuclear_terms(self, rho_x, grad_rho_x, hess=True, grad=False, resp=False, fock=False,
                      w_x=None, w_coef=False, energy=False, potential=False):
        """Any subset of the nuclear-perturbation outputs of one pass; w_x
        ([3 n_atom, N], or None) are the weights' nuclear derivatives."""
        t = self.torch
        P = 3 * self.n_atom
        rx, gx, wx = self._in(rho_x), self._in(grad_rho_x), self._in(w_x)
        mk = lambda on, shape: t.empty(shape, dtype=t.float64, device=self.device) if on else None
        out = {"hess": mk(hess, (P, P)), "grad": mk(grad, P),
               "resp_rho": mk(resp, (P, self.n)), "resp_gamma": mk(resp, (P, self.n)),
               "fock_rho": mk(fock, (P, self.n)), "fock_gamma": mk(fock, (P, self.n)),
               "w_coef": mk(w_coef, self.n), "energy": mk(energy, 1),
               "f_rho": mk(potential, self.n), "f_gamma": mk(potential, self.n)}
        vv10_nuclear_terms(self.handle, P, rx, gx, w_x=wx, **out)
        return {k: v for k, v in out.items() if v is not None}

    def gradient(self, rho_x, grad_rho_x, w_x=None):
        """Nuclear gradient [3 n_atom] alone (with E_w when w_x is given)."""
        t = self.torch
        P = 3 * self.n_atom
        rx, gx, wx = self._in(rho_x), self._in(grad_rho_x), self._in(w_x)
        g = t.empty(P, dtype=t.float64, device=self.device)
        vv10_gradient(self.handle, P, rx, gx, g, w_x=wx)
        return g

    def trial_response(self, rho_t, grad_rho_t):
        """f^{rho,t}, f^{gamma,t} ([n_t, N] each) of n_t trial densities."""
        t = self.torch
        rt = rho_t if isinstance(rho_t, t.Tensor) and rho_t.is_cuda else self._dev(rho_t)
        gt = grad_rho_t if isinstance(grad_rho_t, t.Tensor) and grad_rho_t.is_cuda else self._dev(grad_rho_t)
        n_t = int(rt.shape[0])
        fr = t.empty((n_t, self.n), dtype=t.float64, device=self.device)
        fg = t.empty((n_t, self.n), dtype=t.float64, device=self.device)
        vv10_trial_response(self.handle, n_t, rt, gt, fr, fg)
        return fr, fg

    def close(self):
        if self.handle:
            vv10_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Many problems evaluated together (one HIP graph per run).

    ``problems`` is a sequence of inputs.Problem-like objects with derivatives;
    all must share b and C.  ``run()`` returns (energies [n_mol] tensor,
    list of Hessian blocks [P_m, P_m])."""

    def __init__(self, problems, prec="bf16x3", device="cuda", tiles=None, stream=None):
        import numpy as np
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        self.problems = list(problems)
        n = [int(p.n_grid) for p in self.problems]
        na = [int(p.n_atom) for p in self.problems]
        self.grid_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
        self.atom_off = np.concatenate([[0], np.cumsum(na)]).astype(np.int32)
        self.P = [3 * a for a in na]
        cat = lambda f: np.concatenate([np.asarray(f(p)).reshape(-1) for p in self.problems])
        d = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt).to(self.device).contiguous()
        self.coords = d(cat(lambda p: p.coords))
        self.weights = d(cat(lambda p: p.weights))
        self.atom_of = d(cat(lambda p: p.atom_of), torch.int32)
        self.rho = d(cat(lambda p: p.rho))
        self.grad_rho = d(cat(lambda p: p.grad_rho))
        self.rho_x = d(cat(lambda p: p.rho_x))
        self.grad_rho_x = d(cat(lambda p: p.grad_rho_x))
        self.energy = torch.empty(len(self.problems), dtype=torch.float64, device=self.device)
        self.hess = torch.empty(sum(P * P for P in self.P), dtype=torch.float64, device=self.device)
        if tiles == "auto":
            from . import autotune
            cache = autotune.load_cache()
            tiles = [autotune.lookup(int(p.n_grid), int(p.n_atom), _prec_name(self.prec), cache)
                     or (0, 0) for p in self.problems]
        self.tiles = tiles
        b0 = self.problems[0]
        self.handle = vv10_batch_create(b0.b, b0.C, self.grid_off, self.atom_off, self.coords,
                                        self.weights, self.atom_of, self.rho, self.grad_rho,
                                        self.prec, tiles, stream)

    def run(self):
        vv10_batch_run(self.handle, self.rho_x, self.grad_rho_x, self.energy, self.hess)
        return self.energy, self.blocks()

    def blocks(self):
        out, off = [], 0
        for P in self.P:
            out.append(self.hess[off:off + P * P].view(P, P))
            off += P * P
        return out

    def info(self):
        return vv10_batch_info(self.handle)

    def close(self):
        if self.handle:
            vv10_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
