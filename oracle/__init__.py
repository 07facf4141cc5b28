"""VV10 oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.

Thin ctypes wrapper over ``vv10_oracle.c``: a plain FP64 CPU evaluation of
the VV10 energy, potential and nuclear-Hessian grid terms written from the
equations of arXiv 2208.14639, Section II.  Only ``tests/``, the smoke check
and the benchmark's CPU-baseline leg may import this package.  It shares no
code with the HIP library.

Build: ``build()`` compiles ``liboracle.so`` with gcc (-O2, OpenMP, no FMA
contraction, no fast-math).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vv10_oracle.c")
# VV10_ORACLE_LIBRARY selects another build of the same source (the
# AddressSanitizer/UBSan build of build_sanitized(), for example)
_LIB = os.environ.get("VV10_ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
SAN_LIB = os.path.join(_HERE, "liboracle_san.so")
_lib = None

PT_FIELDS = ("omega", "kappa", "omega_r", "omega_g", "kappa_r", "omega_rr",
             "omega_rg", "omega_gg", "kappa_rr")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_sanitized() -> str:
    """The oracle built with clang's AddressSanitizer and UndefinedBehavior-
    Sanitizer (any report aborts), for the host sanitizer run of the CPU
    test suite; load it with VV10_ORACLE_LIBRARY and the ASan runtime
    preloaded."""
    cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall",
           "-o", SAN_LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(SAN_LIB + ".tmp", SAN_LIB)
    return SAN_LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        d, i64, i32, P = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        _lib.oracle_beta.restype = d
        _lib.oracle_beta.argtypes = [d]
        _lib.oracle_point.argtypes = [d, d, d, d, P]
        _lib.oracle_gamma.argtypes = [i64, P, P]
        _lib.oracle_gamma_x.argtypes = [i64, i32, P, P, P]
        _lib.oracle_pair_integrals.argtypes = [i64, P, P, P, P, d, d, P]
        _lib.oracle_energy_potential.argtypes = [i64, P, P, P, P, d, d, P, P, P, P]
        _lib.oracle_second_matrices.argtypes = [i64, P, P, P, P, d, d, P, P, P, P]
        _lib.oracle_response_rows.argtypes = [i64, i64, i64, P, P, P, P, d, d, i32, P, P, P, P]
        _lib.oracle_potential_rows.argtypes = [i64, i64, i64, P, P, P, P, d, d, P, P, P]
        _lib.oracle_grid_vectors.argtypes = [i64, i32, P, P, P, P, P, d, d, P, P, P]
        _lib.oracle_grid_D.restype = ctypes.c_int
        _lib.oracle_grid_D.argtypes = [i64, i32, i64, i32, P, P, P, P, P, d, d, P]
        _lib.oracle_gradient.restype = ctypes.c_int
        _lib.oracle_gradient.argtypes = [i64, i32, P, P, P, P, P, d, d, P, P, P, P]
        _lib.oracle_weight_integrals.argtypes = [i64, i64, i64, P, P, P, d, d, i32, P, P, P, P]
        _lib.oracle_hessian_terms.restype = ctypes.c_int
        _lib.oracle_hessian_terms.argtypes = [i64, i32, P, P, P, P, P, d, d, i32, P, P,
                                              P, P, P, P, P]
        _lib.oracle_num_threads.restype = ctypes.c_int
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def num_threads() -> int:
    return _load().oracle_num_threads()


def beta(b: float) -> float:
    return _load().oracle_beta(b)


def point(b, C, rho, gamma) -> dict:
    out = np.zeros(len(PT_FIELDS))
    _load().oracle_point(b, C, rho, gamma, _ptr(out))
    return dict(zip(PT_FIELDS, out))


def gamma(grad_rho):
    g = _f64(grad_rho)
    n = g.shape[0]
    out = np.zeros(n)
    _load().oracle_gamma(n, _ptr(g), _ptr(out))
    return out


def gamma_x(grad_rho, grad_rho_x):
    g = _f64(grad_rho)
    gx = _f64(grad_rho_x)
    P, n = gx.shape[0], gx.shape[1]
    out = np.zeros((P, n))
    _load().oracle_gamma_x(n, P, _ptr(g), _ptr(gx), _ptr(out))
    return out


def pair_integrals(coords, w, rho, gam, b, C):
    """[6, n]: E_i, U_i, W_i, A_i, B_i, C_i."""
    c, w, r, g = map(_f64, (coords, w, rho, gam))
    n = w.shape[0]
    out = np.zeros((6, n))
    _load().oracle_pair_integrals(n, _ptr(c), _ptr(w), _ptr(r), _ptr(g), b, C, _ptr(out))
    return out


def energy_potential(coords, w, rho, gam, b, C, with_integrals=False):
    c, w, r, g = map(_f64, (coords, w, rho, gam))
    n = w.shape[0]
    e = np.zeros(1)
    fr = np.zeros(n)
    fg = np.zeros(n)
    ints = np.zeros((6, n)) if with_integrals else None
    _load().oracle_energy_potential(n, _ptr(c), _ptr(w), _ptr(r), _ptr(g), b, C,
                                    _ptr(e), _ptr(fr), _ptr(fg), _ptr(ints))
    if with_integrals:
        return float(e[0]), fr, fg, ints
    return float(e[0]), fr, fg


def potential_rows(i0, i1, coords, w, rho, gam, b, C):
    """f^rho_i, f^gamma_i and the six inner integrals [6, k] of the rows
    i0 <= i < i1 only (Section II.A): O(k N) work, for sampled checks of
    large grids."""
    c, w, r, g = map(_f64, (coords, w, rho, gam))
    n = w.shape[0]
    ints = np.zeros((6, n))
    fr = np.zeros(n)
    fg = np.zeros(n)
    _load().oracle_potential_rows(i0, i1, n, _ptr(c), _ptr(w), _ptr(r), _ptr(g), b, C,
                                  _ptr(ints), _ptr(fr), _ptr(fg))
    return fr[i0:i1], fg[i0:i1], ints[:, i0:i1]


def second_matrices(coords, w, rho, gam, b, C):
    """f^{rho rho}, f^{gamma rho}, f^{rho gamma}, f^{gamma gamma} as n x n (tiny n)."""
    c, w, r, g = map(_f64, (coords, w, rho, gam))
    n = w.shape[0]
    mats = [np.zeros((n, n)) for _ in range(4)]
    _load().oracle_second_matrices(n, _ptr(c), _ptr(w), _ptr(r), _ptr(g), b, C,
                                   *[_ptr(m) for m in mats])
    return mats


def response_rows(i0, i1, coords, w, rho, gam, b, C, rho_x, gam_x):
    c, w, r, g, rx, gx = map(_f64, (coords, w, rho, gam, rho_x, gam_x))
    n = w.shape[0]
    P = rx.shape[0]
    Yr = np.zeros((P, n))
    Yg = np.zeros((P, n))
    _load().oracle_response_rows(i0, i1, n, _ptr(c), _ptr(w), _ptr(r), _ptr(g), b, C, P,
                                 _ptr(rx), _ptr(gx), _ptr(Yr), _ptr(Yg))
    return Yr[:, i0:i1], Yg[:, i0:i1]


def grid_vectors(atom_of, n_atom, coords, w, rho, gam, b, C):
    """E^{Bgr}_i, U^{Bgr}_i, W^{Bgr}_i as [n, n_atom, 3] each."""
    c, w, r, g = map(_f64, (coords, w, rho, gam))
    ao = np.ascontiguousarray(atom_of, dtype=np.int32)
    n = w.shape[0]
    E, U, W = (np.zeros((n, n_atom, 3)) for _ in range(3))
    _load().oracle_grid_vectors(n, n_atom, _ptr(ao), _ptr(c), _ptr(w), _ptr(r), _ptr(g),
                                b, C, _ptr(E), _ptr(U), _ptr(W))
    return E, U, W


def grid_D(i, B, atom_of, n_atom, coords, w, rho, gam, b, C):
    c, w, r, g = map(_f64, (coords, w, rho, gam))
    ao = np.ascontiguousarray(atom_of, dtype=np.int32)
    D = np.zeros(9)
    rc = _load().oracle_grid_D(i, B, w.shape[0], n_atom, _ptr(ao), _ptr(c), _ptr(w), _ptr(r),
                               _ptr(g), b, C, _ptr(D))
    if rc:
        raise ValueError(f"oracle_grid_D failed: {rc}")
    return D.reshape(3, 3)


def gradient(atom_of, n_atom, coords, w, rho, gam, b, C, rho_x, gam_x, parts=False, w_x=None):
    """E^A = E^A_G + E^A_gr (+ E^A_w when the weight derivatives w_x [P, n] are
    given; Section II.A).  parts: (E_G, E_gr[, E_w]) as rows."""
    c, w, r, g, rx, gx = map(_f64, (coords, w, rho, gam, rho_x, gam_x))
    ao = np.ascontiguousarray(atom_of, dtype=np.int32)
    n = w.shape[0]
    P = 3 * n_atom
    out = np.zeros(P)
    pa = np.zeros((2, P))
    rc = _load().oracle_gradient(n, n_atom, _ptr(ao), _ptr(c), _ptr(w), _ptr(r), _ptr(g),
                                 b, C, _ptr(rx), _ptr(gx), _ptr(out), _ptr(pa))
    if rc:
        raise ValueError(f"oracle_gradient failed: {rc}")
    if w_x is not None:
        Ew = _f64(w_x) @ weight_coefficients(c, w, r, g, b, C)
        out = out + Ew
        pa = np.concatenate([pa, Ew[None]])
    return (out, pa) if parts else out


def weight_coefficients(coords, w, rho, gam, b, C):
    """rho_i (beta + E_i): the coefficient of w^A_i in E^A_w and of w^{AB}_i in
    the first sum of E^{AB}_{w,w} (Sections II.A, II.B)."""
    E = pair_integrals(coords, w, rho, gam, b, C)[0]
    return _f64(rho) * (beta(b) + E)


def weight_integrals(coords, rho, gam, b, C, w_x, i0=0, i1=None):
    """E^{xw}_i, U^{xw}_i, W^{xw}_i for every column x of w_x and the rows
    i0 <= i < i1 (default all), each [P, i1 - i0] (Section II.B)."""
    c, r, g, wx = map(_f64, (coords, rho, gam, w_x))
    n = r.shape[0]
    i1 = n if i1 is None else i1
    P = wx.shape[0]
    Ew, Uw, Ww = (np.zeros((P, i1 - i0)) for _ in range(3))
    _load().oracle_weight_integrals(i0, i1, n, _ptr(c), _ptr(r), _ptr(g), b, C, P, _ptr(wx),
                                    _ptr(Ew), _ptr(Uw), _ptr(Ww))
    return Ew, Uw, Ww


def _partials(b, C, rho, gam):
    n = len(rho)
    kr, orr, og = np.zeros(n), np.zeros(n), np.zeros(n)
    for i in range(n):
        pt = point(b, C, float(rho[i]), float(gam[i]))
        kr[i], orr[i], og[i] = pt["kappa_r"], pt["omega_r"], pt["omega_g"]
    return kr, orr, og


def hessian_weight_terms(atom_of, n_atom, coords, w, rho, gam, b, C, rho_x, gam_x, w_x):
    """The weight terms of the nine-term Hessian split (Section II.B) other
    than the caller's sum_i w^{AB}_i rho_i (beta + E_i):
      E_ww  = sum_i w^A_i rho_i E^{Bw}_i                    (second sum of E_{w,w})
      E_Gw  = sum_i w^B_i (f^rho_i rho^A_i + f^gamma_i gamma^A_i)
            + sum_i w_i rho^A_i (E^{Bw}_i + rho_i (kappa_r U^{Bw}_i + omega_r W^{Bw}_i))
            + sum_i w_i gamma^A_i rho_i omega_g W^{Bw}_i
      E_wgr = sum_i w^A_i rho_i E^{Bgr}_i
    returned as E_ww + E_Gw + E_Gw^T + E_wgr + E_wgr^T, with the parts."""
    rho, w, wx = _f64(rho), _f64(w), _f64(w_x)
    n = len(w)
    P = wx.shape[0]
    _, fr, fg = energy_potential(coords, w, rho, gam, b, C)
    Ew, Uw, Ww = weight_integrals(coords, rho, gam, b, C, wx)
    Egr, _, _ = grid_vectors(atom_of, n_atom, coords, w, rho, gam, b, C)
    Egr_x = Egr.reshape(n, P).T                      # [x = (B, a), i]
    kr, orr, og = _partials(b, C, rho, gam)
    rx, gx = _f64(rho_x), _f64(gam_x)
    Eww = (wx * rho) @ Ew.T
    EGw = ((fr * rx + fg * gx) @ wx.T
           + (w * rx) @ (Ew + rho * (kr * Uw + orr * Ww)).T
           + (w * gx) @ (rho * og * Ww).T)
    Ewgr = (wx * rho) @ Egr_x.T
    return Eww + EGw + EGw.T + Ewgr + Ewgr.T, (Eww, EGw, Ewgr)


def weight_second_term(w_xy, coef):
    """sum_i w^{AB}_i rho_i (beta + E_i): the first sum of E_{w,w} (Section II.B),
    from the second nuclear derivatives of the weights [P, P, n] and
    weight_coefficients."""
    return _f64(w_xy) @ _f64(coef)


def hessian_terms(atom_of, n_atom, coords, w, rho, gam, b, C, rho_x, gam_x,
                  parts=False, resp=False, w_x=None):
    """H_nl = E_GG (no rho^{AB} term) + E_Ggr + E_Ggr^T + E_grgr, symmetrised,
    plus, when the weight derivatives w_x [P, n] are given, the weight terms
    of hessian_weight_terms (no w^{AB} term).

    Returns (H, info) where info has 'asym' and optionally 'parts'
    ([3, P, P]: GG, Ggr + Ggr^T, grgr; with w_x also 'wparts': E_ww, E_Gw,
    E_wgr) and 'resp' (Yr, Yg as [P, n])."""
    c, w, r, g, rx, gx = map(_f64, (coords, w, rho, gam, rho_x, gam_x))
    ao = np.ascontiguousarray(atom_of, dtype=np.int32)
    n = w.shape[0]
    P = rx.shape[0]
    H = np.zeros((P, P))
    pa = np.zeros((3, P, P)) if parts else None
    Yr = np.zeros((P, n)) if resp else None
    Yg = np.zeros((P, n)) if resp else None
    asym = np.zeros(1)
    rc = _load().oracle_hessian_terms(n, n_atom, _ptr(ao), _ptr(c), _ptr(w), _ptr(r), _ptr(g),
                                      b, C, P, _ptr(rx), _ptr(gx), _ptr(H), _ptr(pa),
                                      _ptr(Yr), _ptr(Yg), _ptr(asym))
    if rc:
        raise ValueError(f"oracle_hessian_terms failed: {rc}")
    info = {"asym": float(asym[0])}
    if w_x is not None:
        HW, wparts = hessian_weight_terms(atom_of, n_atom, coords, w, rho, gam, b, C, rho_x,
                                          gam_x, w_x)
        H = H + 0.5 * (HW + HW.T)
        if parts:
            info["wparts"] = wparts
    if parts:
        info["parts"] = pa
    if resp:
        info["resp"] = (Yr, Yg)
    return H, info


def fock_nuclear_terms(atom_of, n_atom, coords, w, rho, gam, b, C, rho_x, gam_x, w_x=None):
    """Grid-level coefficients of the VV10 Fock nuclear derivative (Section II.B,
    the second line of F^A_{mu nu,G} and F^A_{mu nu,gr}; weight terms zero): for
    perturbation x = 3 B + a and point i,
      v_rho[x][i]   = sum_j w_j (f^{rho rho}_ij rho^x_j + f^{rho gamma}_ij gamma^x_j)
                      + E^{Bgr}_{i,a} + rho_i (kappa_r U^{Bgr}_{i,a} + omega_r W^{Bgr}_{i,a})
      v_gamma[x][i] = sum_j w_j (f^{gamma rho}_ij rho^x_j + f^{gamma gamma}_ij gamma^x_j)
                      + rho_i omega_g W^{Bgr}_{i,a}
    (the coefficients of w_i phi_mu phi_nu and of 2 w_i grad rho . grad(phi_mu phi_nu)),
    with the own-atom slot of E/U/W^{Bgr} from translational invariance.
    With the weight derivatives w_x, the F^A_w coefficients of the same two
    products are added (its second and third lines):
      v_rho   += E^{xw}_i + rho_i (kappa_r U^{xw}_i + omega_r W^{xw}_i)
      v_gamma += rho_i omega_g W^{xw}_i
    (its first line, w^x_i times f^rho_i and f^gamma_i, belongs to the caller)."""
    n = len(w)
    Yr, Yg = response_rows(0, n, coords, w, rho, gam, b, C, rho_x, gam_x)
    E, U, W = grid_vectors(atom_of, n_atom, coords, w, rho, gam, b, C)
    kr, orr, og = _partials(b, C, rho, gam)
    P = 3 * n_atom
    vr, vg = Yr.copy(), Yg.copy()
    for x in range(P):
        B, a = divmod(x, 3)
        vr[x] += E[:, B, a] + rho * (kr * U[:, B, a] + orr * W[:, B, a])
        vg[x] += rho * og * W[:, B, a]
    if w_x is not None:
        Ew, Uw, Ww = weight_integrals(coords, rho, gam, b, C, w_x)
        vr += Ew + rho * (kr * Uw + orr * Ww)
        vg += rho * og * Ww
    return vr, vg


def problem_inputs(p):
    """(gamma, gamma^x) of an inputs.Problem via the oracle's own definitions."""
    g = gamma(p.grad_rho)
    gx = gamma_x(p.grad_rho, p.grad_rho_x) if p.grad_rho_x is not None else None
    return g, gx
