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
_LIB = os.path.join(_HERE, "liboracle.so")
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
        _lib.oracle_grid_vectors.argtypes = [i64, i32, P, P, P, P, P, d, d, P, P, P]
        _lib.oracle_grid_D.restype = ctypes.c_int
        _lib.oracle_grid_D.argtypes = [i64, i32, i64, i32, P, P, P, P, P, d, d, P]
        _lib.oracle_gradient.restype = ctypes.c_int
        _lib.oracle_gradient.argtypes = [i64, i32, P, P, P, P, P, d, d, P, P, P, P]
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


def gradient(atom_of, n_atom, coords, w, rho, gam, b, C, rho_x, gam_x, parts=False):
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
    return (out, pa) if parts else out


def hessian_terms(atom_of, n_atom, coords, w, rho, gam, b, C, rho_x, gam_x,
                  parts=False, resp=False):
    """H_nl = E_GG (no rho^{AB} term) + E_Ggr + E_Ggr^T + E_grgr, symmetrised.

    Returns (H, info) where info has 'asym' and optionally 'parts'
    ([3, P, P]: GG, Ggr + Ggr^T, grgr) and 'resp' (Yr, Yg as [P, n])."""
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
    if parts:
        info["parts"] = pa
    if resp:
        info["resp"] = (Yr, Yg)
    return H, info


def fock_nuclear_terms(atom_of, n_atom, coords, w, rho, gam, b, C, rho_x, gam_x):
    """Grid-level coefficients of the VV10 Fock nuclear derivative (Section II.B,
    the second line of F^A_{mu nu,G} and F^A_{mu nu,gr}; weight terms zero): for
    perturbation x = 3 B + a and point i,
      v_rho[x][i]   = sum_j w_j (f^{rho rho}_ij rho^x_j + f^{rho gamma}_ij gamma^x_j)
                      + E^{Bgr}_{i,a} + rho_i (kappa_r U^{Bgr}_{i,a} + omega_r W^{Bgr}_{i,a})
      v_gamma[x][i] = sum_j w_j (f^{gamma rho}_ij rho^x_j + f^{gamma gamma}_ij gamma^x_j)
                      + rho_i omega_g W^{Bgr}_{i,a}
    (the coefficients of w_i phi_mu phi_nu and of 2 w_i grad rho . grad(phi_mu phi_nu)),
    with the own-atom slot of E/U/W^{Bgr} from translational invariance."""
    n = len(w)
    Yr, Yg = response_rows(0, n, coords, w, rho, gam, b, C, rho_x, gam_x)
    E, U, W = grid_vectors(atom_of, n_atom, coords, w, rho, gam, b, C)
    kr, orr, og = np.zeros(n), np.zeros(n), np.zeros(n)
    for i in range(n):
        pt = point(b, C, float(rho[i]), float(gam[i]))
        kr[i], orr[i], og[i] = pt["kappa_r"], pt["omega_r"], pt["omega_g"]
    P = 3 * n_atom
    vr, vg = Yr.copy(), Yg.copy()
    for x in range(P):
        B, a = divmod(x, 3)
        vr[x] += E[:, B, a] + rho * (kr * U[:, B, a] + orr * W[:, B, a])
        vg[x] += rho * og * W[:, B, a]
    return vr, vg


def problem_inputs(p):
    """(gamma, gamma^x) of an inputs.Problem via the oracle's own definitions."""
    g = gamma(p.grad_rho)
    gx = gamma_x(p.grad_rho, p.grad_rho_x) if p.grad_rho_x is not None else None
    return g, gx
