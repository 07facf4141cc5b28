"""Seeded synthetic inputs for the VV10 double-grid sums.

This module only builds *problems*: water-cluster geometries, an
atom-centred Monte-Carlo quadrature grid, a model density with its analytic
gradient, and the analytic nuclear derivatives of that density on grid points
that move with their owning atom.  It holds none of the VV10 arithmetic
(no omega, kappa, Phi or any sum over grid pairs); both the HIP library and
the CPU oracle take what is built here as plain arrays.

Recipe (atomic units, bohr):
  * water monomer: r(OH) = 0.96 Angstrom, angle HOH = 104.5 degrees, rotated by
    a uniform random rotation; atoms ordered O, H, H per molecule;
  * clusters: the first O at the origin; each further O is placed at
    2.9 +- 0.1 Angstrom from a randomly chosen existing O in a uniformly random
    direction, rejected when it comes within 2.6 Angstrom of another O or when
    any of its atoms comes within 1.0 Angstrom of an atom of another molecule;
  * grid: n_pa points per atom at R_A + r u with ln r uniform on
    [ln 0.05, ln 10] and u uniform on the unit sphere; points are stored
    grouped by owning atom (atom_of is nondecreasing), within an atom in
    sampling order or (radial_order) by increasing radius;
  * weights, two kinds:
    - "atomic" (default): w = 1/(N q(r)) with q(r) = 1/(4 pi r^3 ln(10/0.05))
      the three-dimensional density of one atom's sampler and N the total
      number of points, so each atom's point set is an unbiased estimate of
      the whole-space integral and the sets are averaged.  w depends only on
      the distance to the owner atom, so it has no nuclear derivatives;
    - "becke": Becke's fuzzy-cell partition (A. D. Becke, J. Chem. Phys. 88,
      2547 (1988), equal atomic sizes): w_i = 1/(n_A q(r)) P_A(r_i) /
      sum_C P_C(r_i) for a point of atom A with n_A points, where
      P_C(r) = prod_{D != C} s(mu_CD), mu_CD = (|r - R_C| - |r - R_D|)/|R_C - R_D|,
      s(mu) = (1 - f(f(f(mu))))/2 and f(x) = 3x/2 - x^3/2.  Each atom's set
      integrates its own cell.  These weights move with every nucleus; their
      first and second nuclear derivatives (grid points moving with their
      owner atoms) come from a forward-mode evaluation of the same formula
      that carries exact derivatives through every operation;
  * density: rho(r) = sum_A Z_A zeta_A^3/pi exp(-2 zeta_A |r - R_A|) with
    zeta_O = 2, zeta_H = 1 and analytic gradient;
  * nuclear derivatives: the total derivative of rho(r_i) and grad rho(r_i)
    with respect to nucleus A's coordinates when grid point i moves rigidly
    with its owner atom O(i):
        d rho(r_i)/dR_A = sum_C grad f_C(r_i - R_C) (delta_{A,O(i)} - delta_{A,C}),
    and likewise for the gradient with the Hessian of f_C.  Perturbation
    index x = 3 A + alpha.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BOHR_PER_ANGSTROM = 1.8897261245650618
R_MIN, R_MAX = 0.05, 10.0
ZETA = {8: 2.0, 1: 1.0}
VV10_B = 6.0
VV10_C = 0.01

# Sizes of the five standard workloads (waters, points per atom).
WORKLOADS = {
    "water_dimer": dict(n_water=2, n_pa=700, seed=1001),
    "water_hexamer": dict(n_water=6, n_pa=1500, seed=1002),
    "water_20mer": dict(n_water=20, n_pa=2000, seed=1003),
}


@dataclasses.dataclass
class Molecule:
    Z: np.ndarray      # [n_atom] int
    zeta: np.ndarray   # [n_atom] float64
    R: np.ndarray      # [n_atom, 3] bohr

    @property
    def n_atom(self) -> int:
        return int(self.Z.shape[0])


@dataclasses.dataclass
class Problem:
    mol: Molecule
    atom_of: np.ndarray     # [N] int32, nondecreasing
    offsets: np.ndarray     # [N, 3] point position relative to its owner atom
    coords: np.ndarray      # [N, 3]
    weights: np.ndarray     # [N]
    rho: np.ndarray         # [N]
    grad_rho: np.ndarray    # [N, 3]
    radii: np.ndarray       # [N] distance of each point to its owner atom
    rho_x: np.ndarray | None = None       # [P, N]
    grad_rho_x: np.ndarray | None = None  # [P, N, 3]
    weight_kind: str = "atomic"
    w_x: np.ndarray | None = None         # [P, N] weight derivatives (becke only)
    w_xy: np.ndarray | None = None        # [P, P, N] second derivatives (on request)
    b: float = VV10_B
    C: float = VV10_C
    seed: int = 0

    @property
    def n_grid(self) -> int:
        return int(self.weights.shape[0])

    @property
    def n_atom(self) -> int:
        return self.mol.n_atom

    @property
    def n_pert(self) -> int:
        return 3 * self.mol.n_atom


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_monomer(rng: np.random.Generator) -> np.ndarray:
    """O, H, H positions (bohr) of one water with O at the origin."""
    r = 0.96 * BOHR_PER_ANGSTROM
    half = math.radians(104.5) / 2
    local = np.array([[0.0, 0.0, 0.0],
                      [r * math.sin(half), 0.0, r * math.cos(half)],
                      [-r * math.sin(half), 0.0, r * math.cos(half)]])
    return local @ _random_rotation(rng).T


def water_cluster(n_water: int, rng: np.random.Generator) -> Molecule:
    ang = BOHR_PER_ANGSTROM
    mols = [water_monomer(rng)]
    tries = 0
    while len(mols) < n_water:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place waters")
        anchor = mols[rng.integers(len(mols))][0]
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        o = anchor + (2.9 + rng.uniform(-0.1, 0.1)) * ang * d
        others_o = np.array([m[0] for m in mols])
        if np.min(np.linalg.norm(others_o - o, axis=1)) < 2.6 * ang - 1e-9:
            continue
        cand = water_monomer(rng) + o
        others = np.concatenate(mols)
        dd = np.linalg.norm(cand[:, None, :] - others[None, :, :], axis=2)
        if dd.min() < 1.0 * ang:
            continue
        mols.append(cand)
    R = np.concatenate(mols)
    Z = np.tile(np.array([8, 1, 1]), n_water)
    zeta = np.array([ZETA[int(z)] for z in Z])
    return Molecule(Z=Z, zeta=zeta, R=R)


def atom_grid(n_atom: int, n_pa: int, rng: np.random.Generator, radial_order: bool = False):
    """Per-atom sampler: returns (atom_of, offsets, radii).  With radial_order
    each atom's points are stored by increasing radius (the shell order of
    atom-centred product grids); the sample itself is the same."""
    lr = rng.uniform(math.log(R_MIN), math.log(R_MAX), size=(n_atom, n_pa))
    r = np.exp(lr)
    u = rng.standard_normal((n_atom, n_pa, 3))
    u /= np.linalg.norm(u, axis=2, keepdims=True)
    if radial_order:
        k = np.argsort(r, axis=1, kind="stable")
        r = np.take_along_axis(r, k, axis=1)
        u = np.take_along_axis(u, k[..., None], axis=1)
    offsets = (r[..., None] * u).reshape(-1, 3)
    atom_of = np.repeat(np.arange(n_atom, dtype=np.int32), n_pa)
    return atom_of, offsets, r.reshape(-1)


def grid_weights(radii: np.ndarray) -> np.ndarray:
    n = radii.shape[0]
    return 4.0 * math.pi * radii ** 3 * math.log(R_MAX / R_MIN) / n


class _Jet:
    """A field over the grid points with its derivatives with respect to the
    3 n_atom nuclear coordinates: value v [N], gradient g [N, P] (order >= 1)
    and Hessian h [N, P, P] (order 2).  A leading dimension of 1 broadcasts
    over the points (quantities that do not depend on the point)."""

    __slots__ = ("v", "g", "h")

    def __init__(self, v, g=None, h=None):
        self.v, self.g, self.h = v, g, h

    def __add__(self, o):
        return _Jet(self.v + o.v, None if self.g is None else self.g + o.g,
                    None if self.h is None else self.h + o.h)

    def __sub__(self, o):
        return _Jet(self.v - o.v, None if self.g is None else self.g - o.g,
                    None if self.h is None else self.h - o.h)

    def __mul__(self, o):
        v = self.v * o.v
        g = h = None
        if self.g is not None:
            g = self.v[:, None] * o.g + o.v[:, None] * self.g
        if self.h is not None:
            h = (self.v[:, None, None] * o.h + o.v[:, None, None] * self.h
                 + self.g[:, :, None] * o.g[:, None, :] + o.g[:, :, None] * self.g[:, None, :])
        return _Jet(v, g, h)

    def chain(self, f, fp, fpp):
        """F(self) for a scalar function with values f, F' = fp, F'' = fpp at self.v."""
        g = h = None
        if self.g is not None:
            g = fp[:, None] * self.g
        if self.h is not None:
            h = fp[:, None, None] * self.h + fpp[:, None, None] * (self.g[:, :, None] * self.g[:, None, :])
        return _Jet(f, g, h)

    def recip(self):
        iv = 1.0 / self.v
        return self.chain(iv, -iv * iv, 2.0 * iv * iv * iv)

    def rows(self, idx):
        return _Jet(self.v[idx], None if self.g is None else self.g[idx],
                    None if self.h is None else self.h[idx])


def _distance_jet(d: np.ndarray, sel: np.ndarray, order: int) -> _Jet:
    """|d| for d = X - Y with dX/dR_A - dY/dR_A = sel[:, A] I: d [K, 3],
    sel [K, n_atom] in {-1, 0, 1}."""
    u = np.sqrt(np.einsum("ka,ka->k", d, d))
    if order == 0:
        return _Jet(u)
    e = d / u[:, None]
    K, M = sel.shape
    g = (sel[:, :, None] * e[:, None, :]).reshape(K, 3 * M)
    h = None
    if order >= 2:
        T = (np.eye(3)[None] - e[:, :, None] * e[:, None, :]) / u[:, None, None]
        h = np.einsum("ka,kb,kxy->kaxby", sel, sel, T).reshape(K, 3 * M, 3 * M)
    return _Jet(u, g, h)


def _becke_step(mu: np.ndarray):
    """s(mu) = (1 - f(f(f(mu))))/2 with f(x) = 3x/2 - x^3/2, and s', s''."""
    f = lambda x: x * (1.5 - 0.5 * x * x)
    fp = lambda x: 1.5 - 1.5 * x * x
    fpp = lambda x: -3.0 * x
    x1 = f(mu)
    x2 = f(x1)
    x3 = f(x2)
    d1 = fp(x2) * fp(x1) * fp(mu)
    d2 = fpp(x2) * (fp(x1) * fp(mu)) ** 2 + fp(x2) * (fpp(x1) * fp(mu) ** 2 + fp(x1) * fpp(mu))
    return 0.5 * (1.0 - x3), -0.5 * d1, -0.5 * d2


def _becke_order1(mol: Molecule, atom_of: np.ndarray, pts: np.ndarray):
    """Becke partition P_O(i)(r_i) / sum_C P_C(r_i) of every point and its first
    nuclear derivatives, [N] and [M, 3, N].  Each cell function's derivative
    comes from its logarithmic derivative d ln P_C = sum_D (s'/s)(mu_CD) d mu_CD,
    where mu_CD depends only on R_{O(i)}, R_C and R_D (three atoms per pair).
    A factor s that rounds to zero has s' = 0 as well (s is flat at mu = 1)
    and makes P_C and its derivative zero."""
    M = mol.n_atom
    N = atom_of.shape[0]
    seg = np.searchsorted(atom_of, np.arange(M + 1))
    d = [(pts - mol.R[C]).T.copy() for C in range(M)]                # [3, N]
    u = [np.sqrt(np.einsum("an,an->n", x, x)) for x in d]
    e = [d[C] / u[C] for C in range(M)]
    Zv = np.zeros(N)
    Zg = np.zeros((M, 3, N))
    ownv = np.zeros(N)
    owng = np.zeros((M, 3, N))
    for C in range(M):
        v = np.ones(N)
        L = np.zeros((M, 3, N))
        Lown = np.zeros((3, N))          # the owner atom's slot, added per segment below
        for D in range(M):
            if D == C:
                continue
            dd = mol.R[C] - mol.R[D]
            dist = math.sqrt(float(dd @ dd))
            nCD = (dd / dist)[:, None]
            mu = (u[C] - u[D]) / dist
            s, sp, _ = _becke_step(mu)
            c = np.divide(sp, s, out=np.zeros(N), where=s > 0.0) / dist
            # d mu / dR_A = (sel_C[A] e_C - sel_D[A] e_D)/|R_CD| - mu (delta_AC - delta_AD) n_CD/|R_CD|
            # with sel_X[A] = delta_{A,O(i)} - delta_{A,X}
            Lown += c * (e[C] - e[D])
            t = c * mu * nCD
            L[C] -= c * e[C] + t
            L[D] += c * e[D] + t
            v = v * s
        for A in range(M):
            L[A, :, seg[A]:seg[A + 1]] += Lown[:, seg[A]:seg[A + 1]]
        g = v * L
        Zv += v
        Zg += g
        ownv[seg[C]:seg[C + 1]] = v[seg[C]:seg[C + 1]]
        owng[:, :, seg[C]:seg[C + 1]] = g[:, :, seg[C]:seg[C + 1]]
    part = ownv / Zv
    dpart = (owng - part * Zg) / Zv
    return part, dpart


def becke_weights(mol: Molecule, atom_of: np.ndarray, offsets: np.ndarray,
                  radii: np.ndarray, order: int = 0, jets: bool = False):
    """Becke-partitioned weights of points r_i = R_{O(i)} + offsets_i and their
    total nuclear derivatives: (w [N], w_x [P, N] or None, w_xy [P, P, N] or None)
    for order 0, 1, 2.  Order 1 uses the sparse structure of mu_CD unless
    jets is set (then the general forward-mode path, as for order 2)."""
    M = mol.n_atom
    N = atom_of.shape[0]
    pts = mol.R[atom_of] + offsets
    counts = np.bincount(atom_of, minlength=M)
    w_rad = 4.0 * math.pi * radii ** 3 * math.log(R_MAX / R_MIN) / counts[atom_of]
    if order == 1 and not jets:
        part, dpart = _becke_order1(mol, atom_of, pts)
        return w_rad * part, np.ascontiguousarray((w_rad * dpart).reshape(3 * M, N)), None
    owner = np.zeros((N, M))
    owner[np.arange(N), atom_of] = 1.0
    u = []
    for C in range(M):
        sel = owner.copy()
        sel[:, C] -= 1.0
        u.append(_distance_jet(pts - mol.R[C], sel, order))
    cell = []
    for C in range(M):
        PC = _Jet(np.ones(N), np.zeros((N, 3 * M)) if order >= 1 else None,
                  np.zeros((N, 3 * M, 3 * M)) if order >= 2 else None)
        for D in range(M):
            if D == C:
                continue
            sel = np.zeros((1, M))
            sel[0, C], sel[0, D] = 1.0, -1.0
            dCD = _distance_jet((mol.R[C] - mol.R[D])[None], sel, order)
            mu = (u[C] - u[D]) * dCD.recip()
            PC = PC * mu.chain(*_becke_step(mu.v))
        cell.append(PC)
    Z = cell[0]
    for C in range(1, M):
        Z = Z + cell[C]
    own = _Jet(np.empty(N), np.empty((N, 3 * M)) if order >= 1 else None,
               np.empty((N, 3 * M, 3 * M)) if order >= 2 else None)
    for C in range(M):
        idx = np.nonzero(atom_of == C)[0]
        r = cell[C].rows(idx)
        own.v[idx] = r.v
        if order >= 1:
            own.g[idx] = r.g
        if order >= 2:
            own.h[idx] = r.h
    wj = (own * Z.recip())
    w = w_rad * wj.v
    w_x = None if order < 1 else np.ascontiguousarray((w_rad[:, None] * wj.g).T)
    w_xy = None if order < 2 else np.ascontiguousarray(np.moveaxis(w_rad[:, None, None] * wj.h, 0, 2))
    return w, w_x, w_xy


def _slater_terms(mol: Molecule, A: int, pts: np.ndarray, order: int):
    """Value, gradient and (order >= 2) Hessian of f_A(r) = Z z^3/pi e^{-2 z |r - R_A|}."""
    z = mol.zeta[A]
    d = pts - mol.R[A]
    r = np.linalg.norm(d, axis=1)
    r = np.maximum(r, 1e-300)
    f = mol.Z[A] * z ** 3 / math.pi * np.exp(-2.0 * z * r)
    n = d / r[:, None]
    g = (-2.0 * z * f)[:, None] * n
    if order < 2:
        return f, g, None
    # d2f/dr_a dr_b = f [4 z^2 n_a n_b - 2 z (delta_ab - n_a n_b)/r]
    nn = n[:, :, None] * n[:, None, :]
    eye = np.eye(3)[None]
    H = f[:, None, None] * (4.0 * z * z * nn - (2.0 * z / r)[:, None, None] * (eye - nn))
    return f, g, H


def model_density(mol: Molecule, pts: np.ndarray, hessian: bool = False):
    rho = np.zeros(pts.shape[0])
    grad = np.zeros((pts.shape[0], 3))
    hess = np.zeros((pts.shape[0], 3, 3)) if hessian else None
    for A in range(mol.n_atom):
        f, g, H = _slater_terms(mol, A, pts, 2 if hessian else 1)
        rho += f
        grad += g
        if hessian:
            hess += H
    return rho, grad, hess


def density_derivatives(mol: Molecule, atom_of: np.ndarray, pts: np.ndarray):
    """rho^x [P, N] and (grad rho)^x [P, N, 3] for all P = 3 n_atom perturbations."""
    n = pts.shape[0]
    na = mol.n_atom
    _, grad, hess = model_density(mol, pts, hessian=True)
    rho_x = np.zeros((3 * na, n))
    grad_x = np.zeros((3 * na, n, 3))
    for A in range(na):
        _, gA, HA = _slater_terms(mol, A, pts, 2)
        own = (atom_of == A)
        for a in range(3):
            x = 3 * A + a
            rho_x[x] = -gA[:, a]
            rho_x[x, own] += grad[own, a]
            grad_x[x] = -HA[:, a, :]
            grad_x[x, own] += hess[own, a, :]
    return rho_x, grad_x


def build_problem(mol: Molecule, atom_of, offsets, radii, with_derivatives=True,
                  seed=0, weights: str = "atomic", weight_hessian: bool = False) -> Problem:
    """weights = "atomic" or "becke"; for "becke" with derivatives, w_x (and,
    with weight_hessian, w_xy) are filled."""
    coords = mol.R[atom_of] + offsets
    atom_of = np.ascontiguousarray(atom_of, dtype=np.int32)
    w_x = w_xy = None
    if weights == "atomic":
        w = grid_weights(radii)
    elif weights == "becke":
        order = 0 if not with_derivatives else (2 if weight_hessian else 1)
        w, w_x, w_xy = becke_weights(mol, atom_of, offsets, radii, order)
    else:
        raise ValueError(f"unknown weight kind {weights!r}")
    rho, grad, _ = model_density(mol, coords)
    p = Problem(mol=mol, atom_of=atom_of,
                offsets=offsets, coords=np.ascontiguousarray(coords), weights=w,
                rho=rho, grad_rho=np.ascontiguousarray(grad), radii=radii, seed=seed,
                weight_kind=weights, w_x=w_x, w_xy=w_xy)
    if with_derivatives:
        rx, gx = density_derivatives(mol, p.atom_of, coords)
        p.rho_x = np.ascontiguousarray(rx)
        p.grad_rho_x = np.ascontiguousarray(gx)
    return p


def make_problem(n_water: int, n_pa: int, seed: int, with_derivatives=True,
                 weights: str = "atomic", weight_hessian: bool = False,
                 radial_order: bool = False) -> Problem:
    rng = np.random.default_rng(seed)
    mol = water_cluster(n_water, rng)
    atom_of, offsets, radii = atom_grid(mol.n_atom, n_pa, rng, radial_order)
    return build_problem(mol, atom_of, offsets, radii, with_derivatives, seed, weights,
                         weight_hessian)


def device_fields(mol: Molecule, atom_of, coords, torch, device):
    """rho [N], grad rho [N, 3], rho^x [P, N] and (grad rho)^x [P, N, 3] of
    the model density evaluated with torch on `device` (the same formulas as
    model_density and density_derivatives; a GPU builds a large problem in
    milliseconds).  atom_of and coords are host arrays."""
    f64 = torch.float64
    X = torch.as_tensor(np.ascontiguousarray(coords), dtype=f64).to(device)
    own_of = torch.as_tensor(np.asarray(atom_of, dtype=np.int64)).to(device)
    n, na = X.shape[0], mol.n_atom
    eye = torch.eye(3, dtype=f64, device=device)
    terms = []
    rho = torch.zeros(n, dtype=f64, device=device)
    grad = torch.zeros((n, 3), dtype=f64, device=device)
    hess = torch.zeros((n, 3, 3), dtype=f64, device=device)
    for A in range(na):
        z = float(mol.zeta[A])
        d = X - torch.as_tensor(mol.R[A], dtype=f64, device=device)
        r = torch.clamp(torch.linalg.vector_norm(d, dim=1), min=1e-300)
        f = float(mol.Z[A]) * z ** 3 / math.pi * torch.exp(-2.0 * z * r)
        u = d / r[:, None]
        g = (-2.0 * z * f)[:, None] * u
        uu = u[:, :, None] * u[:, None, :]
        H = f[:, None, None] * (4.0 * z * z * uu - (2.0 * z / r)[:, None, None] * (eye - uu))
        rho += f
        grad += g
        hess += H
        terms.append((g, H))
    rho_x = torch.empty((3 * na, n), dtype=f64, device=device)
    grad_x = torch.empty((3 * na, n, 3), dtype=f64, device=device)
    for A, (gA, HA) in enumerate(terms):
        own = (own_of == A).to(f64)
        for a in range(3):
            rho_x[3 * A + a] = -gA[:, a] + own * grad[:, a]
            grad_x[3 * A + a] = -HA[:, a, :] + own[:, None] * hess[:, a, :]
    return rho, grad, rho_x, grad_x


def make_problem_on_device(n_water: int, n_pa: int, seed: int, torch, device) -> Problem:
    """make_problem's molecule and grid (same seed, same sample) with the
    density and its nuclear derivatives built on `device` (device_fields):
    rho, grad_rho, rho_x and grad_rho_x are torch tensors there; coords,
    weights and atom_of stay host arrays."""
    rng = np.random.default_rng(seed)
    mol = water_cluster(n_water, rng)
    atom_of, offsets, radii = atom_grid(mol.n_atom, n_pa, rng)
    coords = np.ascontiguousarray(mol.R[atom_of] + offsets)
    rho, grad, rho_x, grad_x = device_fields(mol, atom_of, coords, torch, device)
    return Problem(mol=mol, atom_of=np.ascontiguousarray(atom_of, dtype=np.int32),
                   offsets=offsets, coords=coords, weights=grid_weights(radii), rho=rho,
                   grad_rho=grad, radii=radii, rho_x=rho_x, grad_rho_x=grad_x, seed=seed)


def make_workload(name: str, with_derivatives=True, weights: str = "atomic",
                  radial_order: bool = False) -> Problem:
    cfg = WORKLOADS[name]
    return make_problem(cfg["n_water"], cfg["n_pa"], cfg["seed"], with_derivatives, weights,
                        radial_order=radial_order)


def displaced(p: Problem, atom: int, axis: int, h: float, with_derivatives=False) -> Problem:
    """The same problem with nucleus `atom` moved by h along `axis`; its grid
    points move with it.  Atomic weights stay the same; Becke weights are
    re-evaluated at the new geometry."""
    R = p.mol.R.copy()
    R[atom, axis] += h
    mol = Molecule(Z=p.mol.Z, zeta=p.mol.zeta, R=R)
    return build_problem(mol, p.atom_of, p.offsets, p.radii, with_derivatives, p.seed,
                         p.weight_kind)


def trial_densities(p: Problem, n_t: int, seed: int, scale: float = 0.2):
    """n_t seeded trial densities with analytic gradients, [n_t, N] and [n_t, N, 3].

    Each is sum_A (c_tA + (r - R_A) . v_tA) f_A(r), with f_A the atom's term of
    the model density and c_tA, v_tA normal with standard deviation `scale`:
    charge moved between atoms and each atom polarised, the shapes a
    first-order density response takes.  Values of either sign."""
    rng = np.random.default_rng(seed)
    mol = p.mol
    n = p.n_grid
    c = rng.standard_normal((n_t, mol.n_atom)) * scale
    v = rng.standard_normal((n_t, mol.n_atom, 3)) * scale
    rt = np.zeros((n_t, n))
    gt = np.zeros((n_t, n, 3))
    for A in range(mol.n_atom):
        f, g, _ = _slater_terms(mol, A, p.coords, 1)
        d = p.coords - mol.R[A]
        s = c[:, A][:, None] + v[:, A, :] @ d.T              # [n_t, N]
        rt += s * f[None, :]
        gt += s[:, :, None] * g[None, :, :] + f[None, :, None] * v[:, A, None, :]
    return np.ascontiguousarray(rt), np.ascontiguousarray(gt)


def random_cluster_sizes(n_mol: int, seed: int, lo: int = 1, hi: int = 30):
    rng = np.random.default_rng(seed)
    return [int(k) for k in rng.integers(lo, hi + 1, size=n_mol)]
