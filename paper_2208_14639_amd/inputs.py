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
    grouped by owning atom (atom_of is nondecreasing);
  * weights: w = 1/(N q(r)) with q(r) = 1/(4 pi r^3 ln(10/0.05)) the
    three-dimensional density of one atom's sampler and N the total number of
    points, so each atom's point set is an unbiased estimate of the
    whole-space integral and the sets are averaged;
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


def atom_grid(n_atom: int, n_pa: int, rng: np.random.Generator):
    """Per-atom sampler: returns (atom_of, offsets, radii)."""
    lr = rng.uniform(math.log(R_MIN), math.log(R_MAX), size=(n_atom, n_pa))
    r = np.exp(lr)
    u = rng.standard_normal((n_atom, n_pa, 3))
    u /= np.linalg.norm(u, axis=2, keepdims=True)
    offsets = (r[..., None] * u).reshape(-1, 3)
    atom_of = np.repeat(np.arange(n_atom, dtype=np.int32), n_pa)
    return atom_of, offsets, r.reshape(-1)


def grid_weights(radii: np.ndarray) -> np.ndarray:
    n = radii.shape[0]
    return 4.0 * math.pi * radii ** 3 * math.log(R_MAX / R_MIN) / n


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
                  seed=0) -> Problem:
    coords = mol.R[atom_of] + offsets
    w = grid_weights(radii)
    rho, grad, _ = model_density(mol, coords)
    p = Problem(mol=mol, atom_of=np.ascontiguousarray(atom_of, dtype=np.int32),
                offsets=offsets, coords=np.ascontiguousarray(coords), weights=w,
                rho=rho, grad_rho=np.ascontiguousarray(grad), radii=radii, seed=seed)
    if with_derivatives:
        rx, gx = density_derivatives(mol, p.atom_of, coords)
        p.rho_x = np.ascontiguousarray(rx)
        p.grad_rho_x = np.ascontiguousarray(gx)
    return p


def make_problem(n_water: int, n_pa: int, seed: int, with_derivatives=True) -> Problem:
    rng = np.random.default_rng(seed)
    mol = water_cluster(n_water, rng)
    atom_of, offsets, radii = atom_grid(mol.n_atom, n_pa, rng)
    return build_problem(mol, atom_of, offsets, radii, with_derivatives, seed)


def make_workload(name: str, with_derivatives=True) -> Problem:
    cfg = WORKLOADS[name]
    return make_problem(cfg["n_water"], cfg["n_pa"], cfg["seed"], with_derivatives)


def displaced(p: Problem, atom: int, axis: int, h: float, with_derivatives=False) -> Problem:
    """The same problem with nucleus `atom` moved by h along `axis`; its grid
    points move with it and every weight stays the same."""
    R = p.mol.R.copy()
    R[atom, axis] += h
    mol = Molecule(Z=p.mol.Z, zeta=p.mol.zeta, R=R)
    return build_problem(mol, p.atom_of, p.offsets, p.radii, with_derivatives, p.seed)


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
