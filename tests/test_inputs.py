"""Checks of the seeded problem generator (no VV10 arithmetic here)."""
import dataclasses

import numpy as np
import pytest

from paper_2208_14639_amd import inputs


def test_deterministic_by_seed():
    a = inputs.make_problem(2, 20, 5)
    b = inputs.make_problem(2, 20, 5)
    c = inputs.make_problem(2, 20, 6)
    assert np.array_equal(a.coords, b.coords) and np.array_equal(a.rho_x, b.rho_x)
    assert not np.array_equal(a.coords, c.coords)


def test_shapes_and_ordering(small_dimer):
    p = small_dimer
    assert p.n_grid == 360 and p.n_pert == 18
    assert p.rho_x.shape == (18, 360) and p.grad_rho_x.shape == (18, 360, 3)
    assert np.all(np.diff(p.atom_of) >= 0)
    assert np.all(p.weights > 0) and np.all(p.rho > 0)
    r = np.linalg.norm(p.coords - p.mol.R[p.atom_of], axis=1)
    assert np.all(r >= inputs.R_MIN * (1 - 1e-12)) and np.all(r <= inputs.R_MAX * (1 + 1e-12))


def test_water_geometry():
    rng = np.random.default_rng(3)
    m = inputs.water_cluster(6, rng)
    ang = inputs.BOHR_PER_ANGSTROM
    for k in range(6):
        O, H1, H2 = m.R[3 * k:3 * k + 3]
        assert abs(np.linalg.norm(H1 - O) - 0.96 * ang) < 1e-12
        cosang = np.dot(H1 - O, H2 - O) / np.linalg.norm(H1 - O) / np.linalg.norm(H2 - O)
        assert abs(np.degrees(np.arccos(cosang)) - 104.5) < 1e-9
    Os = m.R[0::3]
    d = np.linalg.norm(Os[:, None] - Os[None], axis=2) + np.eye(6) * 100
    assert d.min() >= 2.6 * ang - 1e-9


def test_weights_integrate_density():
    """Monte-Carlo estimate of the electron count: sum_i w_i rho_i ~ 20 for a dimer."""
    p = inputs.make_workload("water_dimer", with_derivatives=False)
    n_el = float(np.dot(p.weights, p.rho))
    assert 10.0 < n_el < 30.0


def test_gradient_matches_fd(small_dimer):
    p = small_dimer
    h = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        rp, _, _ = inputs.model_density(p.mol, p.coords + e)
        rm, _, _ = inputs.model_density(p.mol, p.coords - e)
        fd = (rp - rm) / (2 * h)
        assert np.max(np.abs(fd - p.grad_rho[:, a]) / (np.abs(p.grad_rho[:, a]) + p.rho)) < 1e-6


def test_nuclear_derivatives_match_fd(small_dimer):
    """rho^x and (grad rho)^x are total derivatives with the grid moving with its owner."""
    p = small_dimer
    h = 1e-5
    for x in (0, 4, 8, 13, 17):
        A, a = divmod(x, 3)
        qp = inputs.displaced(p, A, a, h)
        qm = inputs.displaced(p, A, a, -h)
        fd = (qp.rho - qm.rho) / (2 * h)
        scale = np.abs(p.rho_x[x]) + p.rho
        assert np.max(np.abs(fd - p.rho_x[x]) / scale) < 1e-6
        fdg = (qp.grad_rho - qm.grad_rho) / (2 * h)
        scale = np.abs(p.grad_rho_x[x]) + p.rho[:, None]
        assert np.max(np.abs(fdg - p.grad_rho_x[x]) / scale) < 1e-5


def test_translational_invariance_of_derivatives(small_dimer):
    p = small_dimer
    s = p.rho_x.reshape(p.n_atom, 3, -1).sum(axis=0)
    assert np.max(np.abs(s)) < 1e-10 * np.max(np.abs(p.rho_x))
    sg = p.grad_rho_x.reshape(p.n_atom, 3, p.n_grid, 3).sum(axis=0)
    assert np.max(np.abs(sg)) < 1e-10 * np.max(np.abs(p.grad_rho_x))


@pytest.mark.parametrize("name,n,P", [("water_dimer", 4200, 18), ("water_hexamer", 27000, 54)])
def test_workload_sizes(name, n, P):
    p = inputs.make_workload(name, with_derivatives=False)
    assert p.n_grid == n and p.n_pert == P


def test_trial_densities_gradient_and_seed():
    """Trial densities: analytic gradient matches central differences of the
    values, and the seed fixes them."""
    p = inputs.make_problem(2, 30, 3, with_derivatives=False)
    rt, gt = inputs.trial_densities(p, 3, 9)
    rt2, gt2 = inputs.trial_densities(p, 3, 9)
    assert np.array_equal(rt, rt2) and np.array_equal(gt, gt2)
    assert rt.shape == (3, p.n_grid) and gt.shape == (3, p.n_grid, 3)
    h = 1e-6
    for k in (0, 17, 101):
        for ax in range(3):
            q1 = dataclasses.replace(p, coords=p.coords.copy())
            q2 = dataclasses.replace(p, coords=p.coords.copy())
            q1.coords[k, ax] += h
            q2.coords[k, ax] -= h
            d = (inputs.trial_densities(q1, 3, 9)[0][:, k] - inputs.trial_densities(q2, 3, 9)[0][:, k]) / (2 * h)
            assert np.allclose(d, gt[:, k, ax], rtol=1e-6, atol=1e-9)


# ---------------------------------------------------------------------------
# Becke-partitioned weights
# ---------------------------------------------------------------------------
def test_becke_step_function_values():
    """s(-1) = 1, s(0) = 1/2, s(1) = 0, s(mu) + s(-mu) = 1, and s', s'' against
    central differences."""
    mu = np.linspace(-1.0, 1.0, 41)
    s, sp, spp = inputs._becke_step(mu)
    assert s[0] == 1.0 and s[20] == 0.5 and s[-1] == 0.0
    assert np.max(np.abs(s + s[::-1] - 1.0)) < 1e-15
    h = 1e-5
    sph = (inputs._becke_step(mu + h)[0] - inputs._becke_step(mu - h)[0]) / (2 * h)
    spph = (inputs._becke_step(mu + h)[1] - inputs._becke_step(mu - h)[1]) / (2 * h)
    assert np.max(np.abs(sph - sp)) < 1e-8 and np.max(np.abs(spph - spp)) < 1e-7


def test_becke_partition_of_unity():
    """Summed over the owner atom, the partition weights P_A / sum_C P_C of any
    point are 1: the same point offered to every atom gets weights that add up
    to the radial weight."""
    rng = np.random.default_rng(3)
    mol = inputs.water_cluster(2, rng)
    pts = rng.standard_normal((50, 3)) * 3.0
    M = mol.n_atom
    tot = np.zeros(50)
    for A in range(M):
        ao = np.full(50, A, dtype=np.int32)
        off = pts - mol.R[A]
        r = np.linalg.norm(off, axis=1)
        w, _, _ = inputs.becke_weights(mol, ao, off, r)
        tot += w / (4 * np.pi * r ** 3 * np.log(inputs.R_MAX / inputs.R_MIN) / 50)
    assert np.max(np.abs(tot - 1.0)) < 1e-14


def test_becke_weights_integrate_density():
    """Each atom integrates its own cell: sum_i w_i rho_i is close to the 20
    electrons of a water dimer (closer than the averaged atomic sets)."""
    p = inputs.make_workload("water_dimer", with_derivatives=False, weights="becke")
    n_el = float(np.dot(p.weights, p.rho))
    assert 18.0 < n_el < 22.0


def test_becke_weight_derivatives_fd(becke_dimer):
    """w_x and w_xy are total derivatives with the grid moving with its owner:
    central differences of the weights and of w_x on displaced geometries."""
    p = becke_dimer
    h = 1e-4
    for x in range(p.n_pert):
        A, a = divmod(x, 3)
        qp = inputs.displaced(p, A, a, h, with_derivatives=True)
        qm = inputs.displaced(p, A, a, -h, with_derivatives=True)
        fd = (qp.weights - qm.weights) / (2 * h)
        assert np.max(np.abs(fd - p.w_x[x])) < 1e-6 * np.max(np.abs(p.w_x))
        fd2 = (qp.w_x - qm.w_x) / (2 * h)
        assert np.max(np.abs(fd2 - p.w_xy[:, x])) < 1e-5 * np.max(np.abs(p.w_xy))
    assert np.max(np.abs(p.w_xy - p.w_xy.transpose(1, 0, 2))) < 1e-12 * np.max(np.abs(p.w_xy))


def test_becke_weight_invariances(becke_dimer):
    """A rigid translation of molecule and grid leaves every weight unchanged:
    sum over atoms of w^{(B,a)}_i and of w^{(B,a)(C,b)}_i vanish."""
    p = becke_dimer
    s = p.w_x.reshape(p.n_atom, 3, -1).sum(axis=0)
    assert np.max(np.abs(s)) < 1e-12 * np.max(np.abs(p.w_x))
    s2 = p.w_xy.reshape(p.n_atom, 3, p.n_pert, -1).sum(axis=0)
    assert np.max(np.abs(s2)) < 1e-12 * np.max(np.abs(p.w_xy))


def test_becke_sparse_and_general_paths_agree(becke_dimer):
    p = becke_dimer
    w1, wx1, _ = inputs.becke_weights(p.mol, p.atom_of, p.offsets, p.radii, 1)
    w2, wx2, _ = inputs.becke_weights(p.mol, p.atom_of, p.offsets, p.radii, 1, jets=True)
    assert np.max(np.abs(w1 - w2)) <= 1e-14 * np.max(np.abs(w2))
    assert np.max(np.abs(wx1 - wx2)) <= 1e-13 * np.max(np.abs(wx2))
    assert np.array_equal(wx2, p.w_x) or np.max(np.abs(wx2 - p.w_x)) <= 1e-13 * np.max(np.abs(wx2))


def test_device_fields_match_host_generator():
    """The torch builder of the density and its nuclear derivatives (run here
    on the CPU) agrees with the numpy one on the same molecule and grid."""
    import torch
    p = inputs.make_problem(2, 40, 91)
    q = inputs.make_problem_on_device(2, 40, 91, torch, torch.device("cpu"))
    assert np.array_equal(p.coords, q.coords) and np.array_equal(p.weights, q.weights)
    assert np.array_equal(p.atom_of, q.atom_of)
    for a, b in ((p.rho, q.rho), (p.grad_rho, q.grad_rho), (p.rho_x, q.rho_x),
                 (p.grad_rho_x, q.grad_rho_x)):
        b = b.numpy()
        assert a.shape == b.shape
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
