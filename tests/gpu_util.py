"""Helpers for the GPU parity tests: error metrics and cached oracle runs."""
import functools

import numpy as np

import oracle
from paper_2208_14639_amd import inputs


def normwise(got, want):
    """max_k |got_k - want_k| / max_k |want_k|"""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def relerr(got, want):
    return abs(float(got) - float(want)) / abs(float(want))


@functools.lru_cache(maxsize=8)
def problem(n_water, n_pa, seed):
    return inputs.make_problem(n_water, n_pa, seed)


@functools.lru_cache(maxsize=8)
def oracle_energy(n_water, n_pa, seed):
    p = problem(n_water, n_pa, seed)
    g = oracle.gamma(p.grad_rho)
    return oracle.energy_potential(p.coords, p.weights, p.rho, g, p.b, p.C)


@functools.lru_cache(maxsize=8)
def oracle_hessian(n_water, n_pa, seed):
    p = problem(n_water, n_pa, seed)
    g, gx = oracle.problem_inputs(p)
    H, info = oracle.hessian_terms(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C,
                                   p.rho_x, gx, resp=True)
    G = oracle.gradient(p.atom_of, p.n_atom, p.coords, p.weights, p.rho, g, p.b, p.C, p.rho_x, gx)
    return H, G, info["resp"]
