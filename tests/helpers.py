"""Shared helpers of the test suite (inputs, tolerances, GPU availability)."""
from __future__ import annotations

import numpy as np

import workloads as wl

# Parity tolerances (relative, max-norm) of the float64 path against the oracle.
TOL_E = 1e-10
TOL_F = 1e-10
TOL_W = 1e-10
TOL_GRADE = 1e-9


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = max(float(np.max(np.abs(want))) if want.size else 0.0, 1e-300)
    return float(np.max(np.abs(got - want))) / den if want.size else 0.0


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def oracle_sizes(level):
    from oracle import mtp as om
    from oracle.basis import radial_count
    b = om.basis_for(level)
    return len(b), radial_count(level, b)


def small_lattice(seed, rep, a, sigma, level, n_species, lattice="bcc", n_cheb=8, r_min=2.0, r_cut=5.0):
    rng = np.random.default_rng(seed)
    sites, cell = (wl.bcc_sites if lattice == "bcc" else wl.fcc_sites)(*rep, a)
    pos = wl.jitter_wrap(sites, cell, sigma, rng)
    species = rng.integers(0, n_species, size=len(pos)).astype(np.int32)
    n_alpha, n_mu = oracle_sizes(level)
    p = wl.draw_params(rng, level, n_species, n_mu, n_cheb, n_alpha, r_min, r_cut)
    return wl.Structure(pos, species, cell), p


def small_batch(seed, n_cfg, level, n_species=3, n_cheb=10, r_min=2.0, r_cut=5.5, n_min=8, n_max=40):
    rng = np.random.default_rng(seed)
    structs = wl.random_cell_batch(rng, n_cfg, n_min, n_max, 0.06, 1.8, n_species)
    n_alpha, n_mu = oracle_sizes(level)
    p = wl.draw_params(rng, level, n_species, n_mu, n_cheb, n_alpha, r_min, r_cut)
    return structs, p
