"""Seeded synthetic inputs for the MTP hot path.

This module is the only code shared by the oracle and the GPU library's
tests and benchmark.  It draws positions, cells, species and parameters;
it holds none of the potential's arithmetic (no radial basis, no moments,
no contractions, no neighbour predicate).

Inputs stand in for the paper's workloads (bulk metals and multi-species
active-learning runs, Section 3 "Illustrative examples" and the potassium
benchmark of Section 2.2); no dataset or trained potential is available,
so every structure and parameter is drawn from a seeded generator.

Draw order inside one workload (one ``numpy.random.default_rng(seed)``
stream): jitter (N x 3, C order) -> species -> radial coefficients ->
linear coefficients -> species constants -> loss-target perturbation ->
active-set noise.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Structure",
    "Params",
    "bcc_sites",
    "fcc_sites",
    "jitter_wrap",
    "draw_params",
    "draw_active_set",
    "random_cell_batch",
    "workload",
    "WORKLOADS",
]


@dataclasses.dataclass
class Structure:
    """One periodic configuration.

    pos:     [N, 3] float64, Cartesian positions (Angstrom).
    species: [N] int32, species index in [0, n_species).
    cell:    [3, 3] float64, rows are the lattice vectors.
    """

    pos: np.ndarray
    species: np.ndarray
    cell: np.ndarray

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])


@dataclasses.dataclass
class Params:
    """Model hyper-parameters and coefficients (all float64 on the host).

    radial:  [n_species, n_species, n_mu, n_cheb] radial coefficients c.
    linear:  [n_alpha] linear coefficients xi.
    shift:   [n_species] per-species energy constants s.
    """

    level: int
    n_species: int
    n_cheb: int
    r_min: float
    r_cut: float
    radial: np.ndarray
    linear: np.ndarray
    shift: np.ndarray


def bcc_sites(nx: int, ny: int, nz: int, a: float):
    """Body-centred cubic sites, cell-major order (ix outer, then iy, iz, basis)."""
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    return _cubic_sites(nx, ny, nz, a, basis)


def fcc_sites(nx: int, ny: int, nz: int, a: float):
    """Face-centred cubic sites, cell-major order."""
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    return _cubic_sites(nx, ny, nz, a, basis)


def _cubic_sites(nx, ny, nz, a, basis):
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    cell = np.diag([nx * a, ny * a, nz * a]).astype(np.float64)
    return sites, cell


def jitter_wrap(sites: np.ndarray, cell: np.ndarray, sigma: float, rng) -> np.ndarray:
    """Add N(0, sigma) per component, then wrap into the cell (fractional [0, 1))."""
    pos = sites + rng.normal(0.0, sigma, size=sites.shape)
    frac = pos @ np.linalg.inv(cell)
    frac -= np.floor(frac)
    return np.ascontiguousarray(frac @ cell)


def draw_params(rng, level, n_species, n_mu, n_cheb, n_alpha, r_min, r_cut,
                radial_sigma=0.1, linear_sigma=0.01, shift_sigma=1.0) -> Params:
    """Radial c ~ N(0, radial_sigma), linear xi ~ N(0, linear_sigma), s ~ N(0, shift_sigma).

    n_mu and n_alpha are passed in by the caller (they follow from the level
    through the basis definition, which this module does not implement).
    """
    radial = rng.normal(0.0, radial_sigma, size=(n_species, n_species, n_mu, n_cheb))
    linear = rng.normal(0.0, linear_sigma, size=(n_alpha,))
    shift = rng.normal(0.0, shift_sigma, size=(n_species,))
    return Params(level, n_species, n_cheb, float(r_min), float(r_cut), radial, linear, shift)


def perturb_params(rng, p: Params, rel=0.1) -> Params:
    """theta* = theta + rel*|theta| * N(0,1), elementwise (loss-target parameters)."""
    def pert(x):
        return x + rel * np.abs(x) * rng.normal(size=x.shape)
    return Params(p.level, p.n_species, p.n_cheb, p.r_min, p.r_cut,
                  pert(p.radial), pert(p.linear), pert(p.shift))


def draw_active_set(rng, n_alpha: int):
    """A = I + 0.1 N(0,1)/sqrt(n_alpha); returns (A, A^-1) in float64 (LAPACK inverse)."""
    a = np.eye(n_alpha) + 0.1 * rng.normal(size=(n_alpha, n_alpha)) / math.sqrt(n_alpha)
    return a, np.linalg.inv(a)


# --------------------------------------------------------------------------------------
# random triclinic cells at fixed density with a minimum image distance


def _perp_widths(cell):
    inv_t = np.linalg.inv(cell).T  # rows b_k: reciprocal vectors without 2*pi
    return 1.0 / np.linalg.norm(inv_t, axis=1)


def _random_cell(rng, n_atoms, density):
    vol = n_atoms / density
    u = rng.uniform(-0.2, 0.2, size=3)
    u -= u.mean()
    diag = vol ** (1.0 / 3.0) * np.exp(u)
    t = rng.uniform(-0.3, 0.3, size=3)
    cell = np.zeros((3, 3))
    cell[0, 0] = diag[0]
    cell[1, 0] = t[0] * diag[0]          # xy tilt, lower-triangular (rows are vectors)
    cell[1, 1] = diag[1]
    cell[2, 0] = t[1] * diag[0]          # xz tilt
    cell[2, 1] = t[2] * diag[1]          # yz tilt
    cell[2, 2] = diag[2]
    return cell


def _min_image_d2(ds, cell, single):
    """Squared distance to the nearest image for fractional differences ds [..., 3].

    After wrapping ds to [-1/2, 1/2), an image closer than half of every perpendicular
    width must be the wrapped one (|ds_k + n_k| <= |d| / width_k < 1/2 forces n_k = 0);
    single=True uses that, otherwise the 27 surrounding images are scanned.
    """
    ds = ds - np.round(ds)
    x0 = ds @ cell
    if single:
        return (x0 * x0).sum(axis=-1)
    best = None
    for t in _IMAGES27 @ cell:
        x = x0 + t
        d2 = (x * x).sum(axis=-1)
        best = d2 if best is None else np.minimum(best, d2)
    return best


_IMAGES27 = np.stack(np.meshgrid([-1.0, 0.0, 1.0], [-1.0, 0.0, 1.0], [-1.0, 0.0, 1.0], indexing="ij"),
                     axis=-1).reshape(-1, 3)


def _rsa_positions(rng, cell, n_atoms, d_min, max_rounds):
    """Random sequential addition in rounds, minimum distance d_min over all periodic images.

    Each round draws as many uniform fractional points as atoms are missing and accepts
    them in draw order when they keep d_min from every accepted point (earlier rounds and
    earlier points of this round).  Requires every perpendicular width > d_min, so the 27
    images around the wrapped difference hold every image closer than d_min (self-images
    included).  Returns None after max_rounds rounds without completion.
    """
    widths = _perp_widths(cell)
    if np.any(widths <= d_min):
        return None
    single = bool(np.all(widths > 2.0 * d_min))
    d2 = d_min * d_min
    acc = np.zeros((0, 3))
    for _ in range(max_rounds):
        need = n_atoms - len(acc)
        if need == 0:
            break
        cand = rng.uniform(0.0, 1.0, size=(need, 3))
        ok = np.ones(need, dtype=bool)
        if len(acc):
            ok &= _min_image_d2(cand[:, None, :] - acc[None, :, :], cell, single).min(axis=1) >= d2
        close = _min_image_d2(cand[:, None, :] - cand[None, :, :], cell, single) < d2
        np.fill_diagonal(close, False)
        blocked = ~ok
        keep = []
        for k in range(need):
            if not blocked[k]:
                keep.append(k)
                blocked |= close[k]
        acc = np.concatenate([acc, cand[keep]])
    if len(acc) < n_atoms:
        return None
    return acc @ cell


def random_cell_batch(rng, n_cfg, n_min, n_max, density, d_min, n_species, max_rounds=200):
    """n_cfg triclinic periodic configurations with N ~ U{n_min..n_max}.

    Cells are lower-triangular with diagonals V^(1/3) e^u (u ~ U(-0.2, 0.2)
    recentred to zero sum) and tilts U(-0.3, 0.3) times the matching diagonal;
    positions come from random sequential addition in rounds under a minimum
    image distance d_min over all images (self-images included); species are
    i.i.d. uniform.  A cell on which placement fails is redrawn.
    Draw order per configuration: N, cell, positions, species.
    """
    out = []
    for _ in range(n_cfg):
        n = int(rng.integers(n_min, n_max + 1))
        while True:
            cell = _random_cell(rng, n, density)
            pos = _rsa_positions(rng, cell, n, d_min, max_rounds)
            if pos is not None:
                break
        species = rng.integers(0, n_species, size=n).astype(np.int32)
        out.append(Structure(pos, species, cell))
    return out


# --------------------------------------------------------------------------------------
# the five workloads

WORKLOADS = {
    1: dict(name="bcc-4x4x4-L10", level=10, n_species=1, n_cheb=8, r_min=2.0, r_cut=5.0),
    2: dict(name="bcc-20x20x20-2sp-L16", level=16, n_species=2, n_cheb=8, r_min=2.0, r_cut=5.0),
    3: dict(name="bcc-80x80x80-L16", level=16, n_species=1, n_cheb=8, r_min=2.0, r_cut=5.0),
    4: dict(name="fcc-50x50x25-3sp-L16-grade", level=16, n_species=3, n_cheb=8, r_min=2.0, r_cut=5.0),
    5: dict(name="batch-4096-triclinic-3sp-L20", level=20, n_species=3, n_cheb=10, r_min=2.0, r_cut=5.5),
}


def workload(k: int, n_alpha: int, n_mu: int, *, small: dict | None = None):
    """Build workload k (1..5) with its seed k.

    n_alpha / n_mu come from the caller's basis.  ``small`` overrides the
    lattice repeat (``{"rep": (nx, ny, nz)}``) or batch size (``{"n_cfg": m}``)
    to make a reduced-size case with the same recipe; the seed stays k.
    Returns dict(structures=[Structure...], params=Params, extra={...}).
    """
    spec = WORKLOADS[k]
    rng = np.random.default_rng(k)
    small = small or {}
    extra = {}
    if k in (1, 2, 3):
        rep, a, sigma = {1: ((4, 4, 4), 3.16, 0.05), 2: ((20, 20, 20), 3.2, 0.08),
                         3: ((80, 80, 80), 3.16, 0.1)}[k]
        rep = small.get("rep", rep)
        sites, cell = bcc_sites(*rep, a)
        pos = jitter_wrap(sites, cell, sigma, rng)
        n = pos.shape[0]
        if k == 2:
            species = rng.permutation(np.repeat(np.arange(2), n // 2)).astype(np.int32)
            if species.shape[0] < n:
                species = np.concatenate([species, np.zeros(n - species.shape[0], np.int32)])
        else:
            species = np.zeros(n, np.int32)
        structs = [Structure(pos, species, cell)]
    elif k == 4:
        rep = small.get("rep", (50, 50, 25))
        sites, cell = fcc_sites(*rep, 3.52)
        pos = jitter_wrap(sites, cell, 0.15, rng)
        species = rng.integers(0, 3, size=pos.shape[0]).astype(np.int32)
        structs = [Structure(pos, species, cell)]
    else:
        n_cfg = small.get("n_cfg", 4096)
        structs = random_cell_batch(rng, n_cfg, 8, 256, 0.06, 1.8, 3)
    params = draw_params(rng, spec["level"], spec["n_species"], n_mu, spec["n_cheb"], n_alpha,
                         spec["r_min"], spec["r_cut"])
    if k in (2, 5):
        extra["target_params"] = perturb_params(rng, params)
    if k == 4:
        extra["active_set"], extra["active_set_inv"] = draw_active_set(rng, n_alpha)
    return dict(structures=structs, params=params, extra=extra, spec=spec)


def batch_arrays(structs):
    """Concatenate a list of structures: atom_off [n_cfg+1] int32, pos [sum N, 3],
    species [sum N] int32, cells [n_cfg, 3, 3]."""
    counts = np.array([s.n_atoms for s in structs], dtype=np.int64)
    off = np.zeros(len(structs) + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    pos = np.ascontiguousarray(np.concatenate([s.pos for s in structs]))
    species = np.ascontiguousarray(np.concatenate([s.species for s in structs]).astype(np.int32))
    cells = np.ascontiguousarray(np.stack([s.cell for s in structs]))
    return off, pos, species, cells
