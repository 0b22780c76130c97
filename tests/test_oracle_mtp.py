"""Pins of the oracle's energies, forces, virial, grade and parameter gradients (CPU only).

Each check is independent of the oracle's own formulas: neighbour-tuple brute
force for the contractions, closed forms at levels 2 and 4, library Chebyshev
routines, symmetry invariants, central finite differences and the MaxVol
property of the grade.
"""
import itertools

import numpy as np
import pytest
import torch
from numpy.polynomial import chebyshev as npcheb

import workloads as wl
from oracle import mtp as om
from oracle import neighbors as onb


def _model(level, n_species, rng, n_cheb=8, r_min=2.0, r_cut=5.0, c_sigma=0.1, xi_sigma=0.01):
    basis = om.basis_for(level)
    from oracle.basis import radial_count
    p = wl.draw_params(rng, level, n_species, radial_count(level, basis), n_cheb, len(basis),
                       r_min, r_cut, c_sigma, xi_sigma)
    return om.Model.from_params(p)


def _small_struct(seed, n_species=2, n=10, level=None):
    rng = np.random.default_rng(seed)
    (s,) = wl.random_cell_batch(rng, 1, n, n, 0.06, 1.8, n_species)
    return s, rng


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ----------------------------------------------------------------------------- contractions


def _tuple_value(bf, f, d):
    """B = sum over neighbour tuples of prod f_mu_k(r_jk) prod_{k<l} (d_jk . d_jl)^m_kl."""
    k = len(bf.labels)
    m = bf.matrix()
    n = d.shape[0]
    dots = d @ d.T
    total = 0.0
    for tup in itertools.product(range(n), repeat=k):
        v = 1.0
        for a in range(k):
            v *= f[tup[a], bf.labels[a][0]]
        for a in range(k):
            for b in range(a + 1, k):
                if m[a][b]:
                    v *= dots[tup[a], tup[b]] ** m[a][b]
        total += v
    return total


@pytest.mark.parametrize("level", [8, 10, 12])
def test_contractions_equal_tuple_sums(level):
    rng = np.random.default_rng(level)
    model = _model(level, 1, rng)
    n = 5
    d = rng.normal(size=(n, 3))
    d *= rng.uniform(2.2, 4.8, size=(n, 1)) / np.linalg.norm(d, axis=1, keepdims=True)
    dt = torch.as_tensor(d)
    centre = torch.zeros(n, dtype=torch.long)
    r = torch.sqrt((dt * dt).sum(1))
    z = torch.zeros(n, dtype=torch.long)
    f = om.radial_functions(model, r, z, z).numpy()
    mom = om.moment_tensors(model, dt, centre, 1, torch.as_tensor(f))
    b = om.basis_values(model, mom).numpy()[0]
    for a, bf in enumerate(model.basis):
        if len(bf.labels) > 4:
            continue
        want = _tuple_value(bf, f, d)
        assert abs(b[a] - want) <= 1e-11 * max(1.0, abs(want)), (bf, b[a], want)


# ----------------------------------------------------------------------------- closed forms


def _pair_phi(model, r, zi, zj, deriv=False):
    """phi(r) = sum_beta c[zi,zj,0,beta] T_beta(u) (rc - r)^2 written with numpy's chebval."""
    rc, rm = model.r_cut, model.r_min
    c = model.radial.numpy()[zi, zj, 0]
    u = (2 * r - (rc + rm)) / (rc - rm)
    t = npcheb.chebval(u, c)
    if not deriv:
        return t * (rc - r) ** 2
    dt = npcheb.chebval(u, npcheb.chebder(c)) * 2.0 / (rc - rm)
    return dt * (rc - r) ** 2 - 2.0 * t * (rc - r)


@pytest.mark.parametrize("level", [2, 4])
def test_levels_2_and_4_closed_forms(level):
    s, rng = _small_struct(11, n_species=2, n=9)
    model = _model(level, 2, rng, c_sigma=0.3, xi_sigma=0.5)
    out = om.energy_forces_virial(model, s)
    nl = out["nl"]
    i, j, n = nl["i"], nl["j"], nl["n"]
    d = onb.displacements(s.pos, s.cell, i, j, n)
    r = np.linalg.norm(d, axis=1)
    z = s.species
    phi = np.array([_pair_phi(model, rr, z[a], z[b]) for rr, a, b in zip(r, i, j)])
    dphi = np.array([_pair_phi(model, rr, z[a], z[b], True) for rr, a, b in zip(r, i, j)])
    rho = np.zeros(s.n_atoms)
    np.add.at(rho, i, phi)
    xi = model.linear.numpy()
    e_i = model.shift.numpy()[z] + xi[0] * rho + (xi[1] * rho ** 2 if level == 4 else 0.0)
    assert _rel(out["E_i"].detach().numpy(), e_i) < 1e-13
    dEdrho = xi[0] + (2 * xi[1] * rho if level == 4 else np.zeros(s.n_atoms))
    g = (dEdrho[i] * dphi / r)[:, None] * d
    f = np.zeros((s.n_atoms, 3))
    np.add.at(f, i, g)
    np.add.at(f, j, -g)
    assert _rel(out["F"].detach().numpy(), f) < 1e-12
    w = [-(d[:, a] * g[:, c]).sum() for a, c in om.VIRIAL_ORDER]
    assert _rel(out["W"].detach().numpy(), w) < 1e-12


# ----------------------------------------------------------------------------- invariants


def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


@pytest.mark.parametrize("level", [10, 16])
def test_rotation_translation_permutation_invariance(level):
    s, rng = _small_struct(21, n_species=2, n=8)
    model = _model(level, 2, rng)
    base = om.energy_forces_virial(model, s)
    e0 = float(base["E"].detach())
    f0 = base["F"].detach().numpy()
    cond = float(np.abs(base["E_i"].detach().numpy()).sum()) + abs(e0)
    q = _rotation(rng)
    rot = wl.Structure(s.pos @ q.T, s.species, s.cell @ q.T)
    out = om.energy_forces_virial(model, rot)
    assert abs(float(out["E"].detach()) - e0) <= 1e-12 * cond
    assert _rel(out["F"].detach().numpy(), f0 @ q.T) < 1e-10
    tr = wl.Structure(s.pos + np.array([0.3, -1.1, 2.7]), s.species, s.cell)
    assert abs(float(om.energy_forces_virial(model, tr)["E"].detach()) - e0) <= 1e-12 * cond
    perm = rng.permutation(s.n_atoms)
    pm = wl.Structure(s.pos[perm], s.species[perm], s.cell)
    out = om.energy_forces_virial(model, pm)
    assert abs(float(out["E"].detach()) - e0) <= 1e-12 * cond
    assert _rel(out["F"].detach().numpy(), f0[perm]) < 1e-11


@pytest.mark.parametrize("level", [10, 16])
def test_forces_are_minus_gradient_and_sum_to_zero(level):
    s, rng = _small_struct(31, n_species=2, n=7)
    model = _model(level, 2, rng)
    out = om.energy_forces_virial(model, s)
    nl = out["nl"]
    f = out["F"].detach().numpy()
    fmax = np.abs(f).max()
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * fmax * s.n_atoms
    h = 1e-5
    fd = np.zeros_like(f)
    for k in range(s.n_atoms):
        for a in range(3):
            p = s.pos.copy()
            p[k, a] += h
            ep = om.energy_from_positions(model, p, s, nl)
            p[k, a] -= 2 * h
            em = om.energy_from_positions(model, p, s, nl)
            fd[k, a] = -(ep - em) / (2 * h)
    assert _rel(f, fd) < 1e-7


@pytest.mark.parametrize("level", [10, 16])
def test_virial_is_minus_strain_derivative(level):
    s, rng = _small_struct(41, n_species=2, n=7)
    model = _model(level, 2, rng)
    out = om.energy_forces_virial(model, s)
    nl = out["nl"]
    w = out["W"].detach().numpy()
    h = 1e-6
    fd = []
    for a, c in om.VIRIAL_ORDER:
        vals = []
        for sign in (1, -1):
            eps = np.zeros((3, 3))
            eps[a, c] = sign * h
            defm = np.eye(3) + eps          # x -> (I + eps) x
            vals.append(om.energy_from_positions(model, s.pos @ defm.T, s, nl, cell=s.cell @ defm.T))
        fd.append(-(vals[0] - vals[1]) / (2 * h))
    assert _rel(w, fd) < 1e-6
    # a symmetric tensor: the xy, xz, yz entries match their mirrored sums
    g = out["g"].detach().numpy()
    d = out["d"].detach().numpy()
    for a, c in ((0, 1), (0, 2), (1, 2)):
        assert abs((d[:, a] * g[:, c]).sum() - (d[:, c] * g[:, a]).sum()) <= 1e-9 * np.abs(w).max()


def test_virial_cluster_limit():
    rng = np.random.default_rng(5)
    model = _model(10, 1, rng)
    pos = rng.uniform(0, 6.0, size=(6, 3)) + 20.0
    cell = np.diag([80.0, 80.0, 80.0])
    s = wl.Structure(pos, np.zeros(6, np.int32), cell)
    out = om.energy_forces_virial(model, s)
    f = out["F"].detach().numpy()
    want = [(pos[:, a] * f[:, c]).sum() for a, c in om.VIRIAL_ORDER]
    assert _rel(out["W"].detach().numpy(), want) < 1e-10


# ----------------------------------------------------------------------------- grade


def test_grade_identity_and_maxvol():
    s, rng = _small_struct(51, n_species=2, n=24)
    model = _model(6, 2, rng)
    b = om.energy_forces_virial(model, s)["B"].detach().numpy()
    np.testing.assert_allclose(om.grade(b, np.eye(b.shape[1])), np.abs(b).max(axis=1), rtol=0, atol=0)
    chosen = rng.choice(s.n_atoms, size=b.shape[1], replace=False)
    a = b[chosen]
    g = om.grade(b, np.linalg.inv(a))
    np.testing.assert_allclose(g[chosen], 1.0, rtol=1e-9)


def test_config_grade_descriptor_is_energy_gradient_and_maxvol():
    """Configuration mode: the descriptor equals dE/dxi (autograd through the whole energy), and
    configurations whose descriptors form A have grade 1 (MaxVol property)."""
    rng = np.random.default_rng(57)
    model = _model(6, 2, rng)
    n_alpha = len(model.basis)
    structs = wl.random_cell_batch(rng, n_alpha + 2, 8, 20, 0.06, 1.8, 2)
    desc = []
    for k, st in enumerate(structs):
        b = om.energy_forces_virial(model, st)["B"].detach().numpy()
        if k < 2:
            dxi, _, _ = om.param_vjp(model, st, 1.0, np.zeros((st.n_atoms, 3)))
            assert _rel(om.config_descriptor(b), dxi) < 1e-12
        desc.append(om.config_descriptor(b))
    desc = np.array(desc)
    a = desc[:n_alpha]
    ainv = np.linalg.inv(a)
    for k, st in enumerate(structs[:n_alpha]):
        b = om.energy_forces_virial(model, st)["B"].detach().numpy()
        assert abs(om.config_grade(b, ainv) - 1.0) < 1e-8
    assert om.config_grade(np.eye(n_alpha)[:1], np.eye(n_alpha)) == 1.0


# ----------------------------------------------------------------------------- parameter gradients


def test_param_vjp_matches_finite_differences():
    s, rng = _small_struct(61, n_species=2, n=6)
    model = _model(8, 2, rng)
    ebar = 0.7
    fbar = rng.normal(size=(s.n_atoms, 3))
    nl = onb.neighbor_csr(s.pos, s.cell, model.r_cut)
    dxi, dc, ds = om.param_vjp(model, s, ebar, fbar, nl)

    def target(radial, linear, shift):
        out = om.energy_forces_virial(model, s, nl, torch.as_tensor(radial), torch.as_tensor(linear),
                                      torch.as_tensor(shift))
        return float((ebar * out["E"] + (out["F"] * torch.as_tensor(fbar)).sum()).detach())

    r0, l0, s0 = model.radial.numpy(), model.linear.numpy(), model.shift.numpy()
    for name, arr, got in (("linear", l0, dxi), ("radial", r0, dc), ("shift", s0, ds)):
        fd = np.zeros_like(arr)
        flat = arr.reshape(-1)
        for idx in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[idx]))
            vals = []
            for sg in (1, -1):
                x = flat.copy()
                x[idx] += sg * h
                xs = x.reshape(arr.shape)
                args = {"radial": r0, "linear": l0, "shift": s0}
                args[name] = xs
                vals.append(target(args["radial"], args["linear"], args["shift"]))
            fd.reshape(-1)[idx] = (vals[0] - vals[1]) / (2 * h)
        assert _rel(got, fd) < 1e-6, name


def test_param_vjp_linear_part_closed_form():
    """d/dxi of (ebar E + fbar.F) = ebar sum_i B_i - D_fbar(sum_i B_i), the last term a
    central difference of the summed basis along the displacement fbar (no autograd)."""
    s, rng = _small_struct(71, n_species=2, n=6)
    model = _model(10, 2, rng)
    ebar = -0.4
    fbar = rng.normal(size=(s.n_atoms, 3))
    nl = onb.neighbor_csr(s.pos, s.cell, model.r_cut)
    dxi, _, ds = om.param_vjp(model, s, ebar, fbar, nl)

    def bsum(pos):
        d = torch.as_tensor(onb.displacements(pos, s.cell, nl["i"], nl["j"], nl["n"]))
        z = torch.as_tensor(s.species.astype(np.int64))
        i = torch.as_tensor(nl["i"].astype(np.int64))
        _, b = om.site_quantities(model, d, i, z, z[torch.as_tensor(nl["j"].astype(np.int64))], s.n_atoms)
        return b.sum(0).numpy()

    h = 1e-5
    # fourth-order central stencil: the polynomial basis curves strongly below r_min
    deriv = (8 * (bsum(s.pos + h * fbar) - bsum(s.pos - h * fbar))
             - (bsum(s.pos + 2 * h * fbar) - bsum(s.pos - 2 * h * fbar))) / (12 * h)
    want = ebar * bsum(s.pos) - deriv
    assert _rel(dxi, want) < 1e-9
    np.testing.assert_allclose(ds, ebar * np.bincount(s.species, minlength=2), rtol=1e-14)


def test_sampled_helpers_equal_full_evaluation():
    rng = np.random.default_rng(81)
    sites, cell = wl.bcc_sites(3, 3, 3, 3.2)
    pos = wl.jitter_wrap(sites, cell, 0.08, rng)
    species = rng.integers(0, 2, size=len(pos)).astype(np.int32)
    s = wl.Structure(pos, species, cell)
    model = _model(10, 2, rng)
    full = om.energy_forces_virial(model, s)
    atoms = [0, 5, 31, 53]
    rows, e, b = om.sampled_site_values(model, s, atoms)
    nl = full["nl"]
    for a, (js, ns) in zip(atoms, rows):
        lo, hi = nl["off"][a], nl["off"][a + 1]
        np.testing.assert_array_equal(js, nl["j"][lo:hi])
        np.testing.assert_array_equal(ns, nl["n"][lo:hi])
    np.testing.assert_allclose(e, full["E_i"].detach().numpy()[atoms], rtol=1e-13)
    np.testing.assert_allclose(b, full["B"].detach().numpy()[atoms], rtol=1e-13, atol=1e-300)
    f = om.sampled_forces(model, s, atoms)
    assert _rel(f, full["F"].detach().numpy()[atoms]) < 1e-12


def test_chunked_vjp_equals_whole():
    s, rng = _small_struct(91, n_species=2, n=12)
    model = _model(10, 2, rng)
    fbar = rng.normal(size=(s.n_atoms, 3))
    nl = onb.neighbor_csr(s.pos, s.cell, model.r_cut)
    whole = om.param_vjp(model, s, 0.6, fbar, nl)
    parts = om.param_vjp_chunked(model, s, 0.6, fbar, nl, chunk=5)
    for a, b in zip(whole, parts):
        assert _rel(b, a) < 1e-12
