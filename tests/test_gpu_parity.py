"""GPU parity of the neighbour list and of energies, forces and virial against the oracle.

Every case runs the HIP path through the C ABI and compares, element by
element, with the float64 CPU oracle on the same seeded inputs.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from helpers import TOL_E, TOL_F, TOL_W, rel_err, small_batch, small_lattice
from oracle import mtp as om
from oracle import neighbors as onb

pytestmark = pytest.mark.gpu


def _dev(s):
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species.astype(np.int32), device="cuda")
    return pos, sp


def _pot(p, **kw):
    from paper_2510_00193_amd import Potential
    return Potential.from_params(p, **kw)


def _check_nlist(nl_gpu, nl_ref):
    np.testing.assert_array_equal(nl_gpu.off.cpu().numpy(), nl_ref["off"])
    np.testing.assert_array_equal(nl_gpu.j.cpu().numpy(), nl_ref["j"])
    np.testing.assert_array_equal(nl_gpu.shift.cpu().numpy(), nl_ref["shift"])
    np.testing.assert_array_equal(nl_gpu.rev.cpu().numpy(), nl_ref["rev"])


def _full_parity(s, p, label, **kw):
    print(f"[{label}] N={s.n_atoms} level={p.level} species={p.n_species}", flush=True)
    model = om.Model.from_params(p)
    ref = om.energy_forces_virial(model, s)
    pot = _pot(p, **kw)
    pos, sp = _dev(s)
    nl = pot.neighbors(pos, sp, s.cell)
    torch.cuda.synchronize()
    _check_nlist(nl, ref["nl"])
    out = pot.compute(pos, sp, s.cell, nlist=nl, e_atom=True)
    torch.cuda.synchronize()
    e = float(out["energy"].cpu())
    assert rel_err(e, float(ref["E"].detach())) < TOL_E
    assert rel_err(out["e_atom"].cpu().numpy(), ref["E_i"].detach().numpy()) < TOL_E
    assert rel_err(out["forces"].cpu().numpy(), ref["F"].detach().numpy()) < TOL_F
    assert rel_err(out["virial"].cpu().numpy(), ref["W"].detach().numpy()) < TOL_W
    return pot, out, ref


def test_workload1_full_parity():
    """128-atom bcc, level 10, one species: the small plain-method case."""
    n_alpha, n_mu = 17, 3
    w = wl.workload(1, n_alpha, n_mu)
    (s,) = w["structures"]
    _full_parity(s, w["params"], "bcc-4x4x4-L10")


def test_level16_two_species_full_parity():
    s, p = small_lattice(202, (4, 4, 4), 3.2, 0.08, 16, 2)
    _full_parity(s, p, "bcc-4x4x4-2sp-L16")


@pytest.mark.parametrize("seed", [301, 302])
def test_thin_triclinic_cells_image_path(seed):
    structs, p = small_batch(seed, 3, 10, n_min=8, n_max=30)
    for k, s in enumerate(structs):
        _full_parity(s, p, f"triclinic-{seed}-{k}")


def test_cell_list_path_matches_oracle_list():
    rng = np.random.default_rng(404)
    sites, cell = wl.bcc_sites(9, 9, 9, 3.16)
    pos = wl.jitter_wrap(sites, cell, 0.1, rng)
    # shift some atoms by whole lattice vectors: positions are used as given
    pos[::7] += cell[0] - 2 * cell[2]
    s = wl.Structure(pos, np.zeros(len(pos), np.int32), cell)
    p = wl.draw_params(rng, 10, 1, 3, 8, 17, 2.0, 5.0)
    print(f"[cell-list] N={s.n_atoms}", flush=True)
    ref = onb.neighbor_csr(s.pos, s.cell, 5.0)
    pot = _pot(p)
    d_pos, d_sp = _dev(s)
    nl = pot.neighbors(d_pos, d_sp, s.cell)
    torch.cuda.synchronize()
    _check_nlist(nl, ref)


def test_internal_list_chunking_and_determinism():
    s, p = small_lattice(505, (5, 5, 5), 3.16, 0.1, 10, 1)
    pos, sp = _dev(s)
    print(f"[chunking] N={s.n_atoms}", flush=True)
    a = _pot(p).compute(pos, sp, s.cell, e_atom=True)
    b = _pot(p).compute(pos, sp, s.cell, e_atom=True)
    c = _pot(p, chunk_atoms=37).compute(pos, sp, s.cell, e_atom=True)
    torch.cuda.synchronize()
    for k in ("energy", "forces", "virial", "e_atom"):
        assert torch.equal(a[k], b[k]), k
    assert torch.equal(a["e_atom"], c["e_atom"])
    assert torch.equal(a["forces"], c["forces"])
    assert torch.equal(a["energy"], c["energy"])
    assert rel_err(c["virial"].cpu().numpy(), a["virial"].cpu().numpy()) < 1e-13


def test_empty_and_isolated_systems():
    s, p = small_lattice(606, (1, 1, 1), 3.16, 0.0, 10, 1)
    pot = _pot(p)
    pos = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    sp = torch.zeros((0,), dtype=torch.int32, device="cuda")
    out = pot.compute(pos, sp, np.eye(3) * 20.0)
    torch.cuda.synchronize()
    assert float(out["energy"].cpu()) == 0.0
    # one atom in a large box: no pairs, energy = species constant
    pos = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    sp = torch.zeros((1,), dtype=torch.int32, device="cuda")
    out = pot.compute(pos, sp, np.eye(3) * 20.0)
    torch.cuda.synchronize()
    assert float(out["energy"].cpu()) == pytest.approx(float(p.shift[0]), rel=1e-15)
    assert float(out["forces"].abs().max().cpu()) == 0.0


def test_error_paths():
    from paper_2510_00193_amd._lib import MtpError
    s, p = small_lattice(707, (2, 2, 2), 3.16, 0.05, 10, 1)
    pot = _pot(p)
    pos, sp = _dev(s)
    with pytest.raises(MtpError) as ei:
        pot.compute(pos, sp, np.zeros((3, 3)))
    assert ei.value.code == 2
    bad = pos.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(MtpError) as ei:
        pot.compute(bad, sp, s.cell)
    assert ei.value.code == 4
    with pytest.raises(MtpError) as ei:
        pot.neighbors(pos, sp, s.cell, cap=5)
    assert ei.value.code == 3


@pytest.mark.parametrize("n_cheb", [1, 2, 5, 10])
def test_chebyshev_counts(n_cheb):
    """Compile-time (8, 10) and runtime Chebyshev counts of the pair kernels."""
    s, p = small_lattice(808 + n_cheb, (4, 4, 4), 3.16, 0.1, 10, 2, n_cheb=n_cheb)
    _full_parity(s, p, f"cheb-{n_cheb}")


@pytest.mark.parametrize("a,rep,r_cut", [(3.16, 10, 5.0), (3.6, 8, 5.0), (3.0, 7, 5.0), (2.2, 5, 5.0)])
def test_cell_list_densities(a, rep, r_cut):
    """Neighbour lists at densities that select each staged capacity of the cell path and the
    unstaged fallback (bcc 3.16: 512 candidates; fcc 3.6: 768; fcc 3.0: 1024 with 256-entry
    rows; fcc 2.2: unstaged)."""
    rng = np.random.default_rng(909)
    sites, cell = wl.fcc_sites(rep, rep, rep, a) if a != 3.16 else wl.bcc_sites(rep, rep, rep, a)
    pos = wl.jitter_wrap(sites, cell, 0.05, rng)
    pos[::5] -= cell[1]   # some atoms one image outside the box
    s = wl.Structure(pos, np.zeros(len(pos), np.int32), cell)
    p = wl.draw_params(rng, 10, 1, 3, 8, 17, 2.0, r_cut)
    print(f"[density a={a} rep={rep} rc={r_cut}] N={s.n_atoms}", flush=True)
    ref = onb.neighbor_csr(s.pos, s.cell, r_cut)
    pot = _pot(p)
    d_pos, d_sp = _dev(s)
    nl = pot.neighbors(d_pos, d_sp, s.cell)
    torch.cuda.synchronize()
    _check_nlist(nl, ref)


def test_caller_built_list_is_validated():
    """A list assembled by the caller (not by the library) is checked before use: a correct one
    gives the oracle's results, and each kind of inconsistency is refused with MTP_ERR_ARG."""
    from paper_2510_00193_amd import NeighborList
    from paper_2510_00193_amd._lib import MtpError
    s, p = small_lattice(1501, (3, 3, 3), 3.16, 0.08, 10, 2)
    ref_nl = onb.neighbor_csr(s.pos, s.cell, p.r_cut)
    ref = om.energy_forces_virial(om.Model.from_params(p), s, ref_nl)
    pot = _pot(p)
    pos, sp = _dev(s)

    def nlist(off, j, shift, rev):
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32), device="cuda")  # noqa: E731
        return NeighborList(t(off), t(j), t(shift), t(rev))

    base = (ref_nl["off"], ref_nl["j"], ref_nl["shift"], ref_nl["rev"])
    print(f"[caller list] N={s.n_atoms} pairs={len(ref_nl['j'])}", flush=True)
    out = pot.compute(pos, sp, s.cell, nlist=nlist(*base))
    torch.cuda.synchronize()
    assert rel_err(out["forces"].cpu().numpy(), ref["F"].detach().numpy()) < TOL_F
    assert rel_err(out["virial"].cpu().numpy(), ref["W"].detach().numpy()) < TOL_W
    bad_cases = {}
    rev = base[3].copy()
    rev[5] = -1
    bad_cases["missing mirror"] = (base[0], base[1], base[2], rev)
    rev = base[3].copy()
    rev[5], rev[6] = rev[6], rev[5]
    bad_cases["swapped mirrors"] = (base[0], base[1], base[2], rev)
    off = base[0].copy()
    off[-1] -= 1
    bad_cases["short last row"] = (off, base[1], base[2], base[3])
    j = base[1].copy()
    j[3] = s.n_atoms
    bad_cases["partner out of range"] = (base[0], j, base[2], base[3])
    sh = base[2].copy()
    sh[7] ^= 1
    bad_cases["unmirrored shift"] = (base[0], base[1], sh, base[3])
    for name, lists in bad_cases.items():
        with pytest.raises(MtpError) as ei:
            pot.compute(pos, sp, s.cell, nlist=nlist(*lists))
        assert ei.value.code == 1, name
    bad_sp = sp.clone()
    bad_sp[2] = p.n_species
    with pytest.raises(MtpError) as ei:
        pot.compute(pos, bad_sp, s.cell, nlist=nlist(*base))
    assert ei.value.code == 1
