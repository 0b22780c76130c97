"""The allocation-free entry point mtp_compute_static against mtp_compute.

mtp_compute_static runs the same kernels out of the library's fixed scratch area; for every
system it must return exactly what mtp_compute returns (energy, site energies, forces, virial),
also on consecutive calls whose second input is smaller than the first (the area keeps the
previous call's contents), at a multi-group level, when the chunk has to shrink to fit, and it
must refuse a system that does not fit before enqueuing anything.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from helpers import TOL_E, TOL_F, TOL_W, rel_err, small_batch

pytestmark = pytest.mark.gpu


def _lattice(seed, rep, level, n_species, sigma=0.08, a=3.2):
    from paper_2510_00193_amd import level_info
    info = level_info(level)
    rng = np.random.default_rng(seed)
    sites, cell = wl.bcc_sites(*rep, a)
    pos = wl.jitter_wrap(sites, cell, sigma, rng)
    species = rng.integers(0, n_species, size=len(pos)).astype(np.int32)
    p = wl.draw_params(rng, level, n_species, info["n_mu"], 8, info["n_alpha"], 2.0, 5.0)
    return wl.Structure(pos, species, cell), p


def _both(pot, s, label, **kw):
    print(f"[{label}] N={s.n_atoms} level={pot.level}", flush=True)
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    nl = pot.neighbors(pos, sp, s.cell)
    want = pot.compute(pos, sp, s.cell, nlist=nl, **kw)
    got = pot.compute_static(pos, sp, s.cell, nl, **kw)
    torch.cuda.synchronize()
    for k in want:
        a, b = got[k].cpu().numpy(), want[k].cpu().numpy()
        assert np.array_equal(a, b), (label, k, rel_err(a, b))
    return got


def test_static_matches_compute_on_consecutive_calls():
    from paper_2510_00193_amd import Potential
    big, p = _lattice(71, (8, 8, 8), 16, 2)
    small, _ = _lattice(72, (5, 5, 5), 16, 2)
    pot = Potential.from_params(p)
    _both(pot, big, "bcc-8^3-L16", e_atom=True)
    _both(pot, small, "bcc-5^3-L16 after a larger call", e_atom=True)
    # energy and forces only (no virial), then energy only (no backward pass)
    _both(pot, small, "bcc-5^3-L16 forces only", virial=False)
    _both(pot, big, "bcc-8^3-L16 energy only", forces=False, virial=False)


def test_static_multigroup_level_and_caller_list():
    from paper_2510_00193_amd import Potential, compiled_levels, level_info
    levels = [lv for lv in compiled_levels() if level_info(lv)["n_groups"] > 1]
    if not levels:
        pytest.skip("no multi-group level compiled")
    lv = max(levels)
    structs, p = small_batch(4000 + lv, 2, lv, n_min=30, n_max=40)
    pot = Potential.from_params(p)
    for k, s in enumerate(structs):
        _both(pot, s, f"cfg{k}-L{lv}", e_atom=True)
    # a caller-assembled (unchecked) list is validated inside the call, with the flag word in
    # the scratch area
    s = structs[1]
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    nl = pot.neighbors(pos, sp, s.cell)
    nl.checked = False
    want = pot.compute(pos, sp, s.cell, nlist=nl)
    got = pot.compute_static(pos, sp, s.cell, nl)
    torch.cuda.synchronize()
    assert np.array_equal(got["forces"].cpu().numpy(), want["forces"].cpu().numpy())
    bad_rev = nl.rev.clone()
    bad_rev[0] = -1
    from paper_2510_00193_amd._lib import MTP_ERR_ARG, MtpError
    bad = type(nl)(nl.off, nl.j, nl.shift, bad_rev, checked=False)
    with pytest.raises(MtpError) as ei:
        pot.compute_static(pos, sp, s.cell, bad)
    assert ei.value.code == MTP_ERR_ARG


def test_static_shrinks_the_chunk_and_refuses_what_does_not_fit():
    from paper_2510_00193_amd import Potential
    from paper_2510_00193_amd._lib import MTP_ERR_CAPACITY, MtpError
    # about 31k atoms at level 16: the moments of one chunk exceed the area, the pair gradients
    # do not, so the call runs in smaller chunks and must still match exactly
    mid, p = _lattice(73, (25, 25, 25), 16, 1, sigma=0.1, a=3.16)
    pot = Potential.from_params(p)
    _both(pot, mid, "bcc-25^3-L16 chunked", e_atom=True)
    # 128k atoms: the pair gradients alone exceed the area
    huge, _ = _lattice(74, (40, 40, 40), 16, 1, sigma=0.1, a=3.16)
    pos = torch.as_tensor(huge.pos, device="cuda")
    sp = torch.as_tensor(huge.species, device="cuda")
    nl = pot.neighbors(pos, sp, huge.cell)
    torch.cuda.synchronize()
    print(f"[refuse] N={huge.n_atoms} pairs={nl.n_pairs}", flush=True)
    with pytest.raises(MtpError) as ei:
        pot.compute_static(pos, sp, huge.cell, nl)
    assert ei.value.code == MTP_ERR_CAPACITY
    # and the next call that fits still runs and matches
    small, _ = _lattice(75, (4, 4, 4), 16, 1, sigma=0.1, a=3.16)
    _both(pot, small, "bcc-4^3-L16 after a refusal")


def test_static_against_oracle_small():
    """The same entry point checked directly against the float64 oracle (the parity bar)."""
    from oracle import mtp as om
    from paper_2510_00193_amd import Potential
    s, p = _lattice(76, (4, 4, 4), 10, 2, sigma=0.05, a=3.16)
    pot = Potential.from_params(p)
    ref = om.energy_forces_virial(om.Model.from_params(p), s)
    got = _both(pot, s, "bcc-4^3-L10 vs oracle", e_atom=True)
    assert rel_err(float(got["energy"].cpu()), float(ref["E"].detach())) < TOL_E
    assert rel_err(got["e_atom"].cpu().numpy(), ref["E_i"].detach().numpy()) < TOL_E
    assert rel_err(got["forces"].cpu().numpy(), ref["F"].detach().numpy()) < TOL_F
    assert rel_err(got["virial"].cpu().numpy(), ref["W"].detach().numpy()) < TOL_W
