"""GPU parity of the small-system form of the pair kernels (several lanes share one atom's
neighbour loop and combine their sums): energies, per-atom energies, forces and virial against
the oracle for every lanes-per-atom setting, chunk invariance and run-to-run determinism."""
import numpy as np
import pytest
import torch

from helpers import TOL_E, TOL_F, TOL_W, rel_err, small_batch, small_lattice
from oracle import mtp as om

pytestmark = pytest.mark.gpu

SPLITS = (1, 2, 4, 8)


def _pot(p, **kw):
    from paper_2510_00193_amd import Potential
    return Potential.from_params(p, **kw)


def _dev(s):
    return torch.as_tensor(s.pos, device="cuda"), torch.as_tensor(s.species, device="cuda")


def _check(out, ref, label):
    errs = {"E": rel_err(float(out["energy"].cpu()), float(ref["E"].detach())),
            "E_i": rel_err(out["e_atom"].cpu().numpy(), ref["E_i"].detach().numpy()),
            "F": rel_err(out["forces"].cpu().numpy(), ref["F"].detach().numpy()),
            "W": rel_err(out["virial"].cpu().numpy(), ref["W"].detach().numpy())}
    print(f"  {label}: {errs}", flush=True)
    assert errs["E"] < TOL_E and errs["E_i"] < TOL_E, label
    assert errs["F"] < TOL_F, label
    assert errs["W"] < TOL_W, label


def test_split_lanes_on_a_lattice_match_the_oracle():
    """bcc 5^3 with two species at level 16 (rows of about 27 pairs, split into 1..8 parts)."""
    s, p = small_lattice(711, (5, 5, 5), 3.2, 0.08, 16, 2)
    ref = om.energy_forces_virial(om.Model.from_params(p), s)
    pos, sp = _dev(s)
    for k in SPLITS:
        print(f"[split lattice L16] N={s.n_atoms} lanes_per_atom={k}", flush=True)
        out = _pot(p, lanes_per_atom=k).compute(pos, sp, s.cell, e_atom=True)
        torch.cuda.synchronize()
        _check(out, ref, f"lanes {k}")


@pytest.mark.parametrize("level", [10, 20])
def test_split_lanes_on_small_triclinic_cells_match_the_oracle(level):
    """Small triclinic cells: rows with repeated partners (periodic images), rows shorter than
    the lanes of an atom, and at level 20 several moment groups (one pair pass per group)."""
    structs, p = small_batch(720 + level, 3, level, n_min=8, n_max=24)
    model = om.Model.from_params(p)
    for c, s in enumerate(structs):
        ref = om.energy_forces_virial(model, s)
        pos, sp = _dev(s)
        for k in SPLITS:
            print(f"[split L{level} cfg{c}] N={s.n_atoms} lanes_per_atom={k}", flush=True)
            out = _pot(p, lanes_per_atom=k).compute(pos, sp, s.cell, e_atom=True)
            torch.cuda.synchronize()
            _check(out, ref, f"cfg{c} lanes {k}")


def test_split_lanes_chunk_invariance_and_determinism():
    s, p = small_lattice(733, (6, 6, 6), 3.16, 0.1, 10, 1)
    pos, sp = _dev(s)
    print(f"[split chunking] N={s.n_atoms}", flush=True)
    for k in (4, 8):
        a = _pot(p, lanes_per_atom=k).compute(pos, sp, s.cell, e_atom=True)
        b = _pot(p, lanes_per_atom=k).compute(pos, sp, s.cell, e_atom=True)
        c = _pot(p, lanes_per_atom=k, chunk_atoms=37).compute(pos, sp, s.cell, e_atom=True)
        d = _pot(p, lanes_per_atom=k, chunk_atoms=64).compute(pos, sp, s.cell, e_atom=True)
        torch.cuda.synchronize()
        for key in ("energy", "forces", "virial", "e_atom"):
            assert torch.equal(a[key], b[key]), (k, key)
            assert torch.equal(a[key], d[key]), (k, key)
        for key in ("energy", "forces", "e_atom"):
            assert torch.equal(a[key], c[key]), (k, key)
        assert rel_err(c["virial"].cpu().numpy(), a["virial"].cpu().numpy()) < 1e-13


def test_split_lanes_agree_with_one_lane_per_atom():
    """Same inputs, different summation order of the row: the results agree to rounding."""
    s, p = small_lattice(744, (8, 8, 8), 3.16, 0.1, 16, 1)
    pos, sp = _dev(s)
    print(f"[split vs one lane] N={s.n_atoms}", flush=True)
    base = _pot(p, lanes_per_atom=1).compute(pos, sp, s.cell, e_atom=True)
    for k in SPLITS[1:]:
        out = _pot(p, lanes_per_atom=k).compute(pos, sp, s.cell, e_atom=True)
        torch.cuda.synchronize()
        for key in ("energy", "forces", "virial", "e_atom"):
            err = rel_err(out[key].cpu().numpy(), base[key].cpu().numpy())
            assert err < 1e-12, (k, key, err)


def test_lanes_per_atom_is_validated():
    from paper_2510_00193_amd._lib import MtpError
    s, p = small_lattice(755, (2, 2, 2), 3.16, 0.05, 6, 1)
    for bad in (3, -1, 16):
        with pytest.raises(MtpError):
            _pot(p, lanes_per_atom=bad)
    # chunks are capped so that a lane's byte offset in a row fits 32 bits
    with pytest.raises(MtpError):
        _pot(p, chunk_atoms=(1 << 28) + 1)
