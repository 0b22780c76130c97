"""The FP32-moment / FP64-accumulation form: errors against the float64 oracle, stated."""
import numpy as np
import pytest
import torch

from helpers import rel_err, small_lattice
from oracle import mtp as om

pytestmark = pytest.mark.gpu

# Bounds of the binary32 form (max-norm relative); measured values are printed.
FP32_TOL = {"E": 1e-5, "F": 1e-4, "W": 1e-4}


@pytest.mark.parametrize("level,species", [(10, 1), (16, 2)])
def test_fp32_form_error_against_oracle(level, species):
    s, p = small_lattice(1001 + level, (4, 4, 4), 3.16, 0.1, level, species)
    from paper_2510_00193_amd import Potential
    pot = Potential.from_params(p, precision="fp32")
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    print(f"[fp32 L{level}] N={s.n_atoms}", flush=True)
    out = pot.compute(pos, sp, s.cell)
    torch.cuda.synchronize()
    ref = om.energy_forces_virial(om.Model.from_params(p), s)
    errs = {"E": rel_err(float(out["energy"].cpu()), float(ref["E"].detach())),
            "F": rel_err(out["forces"].cpu().numpy(), ref["F"].detach().numpy()),
            "W": rel_err(out["virial"].cpu().numpy(), ref["W"].detach().numpy())}
    print(f"  fp32 form errors {errs}", flush=True)
    for k, v in errs.items():
        assert v < FP32_TOL[k], (k, v)
    # forces still sum to zero to binary64 rounding: the gather is exact pairwise
    f = out["forces"].cpu().numpy()
    assert np.abs(f.sum(axis=0)).max() <= 1e-9 * np.abs(f).max()
