"""GPU checks of the long fixed-order row sums (64 workgroups per row, then a sum of the parts)
against the same sums taken chunk by chunk with one workgroup per row: the configuration
descriptor sum_i B_i and the parameter gradient over 20,000 atoms.  Both orders are exact up
to rounding, so they agree to a few ulps of the terms' magnitude; each is also pinned to the
oracle by the smaller parity tests."""
import numpy as np
import pytest
import torch

from helpers import rel_err, small_lattice

pytestmark = pytest.mark.gpu


def _pot(p, **kw):
    from paper_2510_00193_amd import Potential
    return Potential.from_params(p, **kw)


def _system():
    s, p = small_lattice(931, (20, 20, 25), 3.16, 0.08, 10, 2)
    assert s.n_atoms >= 20000  # above the size where the two-level row sums take over
    return s, p


def test_descriptor_two_level_sum_matches_chunked_sum():
    s, p = _system()
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    print(f"[descriptor sums] N={s.n_atoms}", flush=True)
    na = _pot(p).n_alpha
    ainv = torch.eye(na, dtype=torch.float64, device="cuda")
    whole = _pot(p).grade_config(pos, sp, s.cell, ainv)["descriptor"]
    chunked = _pot(p, chunk_atoms=4096).grade_config(pos, sp, s.cell, ainv)["descriptor"]
    torch.cuda.synchronize()
    err = rel_err(whole.cpu().numpy(), chunked.cpu().numpy())
    print(f"  descriptor, two-level vs chunked: {err:.2e}", flush=True)
    assert err < 1e-12


def test_parameter_gradient_two_level_sum_matches_chunked_sum():
    s, p = _system()
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    print(f"[gradient sums] N={s.n_atoms}", flush=True)
    rng = np.random.default_rng(932)
    fbar = torch.as_tensor(rng.normal(size=(s.n_atoms, 3)), device="cuda")
    whole = _pot(p).param_grad(pos, sp, s.cell, 0.7, fbar)
    chunked = _pot(p, chunk_atoms=4096).param_grad(pos, sp, s.cell, 0.7, fbar)
    torch.cuda.synchronize()
    for name, a, b in zip(("dxi", "dc", "ds"), whole, chunked):
        err = rel_err(a.cpu().numpy(), b.cpu().numpy())
        print(f"  {name}, two-level vs chunked: {err:.2e}", flush=True)
        assert err < 1e-12, name
