"""mtp_compute_static under stream capture: a captured evaluation replayed several times, with
the positions updated in place and eager library work between the replays, matches the eager
call on the same inputs bit for bit at every replay."""
import numpy as np
import pytest
import torch

from helpers import small_lattice

pytestmark = pytest.mark.gpu


def test_captured_static_evaluation_replays_match_eager():
    from paper_2510_00193_amd import Potential
    s, p = small_lattice(951, (4, 4, 4), 3.16, 0.05, 10, 1)
    pot = Potential.from_params(p)
    other = Potential.from_params(p)  # eager work between the replays (its own workspace)
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    nl = pot.neighbors(pos, sp, s.cell)
    print(f"[graph] N={s.n_atoms} pairs={nl.n_pairs}", flush=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pot.compute_static(pos, sp, s.cell, nl)  # warm-up on the capturing stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = pot.compute_static(pos, sp, s.cell, nl)
    rng = np.random.default_rng(952)
    base = pos.clone()
    for rep in range(4):
        pos.copy_(base + torch.as_tensor(rng.normal(0.0, 0.01, size=tuple(base.shape)), device="cuda"))
        other.compute(pos, sp, s.cell)  # eager library work, neighbour list built inside
        g.replay()
        torch.cuda.synchronize()
        ref = pot.compute_static(pos, sp, s.cell, nl)
        torch.cuda.synchronize()
        print(f"  replay {rep}: E={float(out['energy'].cpu()):.12e}", flush=True)
        for k in ("energy", "forces", "virial"):
            assert torch.equal(out[k], ref[k]), (rep, k)
