"""The coefficient adjoint behind torch.autograd: gradients of the energy + force loss
(E - E0)^2 + sum |F - F0|^2 through MTPFunction / MTPBatchFunction against the oracle's
vector-Jacobian product, against central differences of the GPU loss, and the refusals
(position derivatives, double backward)."""
import numpy as np
import pytest
import torch

import workloads as wl
from helpers import rel_err, small_batch, small_lattice
from oracle import mtp as om
from oracle import neighbors as onb

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-9


def _coefs(p, requires_grad=True):
    out = []
    for a in (p.linear, p.radial, p.shift):
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
        out.append(t.requires_grad_(requires_grad))
    return out


def _oracle_targets(p, s, seed):
    rng = np.random.default_rng(seed)
    tp = wl.perturb_params(rng, p)
    tgt = om.energy_forces_virial(om.Model.from_params(tp), s)
    return float(tgt["E"].detach()), tgt["F"].detach().numpy()


def test_autograd_loss_gradient_matches_oracle():
    from paper_2510_00193_amd import Potential, energy_forces
    s, p = small_lattice(3101, (3, 3, 3), 3.2, 0.08, 16, 2)
    e0, f0 = _oracle_targets(p, s, 31)
    model = om.Model.from_params(p)
    cur = om.energy_forces_virial(model, s)
    ebar = 2.0 * (float(cur["E"].detach()) - e0)
    fbar = 2.0 * (cur["F"].detach().numpy() - f0)
    want = om.param_vjp(model, s, ebar, fbar, onb.neighbor_csr(s.pos, s.cell, p.r_cut))
    print(f"[autograd L16] N={s.n_atoms}", flush=True)
    pot = Potential.from_params(p)
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    xi, c, sh = _coefs(p)
    e, f = energy_forces(pot, pos, sp, s.cell, xi, c, sh)
    loss = (e - e0) ** 2 + ((f - torch.as_tensor(f0, device="cuda")) ** 2).sum()
    got = torch.autograd.grad(loss, [xi, c, sh])
    torch.cuda.synchronize()
    for name, g, w in zip(("d_linear", "d_radial", "d_shift"), got, want):
        err = rel_err(g.cpu().numpy(), w)
        print(f"  {name}: rel err {err:.2e}", flush=True)
        assert err < TOL_GRAD, name


def test_autograd_directional_derivative_vs_central_difference():
    """<grad L, v> against (L(theta + h v) - L(theta - h v)) / 2h, all on the GPU."""
    from paper_2510_00193_amd import Potential, energy_forces
    s, p = small_lattice(3102, (3, 3, 3), 3.16, 0.08, 10, 2)
    rng = np.random.default_rng(32)
    f0 = torch.as_tensor(rng.normal(size=(s.n_atoms, 3)), device="cuda")
    e0 = 0.5
    pot = Potential.from_params(p)
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    xi, c, sh = _coefs(p)

    def loss(a, b, d):
        e, f = energy_forces(pot, pos, sp, s.cell, a, b, d)
        return (e - e0) ** 2 + ((f - f0) ** 2).sum()

    grads = torch.autograd.grad(loss(xi, c, sh), [xi, c, sh])
    v = [torch.as_tensor(rng.normal(size=t.shape), device="cuda") for t in (xi, c, sh)]
    scale = [t.detach().abs().max() for t in (xi, c, sh)]
    v = [vi * si for vi, si in zip(v, scale)]
    slope = float(sum((g * vi).sum() for g, vi in zip(grads, v)))
    h = 1e-6
    with torch.no_grad():
        lp = float(loss(*[t.detach() + h * vi for t, vi in zip((xi, c, sh), v)]))
        lm = float(loss(*[t.detach() - h * vi for t, vi in zip((xi, c, sh), v)]))
    fd = (lp - lm) / (2 * h)
    print(f"[autograd fd L10] slope {slope:.10e} fd {fd:.10e}", flush=True)
    assert abs(slope - fd) <= 1e-6 * max(abs(fd), 1e-12)


def test_autograd_refuses_position_and_second_derivatives():
    from paper_2510_00193_amd import Potential, energy_forces
    s, p = small_lattice(3103, (2, 2, 2), 3.16, 0.05, 10, 1)
    pot = Potential.from_params(p)
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    xi, c, sh = _coefs(p)
    with pytest.raises(NotImplementedError):
        energy_forces(pot, pos.clone().requires_grad_(True), sp, s.cell, xi, c, sh)
    e, f = energy_forces(pot, pos, sp, s.cell, xi, c, sh)
    (g,) = torch.autograd.grad(e + f.square().sum(), [xi], create_graph=True)
    with pytest.raises(RuntimeError):
        torch.autograd.grad(g.sum(), [xi])


def test_batch_autograd_matches_oracle_sum():
    from paper_2510_00193_amd import Batch, Potential, batch_energy_forces
    structs, p = small_batch(3104, 4, 10, n_min=8, n_max=30)
    off, pos, species, cells = wl.batch_arrays(structs)
    rng = np.random.default_rng(34)
    tp = wl.perturb_params(rng, p)
    model, tmodel = om.Model.from_params(p), om.Model.from_params(tp)
    grads = [np.zeros(np.shape(p.linear)), np.zeros(np.shape(p.radial)), np.zeros(np.shape(p.shift))]
    e0, f0 = [], []
    for s in structs:
        nl = onb.neighbor_csr(s.pos, s.cell, p.r_cut)
        cur, tgt = om.energy_forces_virial(model, s, nl), om.energy_forces_virial(tmodel, s, nl)
        e0.append(float(tgt["E"].detach()))
        f0.append(tgt["F"].detach().numpy())
        de = float(cur["E"].detach()) - e0[-1]
        df = cur["F"].detach().numpy() - f0[-1]
        for acc, g in zip(grads, om.param_vjp(model, s, 2 * de, 2 * df, nl)):
            acc += g
    print(f"[batch autograd L10] {len(structs)} configurations, {off[-1]} atoms", flush=True)
    pot = Potential.from_params(p)
    b = Batch(pot, off, torch.as_tensor(pos, device="cuda"), torch.as_tensor(species, device="cuda"), cells)
    xi, c, sh = _coefs(p)
    e, f = batch_energy_forces(b, xi, c, sh)
    e0d = torch.as_tensor(np.array(e0), device="cuda")
    f0d = torch.as_tensor(np.concatenate(f0), device="cuda")
    loss = ((e - e0d) ** 2).sum() + ((f - f0d) ** 2).sum()
    got = torch.autograd.grad(loss, [xi, c, sh])
    torch.cuda.synchronize()
    for name, g, w in zip(("d_linear", "d_radial", "d_shift"), got, grads):
        err = rel_err(g.cpu().numpy(), w)
        print(f"  {name}: rel err {err:.2e}", flush=True)
        assert err < TOL_GRAD, name
