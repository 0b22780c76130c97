"""Parity at the workloads' full sizes, in the launch configuration the benchmark times.

The oracle computes sampled outputs one by one (neighbour rows, site energies, basis
vectors and forces of a few atoms); properties that hold at any size are checked on the
whole system.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from helpers import TOL_E, TOL_F, TOL_GRADE, rel_err
from oracle import mtp as om
from oracle import neighbors as onb

pytestmark = pytest.mark.gpu


def _load(k):
    from paper_2510_00193_amd import Potential, level_info
    info = level_info(wl.WORKLOADS[k]["level"])
    w = wl.workload(k, info["n_alpha"], info["n_mu"])
    (s,) = w["structures"]
    return s, w, Potential.from_params(w["params"])


def _sampled_checks(s, p, pot, atoms, label):
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    print(f"[{label}] N={s.n_atoms}", flush=True)
    nl = pot.neighbors(pos, sp, s.cell)
    out = pot.compute(pos, sp, s.cell, nlist=nl, e_atom=True)
    torch.cuda.synchronize()
    off = nl.off.cpu().numpy()
    j = nl.j.cpu().numpy()
    sh = onb.unpack_shift(nl.shift.cpu().numpy())
    rev = nl.rev.cpu().numpy()
    # the whole list: mirrored pairs, sorted rows
    assert np.array_equal(rev[rev], np.arange(len(rev)))
    assert np.array_equal(j[rev], np.repeat(np.arange(s.n_atoms), np.diff(off)))
    model = om.Model.from_params(p)
    rows, e_ref, _ = om.sampled_site_values(model, s, atoms)
    for a, (js, ns) in zip(atoms, rows):
        np.testing.assert_array_equal(j[off[a]:off[a + 1]], js)
        np.testing.assert_array_equal(sh[off[a]:off[a + 1]], ns)
    e_gpu = out["e_atom"].cpu().numpy()
    assert rel_err(e_gpu[atoms], e_ref) < TOL_E
    f_ref = om.sampled_forces(model, s, atoms[:3])
    f_gpu = out["forces"].cpu().numpy()
    # forces relative to the largest force of the system
    assert np.max(np.abs(f_gpu[atoms[:3]] - f_ref)) / np.abs(f_gpu).max() < TOL_F
    assert np.abs(f_gpu.sum(axis=0)).max() <= 1e-9 * np.abs(f_gpu).max()
    etot = float(out["energy"].cpu())
    assert abs(etot - e_gpu.sum()) <= 1e-12 * np.abs(e_gpu).sum()
    return pot, pos, sp, nl


def test_workload2_sampled():
    s, w, pot = _load(2)
    rng = np.random.default_rng(22)
    _sampled_checks(s, w["params"], pot, list(rng.choice(s.n_atoms, 6, replace=False)), "bcc-20^3-2sp-L16")


def test_workload3_sampled():
    s, w, pot = _load(3)
    rng = np.random.default_rng(33)
    atoms = [0, s.n_atoms - 1] + list(rng.choice(s.n_atoms, 4, replace=False))
    _sampled_checks(s, w["params"], pot, atoms, "bcc-80^3-L16")


def test_workload4_sampled_grade():
    s, w, pot = _load(4)
    rng = np.random.default_rng(44)
    atoms = list(rng.choice(s.n_atoms, 6, replace=False))
    pot, pos, sp, nl = _sampled_checks(s, w["params"], pot, atoms, "fcc-50x50x25-3sp-L16")
    ainv = w["extra"]["active_set_inv"]
    out = pot.grade(pos, sp, s.cell, torch.as_tensor(ainv, device="cuda"), nlist=nl)
    torch.cuda.synchronize()
    _, _, b_ref = om.sampled_site_values(om.Model.from_params(w["params"]), s, atoms)
    g_ref = om.grade(b_ref, ainv)
    g = out["grade"].cpu().numpy()
    assert np.max(np.abs(g[atoms] - g_ref) / np.maximum(1.0, g_ref)) < TOL_GRADE
    assert float(out["grade_max"].cpu()) == pytest.approx(g.max(), rel=0, abs=0)


def test_workload2_parameter_gradient_full_size():
    """VJP of (E, F) at 16,000 atoms against the oracle accumulated over centre chunks."""
    s, w, pot = _load(2)
    p = w["params"]
    rng = np.random.default_rng(222)
    fbar = rng.normal(size=(s.n_atoms, 3))
    ebar = 0.37
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    print(f"[vjp full size] N={s.n_atoms}", flush=True)
    got = pot.param_grad(pos, sp, s.cell, ebar, torch.as_tensor(fbar, device="cuda"))
    torch.cuda.synchronize()
    got = [x.cpu().numpy() for x in got]
    nl = onb.neighbor_csr(s.pos, s.cell, p.r_cut)
    want = om.param_vjp_chunked(om.Model.from_params(p), s, ebar, fbar, nl, chunk=1000)
    for name, g, r in zip(("d_linear", "d_radial", "d_shift"), got, want):
        err = rel_err(g, r)
        print(f"  {name}: rel err {err:.2e}", flush=True)
        assert err < 1e-9, name


def test_workload3_fp32_form_sampled_against_oracle():
    """The binary32-moment form at 1,024,000 atoms: site energies and forces of sampled atoms
    against the float64 oracle (errors stated; bounds as for the small cases)."""
    from paper_2510_00193_amd import Potential, level_info
    info = level_info(16)
    w = wl.workload(3, info["n_alpha"], info["n_mu"])
    (s,) = w["structures"]
    p = w["params"]
    pot = Potential.from_params(p, precision="fp32")
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    print(f"[fp32 bcc-80^3-L16] N={s.n_atoms}", flush=True)
    out = pot.compute(pos, sp, s.cell, e_atom=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(333)
    atoms = list(rng.choice(s.n_atoms, 6, replace=False))
    model = om.Model.from_params(p)
    _, e_ref, _ = om.sampled_site_values(model, s, atoms)
    e_gpu = out["e_atom"].cpu().numpy()[atoms]
    f_ref = om.sampled_forces(model, s, atoms[:3])
    f_all = out["forces"].cpu().numpy()
    e_err = float(np.max(np.abs(e_gpu - e_ref)) / np.max(np.abs(e_ref)))
    f_err = float(np.max(np.abs(f_all[atoms[:3]] - f_ref)) / np.abs(f_all).max())
    print(f"  fp32 form vs oracle: site energy {e_err:.2e}, force {f_err:.2e}", flush=True)
    assert e_err < 1e-5
    assert f_err < 1e-4


def test_workload4_fp32split_grade_sampled_against_oracle():
    """The FP32-split grade product at 250,000 atoms against the oracle's float64 grade."""
    s, w, pot = _load(4)
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    ainv = w["extra"]["active_set_inv"]
    print(f"[fp32split grade fcc-50x50x25] N={s.n_atoms}", flush=True)
    out = pot.grade(pos, sp, s.cell, torch.as_tensor(ainv, device="cuda"), mode="fp32split")
    torch.cuda.synchronize()
    rng = np.random.default_rng(444)
    atoms = list(rng.choice(s.n_atoms, 6, replace=False))
    _, _, b_ref = om.sampled_site_values(om.Model.from_params(w["params"]), s, atoms)
    g_ref = om.grade(b_ref, ainv)
    g = out["grade"].cpu().numpy()[atoms]
    err = float(np.max(np.abs(g - g_ref) / np.maximum(1.0, g_ref)))
    print(f"  fp32-split grade vs oracle: {err:.2e}", flush=True)
    assert err < 1e-5


def test_workload2_virial_is_strain_derivative():
    """At 16,000 atoms the virial equals -dE/d(strain) (a property at any size), by central
    differences of the GPU energy under R -> (I + e) R, H -> H (I + e)^T."""
    s, w, pot = _load(2)
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    print(f"[virial strain bcc-20^3] N={s.n_atoms}", flush=True)
    wv = pot.compute(pos, sp, s.cell)["virial"].cpu().numpy()
    h = 1e-6
    order = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for k in (0, 4):
        a, b = order[k]
        es = []
        for sign in (1.0, -1.0):
            eps = np.zeros((3, 3))
            eps[a, b] = sign * h
            if a != b:
                eps[b, a] = sign * h  # symmetric strain: W is symmetric
            m = np.eye(3) + eps
            pp = torch.as_tensor(s.pos @ m.T, device="cuda")
            es.append(float(pot.compute(pp, sp, s.cell @ m.T, forces=False, virial=False)["energy"].cpu()))
        de = (es[0] - es[1]) / (2 * h)
        want = -de if a == b else -de / 2.0
        print(f"  W[{a}{b}] {wv[k]:.10e} fd {want:.10e}", flush=True)
        assert abs(wv[k] - want) <= 1e-6 * np.abs(wv).max()
