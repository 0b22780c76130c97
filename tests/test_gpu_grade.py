"""GPU parity of the neighbourhood-mode extrapolation grade (float64 and FP32-split MFMA)."""
import numpy as np
import pytest
import torch

import workloads as wl
from helpers import TOL_GRADE, small_lattice
from oracle import mtp as om

pytestmark = pytest.mark.gpu


def _setup(seed=808, rep=(3, 3, 3)):
    s, p = small_lattice(seed, rep, 3.52, 0.15, 16, 3, lattice="fcc")
    model = om.Model.from_params(p)
    ref = om.energy_forces_virial(model, s)
    b = ref["B"].detach().numpy()
    return s, p, b


def _grade_err(got, want):
    return float(np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want))))


def _run(p, s, ainv, mode, **kw):
    from paper_2510_00193_amd import Potential
    pot = Potential.from_params(p, **kw)
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    out = pot.grade(pos, sp, s.cell, torch.as_tensor(ainv, device="cuda"), mode=mode)
    torch.cuda.synchronize()
    return out


def test_grade_fp64_matches_oracle():
    s, p, b = _setup()
    rng = np.random.default_rng(9)
    _, ainv = wl.draw_active_set(rng, b.shape[1])
    want = om.grade(b, ainv)
    print(f"[grade fp64] N={s.n_atoms} n_alpha={b.shape[1]}", flush=True)
    out = _run(p, s, ainv, "fp64")
    got = out["grade"].cpu().numpy()
    assert _grade_err(got, want) < TOL_GRADE
    assert float(out["grade_max"].cpu()) == pytest.approx(want.max(), rel=TOL_GRADE)


def test_grade_fp32split_error_is_bounded():
    s, p, b = _setup()
    rng = np.random.default_rng(9)
    _, ainv = wl.draw_active_set(rng, b.shape[1])
    want = om.grade(b, ainv)
    print(f"[grade fp32split] N={s.n_atoms}", flush=True)
    got = _run(p, s, ainv, "fp32split")["grade"].cpu().numpy()
    err = _grade_err(got, want)
    print(f"fp32-split grade error {err:.3e}", flush=True)
    assert err < 1e-5


def test_grade_maxvol_active_set_rows_are_one():
    """A built from the oracle's B rows of n_alpha chosen atoms: those atoms have grade 1."""
    s, p, b = _setup(seed=809, rep=(4, 4, 3))
    rng = np.random.default_rng(10)
    chosen = rng.choice(s.n_atoms, size=b.shape[1], replace=False)
    ainv = np.linalg.inv(b[chosen])
    print(f"[grade maxvol] N={s.n_atoms}", flush=True)
    got = _run(p, s, ainv, "fp64")["grade"].cpu().numpy()
    np.testing.assert_allclose(got[chosen], 1.0, rtol=1e-7)
    assert _grade_err(got, om.grade(b, ainv)) < 1e-7


def test_grade_thresholds_and_chunks():
    s, p, b = _setup()
    ainv = np.eye(b.shape[1])
    want = om.grade(b, ainv)
    gmax = want.max()
    print(f"[grade thresholds] gmax={gmax:.3e}", flush=True)
    out = _run(p, s, ainv, "fp64", chunk_atoms=29, grade_select=gmax * 0.5, grade_break=gmax * 2)
    assert out["status"] == 9
    assert _grade_err(out["grade"].cpu().numpy(), want) < TOL_GRADE
    out = _run(p, s, ainv, "fp64", grade_select=gmax * 0.25, grade_break=gmax * 0.5)
    assert out["status"] == 8
    out = _run(p, s, ainv, "fp64", grade_select=gmax * 4, grade_break=gmax * 8)
    assert out["status"] == 0


def test_config_grade_matches_oracle_and_maxvol():
    """Configuration mode: descriptor sum_i B_i and max |b Ainv| against the oracle on small
    triclinic configurations; configurations whose oracle descriptors form A have grade 1;
    thresholds return their status codes; an empty configuration has grade 0."""
    from paper_2510_00193_amd import Potential
    from helpers import small_batch
    structs, p = small_batch(611, 19, 10, n_min=8, n_max=40)
    model = om.Model.from_params(p)
    n_alpha = len(model.basis)
    desc = np.array([om.config_descriptor(om.energy_forces_virial(model, st)["B"].detach().numpy())
                     for st in structs])
    ainv = np.linalg.inv(desc[:n_alpha])
    pot = Potential.from_params(p)
    a_dev = torch.as_tensor(ainv, device="cuda")
    for k, st in enumerate(structs):
        print(f"[config grade] cfg {k} N={st.n_atoms}", flush=True)
        out = pot.grade_config(torch.as_tensor(st.pos, device="cuda"), torch.as_tensor(st.species, device="cuda"),
                               st.cell, a_dev)
        torch.cuda.synchronize()
        want = om.config_grade(desc[k][None, :], ainv)
        got_desc = out["descriptor"].cpu().numpy()
        assert np.max(np.abs(got_desc - desc[k])) / np.max(np.abs(desc[k])) < 1e-10
        assert _grade_err(np.array([float(out["grade"].cpu())]), np.array([want])) < TOL_GRADE
        if k < n_alpha:
            assert abs(float(out["grade"].cpu()) - 1.0) < 1e-8
    # thresholds on the last configuration (grade well above 1 for a configuration outside A)
    st = structs[-1]
    g = float(pot.grade_config(torch.as_tensor(st.pos, device="cuda"), torch.as_tensor(st.species, device="cuda"),
                               st.cell, a_dev)["grade"].cpu())
    from paper_2510_00193_amd import _lib
    pot_sel = Potential.from_params(p, grade_select=0.5 * g)
    pot_brk = Potential.from_params(p, grade_select=0.25 * g, grade_break=0.5 * g)
    args = (torch.as_tensor(st.pos, device="cuda"), torch.as_tensor(st.species, device="cuda"), st.cell, a_dev)
    assert pot_sel.grade_config(*args)["status"] == _lib.MTP_GRADE_SELECT
    assert pot_brk.grade_config(*args)["status"] == _lib.MTP_GRADE_BREAK
    empty = pot.grade_config(torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                             torch.zeros((0,), dtype=torch.int32, device="cuda"), np.eye(3) * 20.0, a_dev)
    torch.cuda.synchronize()
    assert float(empty["grade"].cpu()) == 0.0
