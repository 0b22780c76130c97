"""Pins of the oracle's periodic neighbour list (CPU only)."""
import itertools

import numpy as np
import pytest

import workloads as wl
from oracle import neighbors as onb


def _naive_pairs(pos, cell, r_cut, nmax):
    """Independent brute force: plain Python loops over every (i, j, n) in a big box."""
    out = set()
    rc2 = r_cut * r_cut
    n_atoms = len(pos)
    for i in range(n_atoms):
        for j in range(n_atoms):
            for n1, n2, n3 in itertools.product(range(-nmax, nmax + 1), repeat=3):
                if i == j and n1 == n2 == n3 == 0:
                    continue
                t = [(n1 * cell[0][a] + n2 * cell[1][a]) + n3 * cell[2][a] for a in range(3)]
                d = [(pos[j][a] - pos[i][a]) + t[a] for a in range(3)]
                dd = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
                if dd < rc2:
                    out.add((i, j, n1, n2, n3))
    return out


def _as_set(nl):
    return {(int(i), int(j), int(n[0]), int(n[1]), int(n[2]))
            for i, j, n in zip(nl["i"], nl["j"], nl["n"])}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_naive_loops_on_thin_triclinic_cells(seed):
    rng = np.random.default_rng(100 + seed)
    (s,) = wl.random_cell_batch(rng, 1, 5, 9, 0.06, 1.8, 2)
    r_cut = 5.5
    nl = onb.neighbor_csr(s.pos, s.cell, r_cut)
    want = _naive_pairs(s.pos.tolist(), s.cell.tolist(), r_cut, 4)
    assert _as_set(nl) == want
    # a cell thinner than the cutoff: every atom sees some of its own images
    assert any(int(i) == int(j) for i, j in zip(nl["i"], nl["j"]))


def test_prefilter_is_exact():
    rng = np.random.default_rng(7)
    sites, cell = wl.bcc_sites(3, 3, 3, 3.16)
    pos = wl.jitter_wrap(sites, cell, 0.1, rng)
    a = onb.neighbor_csr(pos, cell, 5.0, prefilter=True)
    b = onb.neighbor_csr(pos, cell, 5.0, prefilter=False)
    for k in ("off", "j", "shift", "rev"):
        np.testing.assert_array_equal(a[k], b[k])


def test_perfect_lattice_shell_counts():
    sites, cell = wl.bcc_sites(4, 4, 4, 3.16)
    nl = onb.neighbor_csr(sites, cell, 5.0)
    assert np.all(np.diff(nl["off"]) == 8 + 6 + 12)
    sites, cell = wl.fcc_sites(3, 3, 3, 3.52)
    nl = onb.neighbor_csr(sites, cell, 5.0)
    # 12 + 6 + 24 + 12 (the a*sqrt(2) = 4.978 shell lies inside 5.0)
    assert np.all(np.diff(nl["off"]) == 54)


def test_canonical_order_and_reverse_map():
    rng = np.random.default_rng(3)
    (s,) = wl.random_cell_batch(rng, 1, 20, 20, 0.06, 1.8, 1)
    nl = onb.neighbor_csr(s.pos, s.cell, 5.5)
    off = nl["off"]
    for i in range(len(off) - 1):
        keys = [(int(nl["j"][p]),) + tuple(int(v) for v in nl["n"][p]) for p in range(off[i], off[i + 1])]
        assert keys == sorted(keys)
        assert len(set(keys)) == len(keys)
    rev = nl["rev"]
    np.testing.assert_array_equal(rev[rev], np.arange(len(rev)))
    np.testing.assert_array_equal(nl["i"][rev], nl["j"])
    np.testing.assert_array_equal(nl["n"][rev], -nl["n"])
    d = onb.displacements(s.pos, s.cell, nl["i"], nl["j"], nl["n"])
    # the mirrored displacement is the exact negative (same expression, round-to-nearest)
    np.testing.assert_array_equal(d[rev], -d)


def test_shift_packing_roundtrip():
    n = np.array([[0, 0, 0], [-1, 2, -3], [127, -128, 5]])
    np.testing.assert_array_equal(onb.unpack_shift(onb.pack_shift(n)), n)
    assert onb.pack_shift(np.array([-1, 0, 1])) == (0xFF | (1 << 16))


def test_cutoff_is_strict():
    cell = np.diag([10.0, 10.0, 10.0])
    pos = np.array([[0.0, 0.0, 0.0], [5.0, 0.0, 0.0]])
    nl = onb.neighbor_csr(pos, cell, 5.0)
    assert len(nl["j"]) == 0
    pos = np.array([[0.0, 0.0, 0.0], [4.999999, 0.0, 0.0]])
    nl = onb.neighbor_csr(pos, cell, 5.0)
    assert len(nl["j"]) == 2
