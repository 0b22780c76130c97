"""Pins of the oracle's basis enumeration and radial basis (CPU only)."""
import os

import numpy as np
import pytest
import torch
from numpy.polynomial import chebyshev as npcheb

from oracle import basis as ob
from oracle import mtp as om

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


def test_counts_match_hand_and_table():
    for row in _read_rows("basis_counts.txt"):
        level, n_alpha, n_conn, n_mom, c, n_mu, max_nu = map(int, row.split())
        b = om.basis_for(level)
        assert len(b) == n_alpha, level
        assert sum(x.connected() for x in b) == n_conn, level
        mom = ob.used_moments(b)
        assert len(mom) == n_mom
        assert sum((nu + 1) * (nu + 2) // 2 for _, nu in mom) == c
        assert ob.radial_count(level, b) == n_mu
        assert max(nu for _, nu in mom) == max_nu


def test_level10_hand_list_and_order():
    want = []
    for row in _read_rows("basis_L10_hand.txt"):
        labs, edges = row.split("|")
        labels = tuple(tuple(int(v) for v in t.split(",")) for t in labs.split())
        want.append((labels, tuple(int(v) for v in edges.split())))
    got = [(b.labels, b.edges) for b in ob.enumerate_basis(10)]
    assert got == want


def test_isomorphic_graphs_collapse():
    # (0,2),(0,2),(0,2),(0,2) at level 16: the 4-cycle with single edges and the
    # double-edge pairings are distinct classes; relabelled copies are not.
    b = [x for x in ob.enumerate_basis(16) if x.labels == ((0, 2),) * 4]
    keys = {x.edges for x in b}
    assert len(keys) == len(b)
    # the two classes: disconnected double pairs, and the 4-cycle
    assert len(b) == 2


def test_chebyshev_vs_numpy_and_cosine():
    u = np.linspace(-1.3, 1.3, 57)
    t = om.chebyshev(torch.as_tensor(u), 11).numpy()
    for beta in range(11):
        coef = np.zeros(beta + 1)
        coef[beta] = 1.0
        np.testing.assert_allclose(t[:, beta], npcheb.chebval(u, coef), rtol=1e-13, atol=1e-13)
    th = np.linspace(0.0, np.pi, 23)
    t = om.chebyshev(torch.as_tensor(np.cos(th)), 9).numpy()
    for beta in range(9):
        np.testing.assert_allclose(t[:, beta], np.cos(beta * th), atol=1e-13)


def test_radial_basis_endpoints():
    r_min, r_cut = 2.0, 5.0
    q = om.radial_basis(torch.tensor([r_min, r_cut, 3.5]), r_min, r_cut, 6).numpy()
    # at r_min: u = -1, T_b(-1) = (-1)^b, times (r_cut - r_min)^2
    np.testing.assert_allclose(q[0], [(-1) ** b * 9.0 for b in range(6)], rtol=1e-15)
    np.testing.assert_allclose(q[1], 0.0, atol=0)
    # at the midpoint u = 0: T_b(0) = cos(b pi / 2)
    np.testing.assert_allclose(q[2], [np.cos(b * np.pi / 2) * 2.25 for b in range(6)], atol=1e-15)
