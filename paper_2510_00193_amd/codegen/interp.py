"""Reference interpreter of a compiled program (float64, NumPy, batched over atoms).

It runs exactly the operations the generated device code runs, in the same
order per block, and is used to check the program compiler on the CPU.
"""
from __future__ import annotations

import numpy as np

from .program import Program


def moments(prog: Program, d, f, centre, n_atoms):
    """m[atom, e] = sum_j f[j, mu_e] x^a y^b z^c for the flat component layout."""
    m = np.zeros((n_atoms, prog.n_mom))
    for e, (mu, a, b, c) in enumerate(prog.layout.items):
        val = f[:, mu] * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c
        np.add.at(m[:, e], centre, val)
    return m


def _get(ref, m, t, cvals):
    kind, k = ref
    if kind == "m":
        return m[:, k]
    if kind == "t":
        return t[k]
    return cvals[k]


def forward(prog: Program, m):
    """Connected outputs C [atoms, n_comp] and basis values B [atoms, n_alpha]."""
    n = m.shape[0]
    cvals = np.zeros((prog.n_comp, n))
    for blk in prog.blocks:
        t = np.zeros((blk.n_temp, n))
        for dst, x, y, w in blk.ops:
            xv = _get(x, m, t, cvals)
            val = xv if y is None else float(w) * xv * m[:, y[1]]
            if dst[0] == "t":
                t[dst[1]] += val
            else:
                cvals[dst[1]] += val
    b = np.zeros((prog.n_alpha, n))
    for a, (parent, comp) in enumerate(prog.trie):
        b[a] = cvals[comp] if parent < 0 else b[parent] * cvals[comp]
    return cvals.T, b.T


def reverse(prog: Program, m, cbar):
    """mbar [atoms, n_mom] = sum_q cbar_q dC_q/dm."""
    n = m.shape[0]
    mbar = np.zeros_like(m)
    for blk in prog.blocks:
        t = np.zeros((blk.n_temp, n))
        for dst, x, y, w in blk.ops:     # forward values of the temporaries
            if dst[0] == "t":
                xv = m[:, x[1]] if x[0] == "m" else t[x[1]]
                t[dst[1]] += float(w) * xv * m[:, y[1]]
        tb = np.zeros((blk.n_temp, n))
        for dst, x, y, w in reversed(blk.ops):
            db = cbar[:, dst[1]] if dst[0] == "c" else tb[dst[1]]
            if y is None:
                mbar[:, x[1]] += db
                continue
            xv = m[:, x[1]] if x[0] == "m" else t[x[1]]
            yv = m[:, y[1]]
            if x[0] == "m":
                mbar[:, x[1]] += float(w) * db * yv
            else:
                tb[x[1]] += float(w) * db * yv
            mbar[:, y[1]] += float(w) * db * xv
    return mbar


def products_adjoint(prog: Program, cvals, b, xi):
    """cbar [atoms, n_comp] for E = sum_alpha xi_alpha B_alpha, via the product trie."""
    n = cvals.shape[0]
    bbar = np.tile(np.asarray(xi, dtype=np.float64)[:, None], (1, n))
    cbar = np.zeros((prog.n_comp, n))
    for a in range(prog.n_alpha - 1, -1, -1):
        parent, comp = prog.trie[a]
        if parent < 0:
            cbar[comp] += bbar[a]
        else:
            cbar[comp] += bbar[a] * b[:, parent]
            bbar[parent] += bbar[a] * cvals[:, comp]
    return cbar.T
