"""Oracle: brute-force periodic neighbour list (test infrastructure only).

The paper's GPU variants run on LAMMPS neighbour lists (Section 2.3 asks for
"newton on neigh half"); it fixes no list format.  The list here is the full,
canonical one the GPU library also returns:

* pairs (j, n) with n in Z^3 and 0 < |R_j - R_i + n H|^2 < r_cut^2, j = i
  allowed when n != 0 (an atom sees its own periodic images in thin cells);
* the squared distance is formed by one fixed expression in IEEE binary64,
  round-to-nearest, no fused multiply-add:
      t_a  = (n1*H[0][a] + n2*H[1][a]) + n3*H[2][a]
      d_a  = (R[j][a] - R[i][a]) + t_a
      dd   = (d_0*d_0 + d_1*d_1) + d_2*d_2
  and the test is the strict ``dd < r_cut*r_cut``;
* each centre's neighbours are sorted by (j, n1, n2, n3) ascending;
* rev[p] is the index of the mirrored pair (j, i, -n).

Numpy evaluates each binary operation separately, so the expression above is
exactly what runs.  The search is plain brute force over all j and all image
vectors inside a box that provably contains every pair (see
``image_bounds``); an optional per-axis prefilter in fractional coordinates
only discards j that no image can bring within the cutoff.
"""
from __future__ import annotations

import math

import numpy as np


def pack_shift(n):
    """(n1, n2, n3) int8 each -> one int32 word: byte k holds n_{k+1} (two's complement)."""
    n = np.asarray(n, dtype=np.int64)
    w = (n[..., 0] & 0xFF) | ((n[..., 1] & 0xFF) << 8) | ((n[..., 2] & 0xFF) << 16)
    return w.astype(np.int32)


def unpack_shift(w):
    w = np.asarray(w, dtype=np.int64)
    out = np.stack([(w >> s) & 0xFF for s in (0, 8, 16)], axis=-1)
    return np.where(out >= 128, out - 256, out).astype(np.int64)


def image_bounds(pos, cell, r_cut):
    """n_hat_k such that every pair within r_cut has |n_k| <= n_hat_k.

    |d| >= |s_j,k - s_i,k + n_k| / |b_k| (b_k = rows of H^-T), so
    |n_k| < r_cut |b_k| + (max s_k - min s_k); one more for rounding.
    """
    inv = np.linalg.inv(cell)
    bnorm = np.linalg.norm(inv.T, axis=1)
    s = pos @ inv
    ext = (s.max(axis=0) - s.min(axis=0)) if len(pos) else np.zeros(3)
    return [int(math.ceil(r_cut * bnorm[k] + ext[k])) + 1 for k in range(3)]


def _centre_pairs(i, pos, cell, rc2, imgs, t, cand):
    d = (pos[cand] - pos[i])[None, :, :] + t[:, None, :]          # [n_img, n_cand, 3]
    dd = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    hit = dd < rc2
    same = (cand == i)[None, :] & np.all(imgs == 0, axis=1)[:, None]
    hit &= ~same
    ii, jj = np.nonzero(hit)
    js = cand[jj]
    ns = imgs[ii]
    order = np.lexsort((ns[:, 2], ns[:, 1], ns[:, 0], js))
    return js[order], ns[order]


def neighbor_rows(pos, cell, r_cut, centres, prefilter=True):
    """Sorted neighbour rows for the given centres: list of (j [m], n [m, 3])."""
    pos = np.asarray(pos, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    nh = image_bounds(pos, cell, r_cut)
    grids = [np.arange(-k, k + 1) for k in nh]
    imgs = np.stack(np.meshgrid(*grids, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.int64)
    nf = imgs.astype(np.float64)
    t = (nf[:, 0:1] * cell[0][None, :] + nf[:, 1:2] * cell[1][None, :]) + nf[:, 2:3] * cell[2][None, :]
    rc2 = r_cut * r_cut
    n_atoms = pos.shape[0]
    every = np.arange(n_atoms)
    if prefilter:
        inv = np.linalg.inv(cell)
        bnorm = np.linalg.norm(inv.T, axis=1)
        s = pos @ inv
        reach = r_cut * bnorm + 1e-9
    rows = []
    for i in centres:
        if prefilter:
            ds = s - s[i]
            ds = np.abs(ds - np.round(ds))
            cand = every[np.all(ds < reach[None, :], axis=1)]
        else:
            cand = every
        rows.append(_centre_pairs(int(i), pos, cell, rc2, imgs, t, cand))
    return rows


def neighbor_csr(pos, cell, r_cut, prefilter=True):
    """Full canonical CSR for every atom: off [N+1], j [P], shift [P] (packed), rev [P]."""
    n_atoms = len(pos)
    rows = neighbor_rows(pos, cell, r_cut, range(n_atoms), prefilter=prefilter)
    counts = np.array([len(r[0]) for r in rows], dtype=np.int64)
    off = np.zeros(n_atoms + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    j = np.concatenate([r[0] for r in rows]) if n_atoms else np.zeros(0, np.int64)
    n = np.concatenate([r[1] for r in rows]) if n_atoms else np.zeros((0, 3), np.int64)
    i = np.repeat(np.arange(n_atoms), counts)
    index = {(int(a), int(b), int(c[0]), int(c[1]), int(c[2])): p
             for p, (a, b, c) in enumerate(zip(i, j, n))}
    rev = np.array([index[(int(b), int(a), -int(c[0]), -int(c[1]), -int(c[2]))]
                    for a, b, c in zip(i, j, n)], dtype=np.int64)
    return dict(off=off.astype(np.int32), j=j.astype(np.int32), shift=pack_shift(n),
                rev=rev.astype(np.int32), i=i.astype(np.int32), n=n)


def displacements(pos, cell, i, j, n):
    """d_p = (R[j_p] - R[i_p]) + (n1 H0 + n2 H1) + n3 H2, the same expression as the predicate."""
    pos = np.asarray(pos, dtype=np.float64)
    nf = np.asarray(n, dtype=np.float64)
    t = (nf[:, 0:1] * cell[0][None, :] + nf[:, 1:2] * cell[1][None, :]) + nf[:, 2:3] * cell[2][None, :]
    return (pos[j] - pos[i]) + t
