"""Oracle: active-set update by MaxVol row swaps, plain float64.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library never
does, and it shares no code with it.

The paper (Section 1) bases the MTP's extrapolation grade on D-optimality and
the MaxVol algorithm: the active set is the n x n matrix A whose rows are the
basis vectors of n selected neighbourhoods (or configurations), the grade of a
candidate row c is max_k |(c A^-1)_k|, and a candidate with grade above one
would enlarge |det A| if it replaced an active row.  The update that keeps A
(locally) volume-maximal is the MaxVol iteration of Goreinov et al. (2010,
"How to find a good submatrix"), written out here step by step:

  repeat
    G = C A^-1                       (m x n; a fresh inverse every step)
    (i, k) = argmax |G_ik|           (first in row-major order among equal values)
    stop if |G_ik| <= 1 + tol, or after max_swaps swaps
    swap active row k with candidate row i
  until stop

Each swap multiplies |det A| by |G_ik| (the determinant of a matrix whose row
k is replaced changes by the factor (c_i A^-1)_k), which the tests pin.
"""
from __future__ import annotations

import numpy as np


def maxvol_update(active, cand, tol=1e-3, max_swaps=None):
    """MaxVol swaps between the active set and the candidates.

    active: (n, n) float64 array, invertible; cand: (m, n) float64 array.
    Returns (active', cand', swaps) where swaps lists (i, k, G_ik) in order.
    The inputs are not modified.
    """
    A = np.array(active, dtype=np.float64, copy=True)
    C = np.array(cand, dtype=np.float64, copy=True)
    swaps = []
    while max_swaps is None or len(swaps) < max_swaps:
        G = C @ np.linalg.inv(A)
        flat = int(np.argmax(np.abs(G)))  # numpy returns the first maximum in row-major order
        i, k = divmod(flat, G.shape[1])
        g = float(G[i, k])
        if abs(g) <= 1.0 + tol:
            break
        row = A[k].copy()
        A[k] = C[i]
        C[i] = row
        swaps.append((i, k, g))
    return A, C, swaps
