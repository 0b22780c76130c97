"""Oracle: enumeration of MTP basis functions (test infrastructure only).

The paper does not print the basis; it defines the Moment Tensor Potential by
reference to its original formulation (Section 1, "Motivation and
significance", citing the MTP paper and MLIP-3).  The reading taken here:

* A moment M_{mu,nu} has level 2 + 4 mu + nu.
* A basis function is a multiset of moments together with a contraction
  multigraph: a symmetric non-negative integer matrix with zero diagonal
  whose k-th row sums to nu_k (every tensor index is contracted with an
  index of another tensor; no self-contractions).  Its level is the sum of
  the moment levels; all functions of level <= L form the basis of level L.
  Disconnected graphs (products of scalars) are included.
* Functions are counted once per isomorphism class (permutations of
  tensors that carry the same label).
* Canonical order: by (total level, labels sorted ascending by (mu, nu),
  canonical key), the canonical key being the smallest row-major
  upper-triangle tuple of the matrix over all label-preserving
  permutations.

This is a brute-force enumeration: every label multiset, every admissible
matrix, canonical key by trying all permutations.  It shares no code with
the GPU library's own enumerator.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass


def moment_level(mu: int, nu: int) -> int:
    return 2 + 4 * mu + nu


@dataclass(frozen=True)
class BasisFunction:
    labels: tuple          # ((mu, nu), ...) sorted ascending
    edges: tuple           # upper-triangle tuple (row-major) of the canonical matrix
    level: int

    def matrix(self):
        k = len(self.labels)
        m = [[0] * k for _ in range(k)]
        it = iter(self.edges)
        for a in range(k):
            for b in range(a + 1, k):
                m[a][b] = m[b][a] = next(it)
        return m

    def connected(self) -> bool:
        k = len(self.labels)
        if k == 1:
            return True
        m = self.matrix()
        seen = {0}
        stack = [0]
        while stack:
            a = stack.pop()
            for b in range(k):
                if m[a][b] and b not in seen:
                    seen.add(b)
                    stack.append(b)
        return len(seen) == k


def _labels_upto(level):
    out = []
    for mu in range(level):
        for nu in range(level):
            if moment_level(mu, nu) <= level:
                out.append((mu, nu))
    return sorted(out)


def _label_multisets(level):
    labels = _labels_upto(level)

    def rec(start, budget, acc):
        if acc:
            yield tuple(acc)
        for idx in range(start, len(labels)):
            lab = labels[idx]
            lv = moment_level(*lab)
            if lv <= budget:
                acc.append(lab)
                yield from rec(idx, budget - lv, acc)
                acc.pop()

    yield from rec(0, level, [])


def _matrices(nus):
    """All symmetric non-negative integer matrices, zero diagonal, row sums nus."""
    k = len(nus)
    pairs = [(a, b) for a in range(k) for b in range(a + 1, k)]
    rem = list(nus)
    vals = [0] * len(pairs)

    def rec(pi):
        if pi == len(pairs):
            if all(r == 0 for r in rem):
                yield tuple(vals)
            return
        a, b = pairs[pi]
        # row a has no pair after the last (a, k-1): force it to finish there
        hi = min(rem[a], rem[b])
        lo = rem[a] if b == k - 1 else 0
        for v in range(lo, hi + 1):
            vals[pi] = v
            rem[a] -= v
            rem[b] -= v
            yield from rec(pi + 1)
            rem[a] += v
            rem[b] += v
        vals[pi] = 0

    if k == 1:
        if nus[0] == 0:
            yield ()
        return
    yield from rec(0)


def _upper(m, perm):
    k = len(perm)
    return tuple(m[perm[a]][perm[b]] for a in range(k) for b in range(a + 1, k))


def _canonical(labels, edges):
    k = len(labels)
    m = [[0] * k for _ in range(k)]
    it = iter(edges)
    for a in range(k):
        for b in range(a + 1, k):
            m[a][b] = m[b][a] = next(it)
    # label-preserving permutations: permute inside each run of equal labels
    groups = []
    a = 0
    while a < k:
        b = a
        while b < k and labels[b] == labels[a]:
            b += 1
        groups.append(list(range(a, b)))
        a = b
    best = None
    for choice in itertools.product(*[itertools.permutations(g) for g in groups]):
        perm = [x for g in choice for x in g]
        key = _upper(m, perm)
        if best is None or key < best:
            best = key
    return best


def enumerate_basis(level: int, connected_only: bool = False):
    """All basis functions of level <= `level`, in canonical order."""
    found = set()
    for labels in _label_multisets(level):
        nus = [nu for _, nu in labels]
        if sum(nus) % 2:
            continue
        for edges in _matrices(nus):
            key = _canonical(labels, edges)
            found.add((labels, key))
    out = []
    for labels, key in found:
        bf = BasisFunction(labels, key, sum(moment_level(*l) for l in labels))
        if connected_only and not bf.connected():
            continue
        out.append(bf)
    out.sort(key=lambda b: (b.level, b.labels, b.edges))
    return out


def radial_count(level: int, basis=None) -> int:
    """Number of radial functions: one per mu used by some basis function."""
    basis = basis if basis is not None else enumerate_basis(level)
    mus = {mu for b in basis for mu, _ in b.labels}
    return max(mus) + 1 if mus else 0


def used_moments(basis):
    """Sorted list of (mu, nu) appearing in the basis."""
    return sorted({lab for b in basis for lab in b.labels})
