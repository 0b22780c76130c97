"""Basis of the Moment Tensor Potential, built component-first for code generation.

The MTP (cited in Section 1 of the paper as the model the package implements)
writes each basis function as a full contraction of moment tensors
M_{mu,nu} = sum_j f_mu(r_ij) d_ij^(x nu); the level of M_{mu,nu} is
2 + 4 mu + nu and a function's level is the sum over its tensors.  The set of
level L holds every contraction multigraph (no self-contractions) of level
<= L, disconnected products included, one per isomorphism class.

This enumerator builds the connected contractions first and forms products
as multisets of them, which is also how the generated code evaluates them:
one polynomial per connected contraction, then one multiplication per
product.  The public order of the functions (the order of the linear
coefficients) is: total level, then the labels sorted by (mu, nu), then the
smallest row-major upper-triangle tuple of the contraction matrix over all
relabelings that keep labels in place.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field


def level_of(mu: int, nu: int) -> int:
    return 2 + 4 * mu + nu


@dataclass(frozen=True)
class Graph:
    """A contraction multigraph over labelled moments.

    labels: tuple of (mu, nu), sorted ascending.
    mult:   dict-like tuple of ((a, b), m) with a < b and m > 0 (edge multiplicities).
    """

    labels: tuple
    mult: tuple

    @property
    def level(self) -> int:
        return sum(level_of(*l) for l in self.labels)

    def matrix(self):
        k = len(self.labels)
        m = [[0] * k for _ in range(k)]
        for (a, b), v in self.mult:
            m[a][b] = m[b][a] = v
        return m


def _relabelings(labels):
    """Yield index maps new->old that keep every label in place."""
    runs = []
    start = 0
    for pos in range(1, len(labels) + 1):
        if pos == len(labels) or labels[pos] != labels[start]:
            runs.append(range(start, pos))
            start = pos
    # only runs whose tensors carry edges can produce different matrices
    for combo in itertools.product(*[itertools.permutations(r) if labels[r[0]][1] > 0 else [tuple(r)]
                                     for r in runs]):
        yield [i for part in combo for i in part]


def canonical_key(labels, matrix):
    k = len(labels)
    best = None
    for perm in _relabelings(labels):
        key = tuple(matrix[perm[a]][perm[b]] for a in range(k) for b in range(a + 1, k))
        if best is None or key < best:
            best = key
    return best


def _connected(matrix) -> bool:
    k = len(matrix)
    reach = {0}
    frontier = [0]
    while frontier:
        a = frontier.pop()
        for b in range(k):
            if matrix[a][b] and b not in reach:
                reach.add(b)
                frontier.append(b)
    return len(reach) == k


def _edge_fillings(nus):
    """Matrices with zero diagonal and row sums nus, by filling upper-triangle cells."""
    k = len(nus)
    cells = [(a, b) for a in range(k) for b in range(a + 1, k)]
    ranges = [range(min(nus[a], nus[b]) + 1) for a, b in cells]
    for vals in itertools.product(*ranges):
        deg = [0] * k
        for (a, b), v in zip(cells, vals):
            deg[a] += v
            deg[b] += v
        if deg == list(nus):
            m = [[0] * k for _ in range(k)]
            for (a, b), v in zip(cells, vals):
                m[a][b] = m[b][a] = v
            yield m


def connected_graphs(level: int):
    """All connected contraction graphs of level <= `level`, one per class."""
    lab_pool = sorted((mu, nu) for mu in range(level) for nu in range(level) if level_of(mu, nu) <= level)
    out = {}
    # single scalar moments
    for mu, nu in lab_pool:
        if nu == 0:
            g = Graph(((mu, 0),), ())
            out[(g.labels, ())] = g
    # two or more tensors, each with nu >= 1
    tensor_labels = [l for l in lab_pool if l[1] >= 1]
    for k in range(2, level // 3 + 1):
        for labels in itertools.combinations_with_replacement(tensor_labels, k):
            if sum(level_of(*l) for l in labels) > level:
                continue
            nus = [nu for _, nu in labels]
            if sum(nus) % 2:
                continue
            for m in _edge_fillings(nus):
                if not _connected(m):
                    continue
                key = canonical_key(labels, m)
                if (labels, key) in out:
                    continue
                cells = [(a, b) for a in range(k) for b in range(a + 1, k)]
                mult = tuple(((a, b), v) for (a, b), v in zip(cells, key) if v)
                out[(labels, key)] = Graph(labels, mult)
    return sorted(out.values(), key=lambda g: (g.level, g.labels, canonical_key(g.labels, g.matrix())))


@dataclass
class BasisEntry:
    """One basis function: a multiset of connected components (indices into the component list)."""

    parts: tuple                 # sorted tuple of component indices
    labels: tuple                # merged labels
    key: tuple                   # canonical upper-triangle tuple
    level: int
    factor: int = -1             # index of the entry this one equals times one component
    factor_part: int = -1        # that component


@dataclass
class Basis:
    level: int
    components: list             # list[Graph], connected
    entries: list                # list[BasisEntry], public order
    moments: list = field(default_factory=list)   # sorted (mu, nu) used

    @property
    def n_alpha(self):
        return len(self.entries)

    @property
    def n_mu(self):
        return max(mu for mu, _ in self.moments) + 1


def _union(components, parts):
    """Labels and matrix of the disjoint union, tensors re-sorted by label."""
    items = []   # (label, part_no, local_index)
    for pn, ci in enumerate(parts):
        for li, lab in enumerate(components[ci].labels):
            items.append((lab, pn, li))
    order = sorted(range(len(items)), key=lambda t: items[t][0])
    where = {(items[t][1], items[t][2]): new for new, t in enumerate(order)}
    k = len(items)
    m = [[0] * k for _ in range(k)]
    for pn, ci in enumerate(parts):
        for (a, b), v in components[ci].mult:
            x, y = where[(pn, a)], where[(pn, b)]
            m[x][y] = m[y][x] = v
    labels = tuple(items[t][0] for t in order)
    return labels, m


def build_basis(level: int) -> Basis:
    comps = connected_graphs(level)
    lv = [c.level for c in comps]
    entries = []

    def rec(start, budget, acc):
        if acc:
            labels, m = _union(comps, acc)
            entries.append(BasisEntry(tuple(acc), labels, canonical_key(labels, m),
                                      sum(lv[c] for c in acc)))
        for c in range(start, len(comps)):
            if lv[c] <= budget:
                acc.append(c)
                rec(c, budget - lv[c], acc)
                acc.pop()

    rec(0, level, [])
    entries.sort(key=lambda e: (e.level, e.labels, e.key))
    index = {e.parts: n for n, e in enumerate(entries)}
    for e in entries:
        if len(e.parts) > 1:
            # peel off the last component; the remainder is itself a basis function
            e.factor_part = e.parts[-1]
            e.factor = index[e.parts[:-1]]
    moments = sorted({lab for c in comps for lab in c.labels})
    return Basis(level, comps, entries, moments)
