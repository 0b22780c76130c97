"""Compressed-symmetric contraction of moment tensors.

A symmetric tensor of rank nu in 3-D is stored by its (nu+1)(nu+2)/2
distinct components m[(a, b, c)], a + b + c = nu, each equal to
sum_j f_mu(r_ij) x^a y^b z^c.  Contracting m_e index pairs between tensors
k and l means summing over the x/y/z values of those pairs; only the counts
(p, q, r) of x, y, z on the edge matter, with multiplicity m!/(p! q! r!).
A connected contraction therefore equals

  sum over counts (p_e, q_e, r_e) per edge of
      prod_e  m_e! / (p_e! q_e! r_e!)
    * prod_k  m_k[ sum_{e at k} (p_e, q_e, r_e) ]

which is a polynomial in the stored components; this module expands it and
merges equal monomials.
"""
from __future__ import annotations

import itertools
from collections import defaultdict
from math import factorial

from .basis import Graph


def components_of(nu: int):
    """(a, b, c) with a + b + c = nu, in the storage order: a descending, then b descending."""
    return [(a, b, nu - a - b) for a in range(nu, -1, -1) for b in range(nu - a, -1, -1)]


class MomentLayout:
    """Flat index of every stored component (mu, a, b, c) of the used moments."""

    def __init__(self, moments):
        self.moments = list(moments)
        self.index = {}
        self.items = []
        for mu, nu in self.moments:
            for abc in components_of(nu):
                self.index[(mu,) + abc] = len(self.items)
                self.items.append((mu,) + abc)

    def __len__(self):
        return len(self.items)


def _compositions3(m):
    return [(p, q, m - p - q) for p in range(m, -1, -1) for q in range(m - p, -1, -1)]


def _multinomial(m, pqr):
    p, q, r = pqr
    return factorial(m) // (factorial(p) * factorial(q) * factorial(r))


def expand(graph: Graph, layout: MomentLayout):
    """Polynomial of a connected contraction: dict {sorted tuple of flat indices: integer weight}."""
    k = len(graph.labels)
    edges = list(graph.mult)
    poly = defaultdict(int)
    if not edges:
        mu, nu = graph.labels[0]
        assert k == 1 and nu == 0
        poly[(layout.index[(mu, 0, 0, 0)],)] += 1
        return dict(poly)
    choices = [_compositions3(v) for _, v in edges]
    for pick in itertools.product(*choices):
        w = 1
        cnt = [[0, 0, 0] for _ in range(k)]
        for ((a, b), v), pqr in zip(edges, pick):
            w *= _multinomial(v, pqr)
            for t in (a, b):
                cnt[t][0] += pqr[0]
                cnt[t][1] += pqr[1]
                cnt[t][2] += pqr[2]
        key = tuple(sorted(layout.index[(graph.labels[t][0],) + tuple(cnt[t])] for t in range(k)))
        poly[key] += w
    return dict(poly)


# --------------------------------------------------------------------------------------
# pairwise contraction through group-symmetrised intermediates
#
# After tensors S of a connected graph are contracted, the intermediate T_S has
# one index group per outside tensor t (the edges from S to t).  Because every
# later partner is a symmetric tensor, T_S may be replaced by its average over
# permutations inside each group, so it is stored by one count triple per group.
# Contracting T_S with tensor l:
#   U[{c_t}] = sum_p mult(p) sum_{a_t + r_t = c_t} prod_t mult(a_t) mult(r_t) / mult(c_t)
#              * T_S[p, {a_t}] * m_l[p + sum_t r_t]
# with p the counts on the group S->l and r_t the counts on l's own edges to t.


def _mult(c):
    return factorial(sum(c)) // (factorial(c[0]) * factorial(c[1]) * factorial(c[2]))


def _add(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def _group_comps(sizes):
    """All tuples of count triples for groups of the given sizes."""
    return list(itertools.product(*[_compositions3(n) for n in sizes]))


def contraction_steps(graph: Graph, order):
    """Simulate contracting graph tensors in `order`; return (total triple count, steps)."""
    k = len(graph.labels)
    m = graph.matrix()
    S = {order[0]}
    groups = {t: m[order[0]][t] for t in range(k) if t != order[0] and m[order[0]][t]}
    steps = []
    total = 0
    for l in order[1:]:
        n_l = groups.get(l, 0)
        rest = {t: m[l][t] for t in range(k) if t not in S and t != l and m[l][t]}
        new = {}
        for t in set(groups) | set(rest):
            if t == l:
                continue
            new[t] = groups.get(t, 0) + rest.get(t, 0)
        size_in = 1
        for t, n in groups.items():
            size_in *= (n + 1) * (n + 2) // 2
        size_rest = 1
        for t, n in rest.items():
            size_rest *= (n + 1) * (n + 2) // 2
        total += size_in * size_rest
        steps.append((l, dict(groups), dict(rest), dict(new)))
        S.add(l)
        groups = new
    return total, steps


def best_order(graph: Graph):
    k = len(graph.labels)
    best = None
    for perm in itertools.permutations(range(k)):
        # only orders where each new tensor touches the contracted set
        m = graph.matrix()
        ok = all(any(m[perm[i]][perm[j]] for j in range(i)) for i in range(1, k))
        if not ok:
            continue
        cost, _ = contraction_steps(graph, perm)
        if best is None or cost < best[0]:
            best = (cost, perm)
    return best[1]
