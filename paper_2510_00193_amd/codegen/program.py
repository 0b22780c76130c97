"""Straight-line evaluation program of one MTP level.

Built from the component-first basis:

* moments: flat component layout (mu, a, b, c) of every used M_{mu,nu};
* one block per connected contraction q: a list of weighted products
  dst += w * x * y, where x is a moment component or a temporary of the
  block, y is a moment component, dst a temporary or the block output C_q;
* products: every basis function is a product of connected outputs; they
  form a trie keyed by the sorted component tuple, evaluated depth first so
  that only the current path is live.

The same program read backwards gives the adjoint: dx += w * d(dst) * y and
dy += w * d(dst) * x.
"""
from __future__ import annotations

import itertools
from collections import defaultdict
from dataclasses import dataclass, field
from fractions import Fraction
from math import factorial

from .basis import Basis, Graph, build_basis
from .contract import MomentLayout, _compositions3, best_order


def _mult(c):
    return factorial(sum(c)) // (factorial(c[0]) * factorial(c[1]) * factorial(c[2]))


def _add(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


@dataclass
class Block:
    """Program of one connected contraction."""

    q: int
    n_temp: int
    ops: list                    # (dst, x, y, weight); dst/x: ("t", k) | ("m", e) | ("c", q)
    entries: list                # sorted moment components read by the block


@dataclass
class Program:
    level: int
    basis: Basis
    layout: MomentLayout
    blocks: list
    trie: list = field(default_factory=list)   # per basis entry: (parent entry or -1, component)

    @property
    def n_alpha(self):
        return self.basis.n_alpha

    @property
    def n_comp(self):
        return len(self.blocks)

    @property
    def n_mom(self):
        return len(self.layout)

    @property
    def n_mu(self):
        return self.basis.n_mu

    @property
    def max_nu(self):
        return max(nu for _, nu in self.basis.moments)

    def triple_count(self):
        return sum(len(b.ops) for b in self.blocks)


def _compile_component(q: int, g: Graph, layout: MomentLayout) -> Block:
    k = len(g.labels)
    if k == 1:
        mu, nu = g.labels[0]
        e = layout.index[(mu, 0, 0, 0)]
        # a scalar moment: C_q = m_e (one op with a unit partner is avoided by a copy marker)
        return Block(q, 0, [(("c", q), ("m", e), None, Fraction(1))], [e])
    m = g.matrix()
    order = best_order(g)
    v0 = order[0]
    S = {v0}
    # current intermediate: groups (targets) with sizes, and a value map comp-tuple -> source
    targets = [t for t in range(k) if t != v0 and m[v0][t]]
    sizes = [m[v0][t] for t in targets]
    mu0 = g.labels[v0][0]

    def src_first(comp):
        tot = (0, 0, 0)
        for c in comp:
            tot = _add(tot, c)
        return ("m", layout.index[(mu0,) + tot])

    comps = list(itertools.product(*[_compositions3(n) for n in sizes]))
    source = {c: src_first(c) for c in comps}
    ops = []
    n_temp = 0
    for step, l in enumerate(order[1:]):
        last = step == k - 2
        mul = g.labels[l][0]
        # group of the current intermediate that points at l
        if l in targets:
            gi = targets.index(l)
            n_l = sizes[gi]
        else:
            gi, n_l = None, 0
        rest_t = [t for t in range(k) if t not in S and t != l and m[l][t]]
        new_targets = [t for t in targets if t != l]
        for t in rest_t:
            if t not in new_targets:
                new_targets.append(t)
        new_sizes = []
        for t in new_targets:
            a = sizes[targets.index(t)] if t in targets else 0
            new_sizes.append(a + m[l][t])
        acc = defaultdict(Fraction)
        rest_choices = [_compositions3(m[l][t]) for t in rest_t]
        for comp, src in source.items():
            p = comp[gi] if gi is not None else (0, 0, 0)
            w_p = _mult(p)
            for rpick in itertools.product(*rest_choices):
                rsum = p
                for r in rpick:
                    rsum = _add(rsum, r)
                y = ("m", layout.index[(mul,) + rsum])
                w = Fraction(w_p)
                out = []
                for t, nsz in zip(new_targets, new_sizes):
                    a = comp[targets.index(t)] if t in targets else (0, 0, 0)
                    r = rpick[rest_t.index(t)] if t in rest_t else (0, 0, 0)
                    c = _add(a, r)
                    w *= Fraction(_mult(a) * _mult(r), _mult(c))
                    out.append(c)
                acc[(tuple(out), src, y)] += w
        if last:
            assert not new_targets
            for (out, src, y), w in acc.items():
                if w:
                    ops.append((("c", q), src, y, w))
        else:
            out_comps = list(itertools.product(*[_compositions3(n) for n in new_sizes]))
            new_source = {}
            for oc in out_comps:
                new_source[oc] = ("t", n_temp)
                n_temp += 1
            for (out, src, y), w in acc.items():
                if w:
                    ops.append((new_source[out], src, y, w))
            source = new_source
        S.add(l)
        targets, sizes = new_targets, new_sizes
    ents = sorted({o[1][1] for o in ops if o[1][0] == "m"} | {o[2][1] for o in ops if o[2] is not None})
    return Block(q, n_temp, ops, ents)


def build_program(level: int) -> Program:
    basis = build_basis(level)
    layout = MomentLayout(basis.moments)
    blocks = [_compile_component(q, g, layout) for q, g in enumerate(basis.components)]
    trie = [(e.factor, e.factor_part if len(e.parts) > 1 else e.parts[0]) for e in basis.entries]
    return Program(level, basis, layout, blocks, trie)
