"""Write basis_counts.txt: basis sizes per level under the contraction rule, counted by
Burnside's lemma (orbit counting), independently of the oracle's enumerator.

Rule (the MTP definition the paper cites in Section 1): a moment M_{mu,nu} has level
2 + 4 mu + nu; a basis function is a multiset of moments with a contraction multigraph (a
symmetric non-negative integer matrix, zero diagonal, row k summing to nu_k) of total level
<= L, one per isomorphism class under permutations of equally labelled tensors; disconnected
products are included.

The oracle builds one canonical representative per class.  This script never forms a
canonical key: for each label multiset it enumerates the admissible matrices X and counts
classes as (1/|G|) sum_X |Stab_G(X)|, G the label-preserving permutation group.  Tensors with
nu = 0 carry no edges, so their permutations fix every X and cancel from that ratio; G is
taken over the nu > 0 tensors only.  Output columns: level, n_alpha, n_connected, n_moments
(distinct (mu, nu) used), C (sum of (nu+1)(nu+2)/2 over them), n_mu, max_nu.

Usage: python tests/golden/count_basis.py > tests/golden/basis_counts.txt
"""
from __future__ import annotations

import itertools
import math
import sys
from fractions import Fraction


def level_of(mu, nu):
    return 2 + 4 * mu + nu


def label_multisets(level):
    """Multisets of (mu, nu) labels with total level <= level (as sorted tuples)."""
    labels = [(mu, nu) for mu in range(level) for nu in range(level) if level_of(mu, nu) <= level]
    labels.sort()
    out = []
    stack = [((), 0, 0)]
    while stack:
        acc, start, used = stack.pop()
        if acc:
            out.append(acc)
        for k in range(start, len(labels)):
            lv = level_of(*labels[k])
            if used + lv <= level:
                stack.append((acc + (labels[k],), k, used + lv))
    return out


def edge_matrices(nus):
    """Every symmetric zero-diagonal non-negative integer matrix with row sums nus, as a dict
    {(a, b): m} over a < b; built row by row, distributing each row's remaining degree over the
    later tensors."""
    k = len(nus)
    results = []

    def fill(row, rem, edges):
        if row == k:
            if all(r == 0 for r in rem):
                results.append(dict(edges))
            return
        later = list(range(row + 1, k))
        need = rem[row]
        # compositions of `need` into len(later) parts bounded by the partners' remaining degrees
        for parts in _bounded_compositions(need, [rem[b] for b in later]):
            new_rem = list(rem)
            new_rem[row] = 0
            new_edges = dict(edges)
            for b, m in zip(later, parts):
                if m:
                    new_rem[b] -= m
                    new_edges[(row, b)] = m
            fill(row + 1, new_rem, new_edges)

    fill(0, list(nus), {})
    return results


def _bounded_compositions(total, bounds):
    if not bounds:
        if total == 0:
            yield ()
        return
    head, rest = bounds[0], bounds[1:]
    for v in range(min(total, head), -1, -1):
        if total - v <= sum(rest):
            for tail in _bounded_compositions(total - v, rest):
                yield (v,) + tail


def is_connected(k, edges):
    if k == 1:
        return True
    adj = {a: set() for a in range(k)}
    for (a, b) in edges:
        adj[a].add(b)
        adj[b].add(a)
    seen, todo = {0}, [0]
    while todo:
        a = todo.pop()
        for b in adj[a] - seen:
            seen.add(b)
            todo.append(b)
    return len(seen) == k


def permutation_group(labels):
    """Label-preserving permutations of the tensors with nu > 0 (as full index maps)."""
    k = len(labels)
    runs = {}
    for a, lab in enumerate(labels):
        if lab[1] > 0:
            runs.setdefault(lab, []).append(a)
    blocks = list(runs.values())
    perms = []
    for choice in itertools.product(*[itertools.permutations(b) for b in blocks]):
        g = list(range(k))
        for block, image in zip(blocks, choice):
            for src, dst in zip(block, image):
                g[src] = dst
        perms.append(g)
    return perms


def fixes(g, edges):
    for (a, b), m in edges.items():
        x, y = g[a], g[b]
        if edges.get((min(x, y), max(x, y)), 0) != m:
            return False
    return True


def counts(level):
    total = Fraction(0)
    connected = Fraction(0)
    used = set()
    for labels in label_multisets(level):
        nus = [nu for _, nu in labels]
        if sum(nus) % 2:
            continue
        mats = edge_matrices(nus)
        if not mats:
            continue
        group = permutation_group(labels)
        for edges in mats:
            stab = sum(1 for g in group if fixes(g, edges))
            w = Fraction(stab, len(group))
            total += w
            if is_connected(len(labels), edges):
                connected += w
        used.update(labels)
    assert total.denominator == 1 and connected.denominator == 1
    n_mu = max(mu for mu, _ in used) + 1
    comps = sum((nu + 1) * (nu + 2) // 2 for _, nu in used)
    return int(total), int(connected), len(used), comps, n_mu, max(nu for _, nu in used)


def main(argv):
    levels = [int(x) for x in argv[1:]] or list(range(2, 21, 2))
    print("# Basis sizes per level under the contraction rule (all scalar contractions,")
    print("# connected subset, distinct moments, compressed components, radial functions,")
    print("# max nu), written by tests/golden/count_basis.py (orbit counting by Burnside's")
    print("# lemma, independent of the oracle's canonical-form enumeration).  Levels 2-10")
    print("# also agree with the hand count in basis_L10_hand.txt.  Rule: the MTP definition")
    print("# cited in Section 1 of the paper.")
    print("# level n_alpha n_connected n_moments C n_mu max_nu")
    for lv in levels:
        print(lv, *counts(lv), flush=True)


if __name__ == "__main__":
    main(sys.argv)
