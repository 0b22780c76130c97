"""Emit the per-level device code of the MTP evaluation as a HIP header.

For one level the header defines a traits struct ``Lv<L>`` with static
device functions, all straight-line code with compile-time indices so that
per-atom state stays in registers:

  acc_moments<G>(m, f, x, y, z)        m[e] += f[mu_e] x^a y^b z^c   (entry group G)
  pair_grad<G>(mb, f, fp, x, y, z, ...) gradient of sum_e mb[e] f_mu x^a y^b z^c w.r.t. d
  fwd(M, C)                             connected contractions C_q from moments
  products(C, xi, Cb, B)                basis values, site energy, adjoints of C_q
  rev<G>(M, Cb, mb)                     mb[e] += sum_q Cb_q dC_q/dm_e   (entries of group G)
  tan(M, Md, C, Cd)                     forward-mode tangent of the contractions
  ...

The host-side tables (moment layout, product trie, basis order) are
emitted too, for argument checking and tests.
"""
from __future__ import annotations

import math
import os
from collections import defaultdict
from fractions import Fraction

from .program import Program, build_program


def _lit(w) -> str:
    v = float(w)
    if v == int(v) and abs(v) < 1e15:
        return f"R({int(v)})"
    return f"R({v!r})"


class _W:
    def __init__(self):
        self.lines = []
        self.ind = 0

    def __call__(self, s=""):
        self.lines.append("  " * self.ind + s)

    def push(self):
        self.ind += 1

    def pop(self):
        self.ind -= 1

    def text(self):
        return "\n".join(self.lines) + "\n"


def entry_groups(prog: Program, n_groups):
    """Split the flat moment layout into contiguous ranges: n_groups ranges of similar size,
    or, given a tuple, the interior boundaries themselves (e.g. (84,) at level 16 separates the
    mu = 0 components from the rest)."""
    n = prog.n_mom
    if isinstance(n_groups, (tuple, list)):
        bounds = [0] + [int(b) for b in n_groups] + [n]
        assert all(bounds[k] < bounds[k + 1] for k in range(len(bounds) - 1))
    else:
        bounds = [round(k * n / n_groups) for k in range(n_groups + 1)]
    return [(bounds[k], bounds[k + 1]) for k in range(len(bounds) - 1)]


# Most moment entries one adjoint pair group holds: the pair kernel of the parameter adjoint
# keeps the adjoint and its tangent of every entry of its group in registers, next to the
# per-lane radial-gradient sums of the group's mu values (64: no spills at levels 16 and 20,
# one pass fewer than 48 at level 20; 100 spills).
ADJ_GROUP_CAP = 64


def adj_entry_groups(prog: Program, cap=ADJ_GROUP_CAP):
    """Split the flat moment layout (mu-major) into contiguous ranges of at most cap entries
    for the adjoint pair kernel: a mu segment longer than cap is cut into equal parts, and
    consecutive short segments share a range while they fit."""
    mus = [it[0] for it in prog.layout.items]
    assert mus == sorted(mus), "the moment layout is mu-major"
    segs = []
    for e, mu in enumerate(mus):
        if segs and segs[-1][2] == mu:
            segs[-1][1] = e + 1
        else:
            segs.append([e, e + 1, mu])
    out, open_range = [], False  # open_range: the last range holds whole short segments
    for lo, hi, _ in segs:
        n = hi - lo
        if n > cap:
            k = -(-n // cap)
            cuts = [lo + round(q * n / k) for q in range(k + 1)]
            out += [(cuts[q], cuts[q + 1]) for q in range(k)]
            open_range = False
        elif open_range and out[-1][1] - out[-1][0] + n <= cap:
            out[-1] = (out[-1][0], hi)
        else:
            out.append((lo, hi))
            open_range = True
    return out


def _ref(r, mvar="me"):
    kind, k = r
    if kind == "m":
        return f"{mvar}{k}"
    if kind == "t":
        return f"t{k}"
    return f"C[{k}]"


def _emit_pair_functions(w: _W, prog: Program, groups):
    """Moment accumulation and pair gradient, emitted degree by degree: the monomials of
    degree nu are formed from those of degree nu - 1 and consumed right away, so only two
    degrees of monomials are live at once."""
    items = prog.layout.items
    for gi, (lo, hi) in enumerate(groups):
        ents = list(range(lo, hi))
        by_mono = defaultdict(list)
        for e in ents:
            mu, a, b, c = items[e]
            by_mono[(a, b, c)].append((e, mu))
        gnu = max(a + b + c for (a, b, c) in by_mono)
        # ---------------- moment accumulation
        w(f"// entries [{lo}, {hi}) of the moment layout")
        w("template <class R>")
        w(f"static __device__ __forceinline__ void acc_moments_g{gi}(R* __restrict__ m, const R* __restrict__ f, R x, R y, R z) {{")
        w.push()
        # degree by degree: the monomials of one degree are independent products, formed
        # together (measured faster here than forming each right before its accumulations)
        need = _monomial_closure(by_mono.keys())
        for nu in range(gnu + 1):
            for abc in _degree(need, nu):
                _emit_one_monomial(w, abc)
            for abc in _degree(by_mono.keys(), nu):
                for e, mu in by_mono[abc]:
                    w(f"m[{e - lo}] = fma(f[{mu}], {_mono_name(abc)}, m[{e - lo}]);")
        w.pop()
        w("}")
        # ---------------- gradient of sum_e mb_e f_mu_e mono_e, and u = sum_mu fp_mu S_mu
        # In scaled monomials q_abc = x^a y^b z^c / (a! b! c!) the gradient of q_abc is
        # (q_(a-1)bc, q_a(b-1)c, q_ab(c-1)) without factors, so the caller passes the adjoints
        # multiplied by a! b! c! (MFACT): mb_e mono_e = (mb_e a!b!c!) q_e.
        w("template <class R>")
        w(f"static __device__ __forceinline__ void pair_grad_g{gi}(const R* __restrict__ mb, const R* __restrict__ f,")
        w("    const R* __restrict__ fp, R x, R y, R z, R& gx, R& gy, R& gz, R& u) {")
        w.push()
        mus = sorted({items[e][0] for e in ents})
        for mu in mus:
            w(f"R s{mu} = R(0);")
        # gradient sums of the monomials with a single radial function, per radial function
        # and degree
        single = set()
        for mu in mus:
            for n in range(1, gnu + 1):
                w(f"R hx{mu}_{n} = R(0), hy{mu}_{n} = R(0), hz{mu}_{n} = R(0);")
        top = max(max(k) for k in by_mono)
        for var in "xyz":
            for k in range(2, top + 1):
                w(f"const R {var}_{k} = {var} * {_lit(Fraction(1, k))};")
        made = set()

        def make(abc):
            # a scaled monomial is formed right before its first use (its chain parent first),
            # so that few monomials of the current degree are live at once
            if abc in made:
                return
            a, b, c = abc
            name = _mono_name(abc)
            if a + b + c == 0:
                w(f"const R {name} = R(1);")
            else:
                parent, var, k = ((a, b, c - 1), "z", c) if c else ((a, b - 1, 0), "y", b) if b else ((a - 1, 0, 0), "x", a)
                make(parent)
                fac = var if k == 1 else f"{var}_{k}"
                w(f"const R {name} = {_mono_name(parent)} * {fac};")
            made.add(abc)

        for nu in range(gnu + 1):
            for abc in _degree(by_mono.keys(), nu):
                make(abc)
                for low in ((abc[0] - 1, abc[1], abc[2]), (abc[0], abc[1] - 1, abc[2]), (abc[0], abc[1], abc[2] - 1)):
                    if min(low) >= 0:
                        make(low)
                lst = by_mono[abc]
                a, b, c = abc
                if len(lst) == 1 and a + b + c > 0:
                    # one radial function: accumulate mb_e grad q_e per degree nu, without the
                    # radial factor (applied once per pair); the value sum of these terms follows
                    # from Euler's relation d . grad P = nu P for a homogeneous P of degree nu
                    e, mu = lst[0]
                    single.add((mu, nu))
                    for d, k, low in (("x", a, (a - 1, b, c)), ("y", b, (a, b - 1, c)), ("z", c, (a, b, c - 1))):
                        if k:
                            w(f"h{d}{mu}_{nu} = fma(mb[{e - lo}], {_mono_name(low)}, h{d}{mu}_{nu});")
                    continue
                for e, mu in lst:
                    w(f"s{mu} = fma(mb[{e - lo}], {_mono_name(abc)}, s{mu});")
                if a + b + c == 0:
                    continue
                dirs = [(d, low) for d, k, low in (("x", a, (a - 1, b, c)), ("y", b, (a, b - 1, c)),
                                                   ("z", c, (a, b, c - 1))) if k]
                first = True
                for e, mu in lst:
                    if first:
                        w(f"{{ R t = f[{mu}] * mb[{e - lo}];")
                        first = False
                    else:
                        w(f"  t = fma(f[{mu}], mb[{e - lo}], t);")
                for d, low in dirs:
                    w(f"  g{d} = fma(t, {_mono_name(low)}, g{d});")
                w("}")
        for mu in sorted({m for m, _ in single}):
            nus = sorted(n for m, n in single if m == mu)
            for d in "xyz":
                terms = " + ".join(f"h{d}{mu}_{n}" for n in nus)
                w(f"g{d} = fma(f[{mu}], {terms}, g{d});")
            for n in nus:
                w(f"s{mu} = fma(fma(z, hz{mu}_{n}, fma(y, hy{mu}_{n}, x * hx{mu}_{n})), {_lit(Fraction(1, n))}, s{mu});")
        for mu in mus:
            w(f"u = fma(fp[{mu}], s{mu}, u);")
        w.pop()
        w("}")


def _degree(keys, nu):
    return sorted((k for k in keys if k[0] + k[1] + k[2] == nu), key=lambda t: (-t[0], -t[1]))


def _monomial_closure(keys):
    """Every monomial on the construction chain of the given ones (z, then y, then x factors)."""
    need = set()
    for a, b, c in keys:
        for k in range(c + 1):
            need.add((a, b, k))
        for k in range(b + 1):
            need.add((a, k, 0))
        for k in range(a + 1):
            need.add((k, 0, 0))
    return need


def _emit_one_monomial(w, abc):
    """mono_a_b_c from the monomial one factor lower on its chain (z, then y, then x)."""
    a, b, c = abc
    name = _mono_name(abc)
    if a + b + c == 0:
        w(f"const R {name} = R(1);")
    elif c > 0:
        w(f"const R {name} = {_mono_name((a, b, c - 1))} * z;")
    elif b > 0:
        w(f"const R {name} = {_mono_name((a, b - 1, 0))} * y;")
    else:
        w(f"const R {name} = {_mono_name((a - 1, 0, 0))} * x;")


def _mono_name(abc):
    a, b, c = abc
    return f"mono_{a}_{b}_{c}"


def _group_ops(ops):
    """Group a block's ops by (dst, x): {(dst, x): [(y, w), ...]} preserving first-seen order."""
    groups = {}
    for dst, x, y, wgt in ops:
        groups.setdefault((dst, x), []).append((y, wgt))
    return groups


def _emit_block_forward(w: _W, blk, with_output=True):
    for k in range(blk.n_temp):
        w(f"R t{k} = R(0);")
    for (dst, x), lst in _group_ops(blk.ops).items():
        if dst[0] == "c" and not with_output:
            continue
        if lst[0][0] is None:
            w(f"{_ref(dst)} = {_ref(x)};")
            continue
        _emit_inner(w, lst, "s")
        w(f"{_ref(dst)} = fma({_ref(x)}, s, {_ref(dst)}); }}")


def _emit_inner(w, lst, var):
    (y0, w0) = lst[0]
    if w0 == 1:
        w(f"{{ R {var} = {_ref(y0)};")
    else:
        w(f"{{ R {var} = {_lit(w0)} * {_ref(y0)};")
    for y, wgt in lst[1:]:
        if wgt == 1:
            w(f"  {var} += {_ref(y)};")
        else:
            w(f"  {var} = fma({_lit(wgt)}, {_ref(y)}, {var});")


# Moment loads kept in flight by the reverse program (whose blocks are fenced to bound register
# pressure): each contraction block takes its entries from a ring of prefetched values and
# issues the load that many positions ahead, so the global-memory latency of one block is
# covered by the arithmetic of the blocks before it.
PREFETCH_DEPTH = int(os.environ.get("MTP_PREFETCH_DEPTH", "24"))
# the same for the tangent of the reverse program (which loads moments, their tangents and
# the contraction adjoints with their tangents)
TAN_PREFETCH_DEPTH = int(os.environ.get("MTP_TAN_PREFETCH_DEPTH", "24"))

# Register estimate (VGPRs) of the reverse tangent of one block: values, tangents, adjoints and
# adjoint tangents of its temporaries, the values and tangents of the entries it reads, and the
# prefetched loads.  A part of the reverse-tangent program adds the accumulators live at each of
# its blocks (two VGPRs each); parts are cut so that this stays within RTAN_REG_BUDGET (the 512
# VGPR + AGPR of one wave per SIMD).  The estimate is rough (some parts spill, some blocks over
# it do not); at level 20 budgets of 430, 512 and 545 measured 8.9, 8.1 and 8.05 ms.
RTAN_REG_BUDGET = int(os.environ.get("MTP_RTAN_BUDGET", "512"))
# blocks tried for each addition to a part (those adding the fewest new entries)
RTAN_CANDIDATES = 12


def _locality_order(blocks):
    """Contraction blocks reordered so that consecutive blocks share moment entries (each next
    block has the largest overlap with the entries of the last three): re-reads of an entry
    come soon after its first read and hit the cache.  The blocks are independent sums, so the
    order is free."""
    rem = list(blocks)
    if not rem:
        return rem
    order = [max(rem, key=lambda b: (len(b.entries), -b.q))]
    rem.remove(order[0])
    while rem:
        recent = set(e for b in order[-3:] for e in b.entries)
        nxt = max(rem, key=lambda b: (len(set(b.entries) & recent), -len(b.entries), -b.q))
        order.append(nxt)
        rem.remove(nxt)
    return order


def _emit_components_forward(w: _W, prog: Program):
    """Connected contractions.  No block fences here: the blocks are independent and the
    scheduler interleaves them freely (their loads overlap the arithmetic of other blocks)."""
    w("template <class R, class MA>")
    w("static __device__ __forceinline__ void fwd(const MA& M, R* __restrict__ C) {")
    w.push()
    for blk in _locality_order(prog.blocks):
        w(f"{{  // contraction {blk.q}")
        w.push()
        for e in blk.entries:
            w(f"const R me{e} = M({e});")
        w(f"C[{blk.q}] = R(0);")
        _emit_block_forward(w, blk)
        w.pop()
        w("}")
    w.pop()
    w("}")


def _emit_components_reverse(w: _W, prog: Program, groups):
    for gi, (lo, hi) in enumerate(groups):
        # Cb: anything indexable by component (a pointer, or a strided accessor of LDS)
        w("template <class R, class MA, class CB>")
        w(f"static __device__ __forceinline__ void rev_g{gi}(const MA& M, const CB& Cb, R* __restrict__ mb) {{")
        w.push()
        blocks = _locality_order([blk for blk in prog.blocks if any(lo <= e < hi for e in blk.entries)])
        seq = [e for blk in blocks for e in blk.entries]   # every moment load, in program order
        depth = max(1, min(PREFETCH_DEPTH, len(seq)))
        for k in range(depth):
            w(f"R pf{k} = M({seq[k]});")
        pos = 0
        for blk in blocks:
            w(f"{{  // contraction {blk.q}")
            w.push()
            w("MTP_BLOCK_FENCE();")
            for e in blk.entries:
                slot = pos % depth
                w(f"const R me{e} = pf{slot};")
                if pos + depth < len(seq):
                    w(f"pf{slot} = M({seq[pos + depth]});")
                pos += 1
            w(f"const R cb = Cb[{blk.q}];")
            _emit_block_forward(w, blk, with_output=False)
            for k in range(blk.n_temp):
                w(f"R tb{k} = R(0);")
            _emit_block_reverse(w, blk, lo, hi)
            w.pop()
            w("}")
        w.pop()
        w("}")


def _adj(ref, lo, hi):
    kind, k = ref
    if kind == "t":
        return f"tb{k}"
    if kind == "m":
        return f"mb[{k - lo}]" if lo <= k < hi else None
    return "cb"


def _emit_block_reverse(w: _W, blk, lo, hi):
    # walk steps backwards: ops were appended step by step
    rev_ops = list(reversed(blk.ops))
    # group by (dst, x) for x-adjoints and by (dst, y) for y-adjoints, in reverse step order
    seen_dst = []
    by_dst = defaultdict(list)
    for dst, x, y, wgt in rev_ops:
        if dst not in by_dst:
            seen_dst.append(dst)
        by_dst[dst].append((x, y, wgt))
    for dst in seen_dst:
        lst = by_dst[dst]
        db = _adj(dst, lo, hi)
        if lst[0][1] is None:
            (x, _, _), = lst
            tgt = _adj(x, lo, hi)
            if tgt:
                w(f"{tgt} += {db};")
            continue
        xs = {}
        ys = {}
        for x, y, wgt in lst:
            xs.setdefault(x, []).append((y, wgt))
            ys.setdefault(y, []).append((x, wgt))
        for x, l2 in xs.items():
            tgt = _adj(x, lo, hi)
            if not tgt:
                continue
            _emit_inner(w, l2, "s")
            w(f"{tgt} = fma({db}, s, {tgt}); }}")
        for y, l2 in ys.items():
            tgt = _adj(y, lo, hi)
            if not tgt:
                continue
            _emit_inner(w, l2, "s")
            w(f"{tgt} = fma({db}, s, {tgt}); }}")


def _emit_products(w: _W, prog: Program):
    children = defaultdict(list)
    roots = []
    for a, (parent, comp) in enumerate(prog.trie):
        if parent < 0:
            roots.append(a)
        else:
            children[parent].append(a)
    w("// E_i contribution sum_alpha xi_alpha B_alpha; Cb_q = dE_i/dC_q; B written when Bo != nullptr")
    w("template <bool WB, class R>")
    w("static __device__ __forceinline__ double products(const R* __restrict__ C, const double* __restrict__ xi,")
    w("    R* __restrict__ Cb, double* __restrict__ Bo, long ldb) {")
    w.push()
    w("double e = 0.0;")
    for q in range(prog.n_comp):
        w(f"Cb[{q}] = R(0);")

    def node2(a, parent_var):
        # variant that leaves bb{a} declared in the enclosing scope
        parent, comp = prog.trie[a]
        w(f"R bb{a};")
        w("{")
        w.push()
        if parent_var is None:
            w(f"const R b = C[{comp}];")
        else:
            w(f"const R b = {parent_var} * C[{comp}];")
        w(f"e = fma(xi[{a}], double(b), e);")
        w(f"if constexpr (WB) Bo[{a} * ldb] = double(b);")
        w(f"bb{a} = R(xi[{a}]);")
        if children[a]:
            w(f"const R p{a} = b;")
            for ch in children[a]:
                node2(ch, f"p{a}")
                _, ccomp = prog.trie[ch]
                w(f"bb{a} = fma(bb{ch}, C[{ccomp}], bb{a});")
        w.pop()
        w("}")
        if parent_var is None:
            w(f"Cb[{comp}] += bb{a};")
        else:
            w(f"Cb[{comp}] = fma(bb{a}, {parent_var}, Cb[{comp}]);")

    for a in roots:
        node2(a, None)
    w("return e;")
    w.pop()
    w("}")


def _emit_dispatchers(w: _W, n_groups: int):
    sigs = (
        ("acc_moments", "R* __restrict__ m, const R* __restrict__ f, R x, R y, R z", "m, f, x, y, z", "class R"),
        ("pair_grad", "const R* __restrict__ mb, const R* __restrict__ f, const R* __restrict__ fp, R x, R y, R z, "
                      "R& gx, R& gy, R& gz, R& u", "mb, f, fp, x, y, z, gx, gy, gz, u", "class R"),
        ("rev", "const MA& M, const CB& Cb, R* __restrict__ mb", "M, Cb, mb", "class R, class MA, class CB"),
    )
    for name, params, args, tparams in sigs:
        w(f"template <int G, {tparams}>")
        w(f"static __device__ __forceinline__ void {name}({params}) {{")
        w.push()
        for g in range(n_groups):
            kw = "if constexpr" if g == 0 else "else if constexpr"
            targs = "<R>" if name != "rev" else "<R, MA, CB>"
            w(f"{kw} (G == {g}) {name}_g{g}{targs}({args});")
        w.pop()
        w("}")


def emit_level(level: int, n_groups: int = 1, rtan_budget: int = RTAN_REG_BUDGET) -> str:
    prog = build_program(level)
    groups = entry_groups(prog, n_groups)
    agroups = adj_entry_groups(prog)
    w = _W()
    w(f"// Generated MTP level-{level} program.  Do not edit; produced by codegen/emit.py.")
    w("#pragma once")
    w(f"struct Lv{level} {{")
    w.push()
    w(f"static constexpr int LEVEL = {level};")
    w(f"static constexpr int NMOM = {prog.n_mom};")
    w(f"static constexpr int NCOMP = {prog.n_comp};")
    w(f"static constexpr int NALPHA = {prog.n_alpha};")
    w(f"static constexpr int NMU = {prog.n_mu};")
    w(f"static constexpr int MAXNU = {prog.max_nu};")
    w(f"static constexpr int NGROUP = {len(groups)};")
    w(f"static constexpr int TRIPLES = {prog.triple_count()};")
    w("static constexpr int GROUP_LO[NGROUP] = {" + ", ".join(str(g[0]) for g in groups) + "};")
    w("static constexpr int GROUP_HI[NGROUP] = {" + ", ".join(str(g[1]) for g in groups) + "};")
    # ranges of the adjoint pair kernel and the mu values [AMU_LO, AMU_HI] each one touches
    w(f"static constexpr int NAGROUP = {len(agroups)};")
    w("static constexpr int AGROUP_LO[NAGROUP] = {" + ", ".join(str(g[0]) for g in agroups) + "};")
    w("static constexpr int AGROUP_HI[NAGROUP] = {" + ", ".join(str(g[1]) for g in agroups) + "};")
    w("static constexpr int AMU_LO[NAGROUP] = {" + ", ".join(str(prog.layout.items[g[0]][0]) for g in agroups) + "};")
    w("static constexpr int AMU_HI[NAGROUP] = {" + ", ".join(str(prog.layout.items[g[1] - 1][0]) for g in agroups) + "};")
    # ranges of the moment-tangent kernel
    tgroups = tangent_moment_groups(groups, agroups, prog.level)
    rparts = rev_tan_parts(prog, rtan_budget)
    # parts of the reverse-tangent program, run in order (one kernel each)
    w(f"static constexpr int NRTPART = {len(rparts)};")
    w(f"static constexpr int NTGROUP = {len(tgroups)};")
    w("static constexpr int TGROUP_LO[NTGROUP] = {" + ", ".join(str(g[0]) for g in tgroups) + "};")
    w("static constexpr int TGROUP_HI[NTGROUP] = {" + ", ".join(str(g[1]) for g in tgroups) + "};")
    w("// flat moment layout: (mu, a, b, c) of component e")
    w("static constexpr int ENTRIES[NMOM][4] = {" + ", ".join("{%d, %d, %d, %d}" % it for it in prog.layout.items) + "};")
    # a! b! c! of each entry: pair_grad takes the moment adjoints scaled by it
    w("static constexpr double MFACT[NMOM] = {" + ", ".join(
        "%d." % (math.factorial(a) * math.factorial(b) * math.factorial(c)) for (_, a, b, c) in prog.layout.items) + "};")
    _emit_pair_functions(w, prog, groups)
    _emit_components_forward(w, prog)
    _emit_components_reverse(w, prog, groups)
    _emit_products(w, prog)
    _emit_dispatchers(w, len(groups))
    emit_tangent_parts(w, prog, groups, agroups, rparts)
    w.pop()
    w("};")
    return w.text()


def write_level(level: int, out_dir: str, n_groups: int = 1) -> str:
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, f"mtp_L{level}.inc")
    text = emit_level(level, n_groups)
    old = None
    if os.path.exists(path):
        with open(path) as fh:
            old = fh.read()
    if old != text:
        with open(path, "w") as fh:
            fh.write(text)
    return path


# ======================================================================================
# tangent (forward-mode) code for the parameter adjoint
#
# The parameter gradient needs, per atom, the directional derivative of every quantity
# along the per-pair displacement change delta_ij = fbar_j - fbar_i:
#   md   = sum_j d/dd [f_mu(r) mono_e(d)] . delta          (tangent of the moments)
#   Cd, Bd                                                  (tangents of contractions/basis)
#   Cbd, mbd                                                (tangents of the adjoints)
# Each generated function mirrors its value counterpart and carries a tangent next to
# every value (forward-over-reverse).


def _emit_tangent_pair_functions(w: _W, prog: Program, groups):
    items = prog.layout.items
    for gi, (lo, hi) in enumerate(groups):
        ents = list(range(lo, hi))
        gnu = max(a + b + c for (_, a, b, c) in (items[e] for e in ents))
        order = sorted({items[e][1:] for e in ents}, key=lambda t: (t[0] + t[1] + t[2], -t[0], -t[1]))
        # ---------------- tangent of the moments along delta
        w("template <class R>")
        w(f"static __device__ __forceinline__ void tan_moments_g{gi}(R* __restrict__ md, const R* __restrict__ f,")
        w("    const R* __restrict__ fp, R x, R y, R z, R ex, R ey, R ez, R rdot) {")
        w.push()
        _emit_monomials_with_tangent(w, order)
        by_mono = defaultdict(list)
        for e in ents:
            mu, a, b, c = items[e]
            by_mono[(a, b, c)].append((e, mu))
        for abc in order:
            for e, mu in by_mono[abc]:
                w(f"md[{e - lo}] = fma(f[{mu}], {_tmono_name(abc)}, fma(fp[{mu}] * rdot, {_mono_name(abc)}, md[{e - lo}]));")
        w.pop()
        w("}")


def _emit_adj_pair_functions(w: _W, prog: Program, agroups):
    """Per-mu sums of the adjoint pair term over one adjoint group:
    S_mu = sum_e mb_e mono_e ;  A_mu = sum_e (mbd_e mono_e + mb_e dmono_e)."""
    items = prog.layout.items
    for gi, (lo, hi) in enumerate(agroups):
        ents = list(range(lo, hi))
        order = sorted({items[e][1:] for e in ents}, key=lambda t: (t[0] + t[1] + t[2], -t[0], -t[1]))
        by_mono = defaultdict(list)
        for e in ents:
            mu, a, b, c = items[e]
            by_mono[(a, b, c)].append((e, mu))
        w(f"// adjoint group {gi}: entries [{lo}, {hi})")
        w("template <class R>")
        w(f"static __device__ __forceinline__ void adj_pair_g{gi}(const R* __restrict__ mb, const R* __restrict__ mbd,")
        w("    R x, R y, R z, R ex, R ey, R ez, R* __restrict__ S, R* __restrict__ A) {")
        w.push()
        # ADJ_CHAINS independent partial sums per mu shorten the dependent fma chains
        mus = sorted({items[e][0] for e in ents})
        nch = {mu: min(ADJ_CHAINS, sum(1 for e in ents if items[e][0] == mu)) for mu in mus}
        for mu in mus:
            w(" ".join(f"R s{mu}_{k} = R(0), a{mu}_{k} = R(0);" for k in range(nch[mu])))
        _emit_monomials_with_tangent(w, order)
        seen = defaultdict(int)
        for abc in order:
            for e, mu in by_mono[abc]:
                k = seen[mu] % nch[mu]
                seen[mu] += 1
                w(f"s{mu}_{k} = fma(mb[{e - lo}], {_mono_name(abc)}, s{mu}_{k});")
                w(f"a{mu}_{k} = fma(mbd[{e - lo}], {_mono_name(abc)}, fma(mb[{e - lo}], {_tmono_name(abc)}, a{mu}_{k}));")
        for mu in mus:
            w(f"S[{mu}] += " + _pair_sum([f"s{mu}_{k}" for k in range(nch[mu])]) + ";")
            w(f"A[{mu}] += " + _pair_sum([f"a{mu}_{k}" for k in range(nch[mu])]) + ";")
        w.pop()
        w("}")


ADJ_CHAINS = 4


def _pair_sum(names):
    """Balanced sum expression of names."""
    if len(names) == 1:
        return names[0]
    h = len(names) // 2
    return f"({_pair_sum(names[:h])} + {_pair_sum(names[h:])})"


def _tmono_name(abc):
    a, b, c = abc
    return f"tmono_{a}_{b}_{c}"


def _emit_monomials_with_tangent(w, order):
    """mono = x^a y^b z^c and tmono = grad(mono) . (ex, ey, ez), built by one factor at a time."""
    have = set()
    need = set()
    # close the set downwards along the construction chain
    for abc in order:
        a, b, c = abc
        for k in range(c + 1):
            need.add((a, b, k))
        for k in range(b + 1):
            need.add((a, k, 0))
        for k in range(a + 1):
            need.add((k, 0, 0))
    for abc in sorted(need, key=lambda t: (t[0] + t[1] + t[2], -t[0], -t[1])):
        a, b, c = abc
        name, tname = _mono_name(abc), _tmono_name(abc)
        if a + b + c == 0:
            w(f"const R {name} = R(1);")
            w(f"const R {tname} = R(0);")
            have.add(abc)
            continue
        if c > 0:
            low, var, ev = (a, b, c - 1), "z", "ez"
        elif b > 0:
            low, var, ev = (a, b - 1, 0), "y", "ey"
        else:
            low, var, ev = (a - 1, 0, 0), "x", "ex"
        assert low in have
        w(f"const R {name} = {_mono_name(low)} * {var};")
        if low == (0, 0, 0):
            w(f"const R {tname} = {ev};")
        else:
            w(f"const R {tname} = fma({_tmono_name(low)}, {var}, {_mono_name(low)} * {ev});")
        have.add(abc)


def _tref(r):
    kind, k = r
    if kind == "m":
        return f"mde{k}"
    if kind == "t":
        return f"td{k}"
    return f"Cd[{k}]"


def _emit_block_forward_tangent(w: _W, blk, with_output=True):
    for k in range(blk.n_temp):
        w(f"R t{k} = R(0), td{k} = R(0);")
    for (dst, x), lst in _group_ops(blk.ops).items():
        if dst[0] == "c" and not with_output:
            continue
        if lst[0][0] is None:
            w(f"{_ref(dst)} = {_ref(x)};")
            w(f"{_tref(dst)} = {_tref(x)};")
            continue
        _emit_inner2(w, lst)
        w(f"  {_tref(dst)} = fma({_tref(x)}, s, fma({_ref(x)}, sd, {_tref(dst)}));")
        w(f"  {_ref(dst)} = fma({_ref(x)}, s, {_ref(dst)}); }}")


def _emit_inner2(w, lst):
    """s = sum w y and sd = sum w yd over a group."""
    (y0, w0) = lst[0]
    if w0 == 1:
        w(f"{{ R s = {_ref(y0)}, sd = {_tref(y0)};")
    else:
        w(f"{{ R s = {_lit(w0)} * {_ref(y0)}, sd = {_lit(w0)} * {_tref(y0)};")
    for y, wgt in lst[1:]:
        if wgt == 1:
            w(f"  s += {_ref(y)}; sd += {_tref(y)};")
        else:
            w(f"  s = fma({_lit(wgt)}, {_ref(y)}, s); sd = fma({_lit(wgt)}, {_tref(y)}, sd);")


def _emit_components_forward_tangent(w: _W, prog: Program):
    w("template <class R, class MA>")
    w("static __device__ __forceinline__ void fwd_tan(const MA& M, const MA& Md, R* __restrict__ C, R* __restrict__ Cd) {")
    w.push()
    for blk in _locality_order(prog.blocks):
        w(f"{{  // contraction {blk.q}")
        w.push()
        for e in blk.entries:
            w(f"const R me{e} = M({e}), mde{e} = Md({e});")
        w(f"C[{blk.q}] = R(0); Cd[{blk.q}] = R(0);")
        _emit_block_forward_tangent(w, blk)
        w.pop()
        w("}")
    w.pop()
    w("}")


def _adj2(ref, slot):
    """(adjoint, adjoint tangent) names of a reference inside a reverse-tangent block; slot maps
    the moment entries accumulated by the part to their register index."""
    kind, k = ref
    if kind == "t":
        return f"tb{k}", f"tbd{k}"
    if kind == "m":
        return (None, f"mbd[{slot[k]}]") if k in slot else (None, None)
    return "cb", "cbd"


def _emit_block_reverse_tangent(w: _W, blk, slot, flush=None):
    """The block read backwards.  flush maps moment entries to the line that stores their
    accumulated adjoint tangent; each such line is emitted right after the entry's last update
    in the block, so its register is free for the rest of the block."""
    rev_ops = list(reversed(blk.ops))
    seen_dst = []
    by_dst = defaultdict(list)
    for dst, x, y, wgt in rev_ops:
        if dst not in by_dst:
            seen_dst.append(dst)
        by_dst[dst].append((x, y, wgt))
    items = []  # (lines, moment entry updated or None)
    for dst in seen_dst:
        lst = by_dst[dst]
        db, dbd = _adj2(dst, slot)
        if lst[0][1] is None:
            (x, _, _), = lst
            xb, xbd = _adj2(x, slot)
            lines = []
            if xb:
                lines.append(f"{xb} += {db};")
            if xbd:
                lines.append(f"{xbd} += {dbd};")
            items.append((lines, x[1] if x[0] == "m" and xbd else None))
            continue
        xs, ys = {}, {}
        for x, y, wgt in lst:
            xs.setdefault(x, []).append((y, wgt))
            ys.setdefault(y, []).append((x, wgt))
        for x, l2 in xs.items():
            xb, xbd = _adj2(x, slot)
            if not xb and not xbd:
                continue
            sub = _W()
            _emit_inner2(sub, l2)
            if xb:
                sub(f"  {xb} = fma({db}, s, {xb});")
            sub(f"  {xbd} = fma({dbd}, s, fma({db}, sd, {xbd})); }}")
            items.append((sub.lines, x[1] if x[0] == "m" else None))
        for y, l2 in ys.items():
            yb, ybd = _adj2(y, slot)
            if not ybd:
                continue
            sub = _W()
            _emit_inner2(sub, l2)
            sub(f"  {ybd} = fma({dbd}, s, fma({db}, sd, {ybd})); }}")
            items.append((sub.lines, y[1] if y[0] == "m" else None))
    flush = dict(flush or {})
    last = {e: i for i, (_, e) in enumerate(items) if e is not None}
    for i, (lines, e) in enumerate(items):
        for line in lines:
            w(line)
        if e is not None and last[e] == i and e in flush:
            w(flush.pop(e))
    for line in flush.values():
        w(line)


def _rtan_peak(blk):
    return 8 * blk.n_temp + 4 * len(blk.entries) + 48


def _rtan_live(order):
    """Register estimate of a part whose blocks run in the given order: an entry's accumulator
    lives from the first block of the part that touches it to the last one (where it is stored
    after its last update), next to the block's own need."""
    first, last = {}, {}
    for i, b in enumerate(order):
        for e in b.entries:
            first.setdefault(e, i)
            last[e] = i
    starts, ends = defaultdict(int), defaultdict(int)
    for e in first:
        starts[first[e]] += 1
        ends[last[e]] += 1
    live = worst = 0
    for i, b in enumerate(order):
        live += starts[i]
        worst = max(worst, 2 * live + _rtan_peak(b))
        live -= ends[i]
    return worst


def rev_tan_parts(prog: Program, budget=RTAN_REG_BUDGET):
    """Contraction blocks of the reverse-tangent program cut into parts (one kernel each).  A
    part starts from the remaining block with the largest register need and takes, while the
    estimate of the part in locality order fits the budget, the block that adds the fewest new
    moment entries (among the closest few candidates).  Returns the parts as lists of blocks
    in locality order."""
    rem = sorted(prog.blocks, key=lambda b: b.q)
    parts = []
    while rem:
        b0 = max(rem, key=lambda b: (_rtan_peak(b), len(b.ops), -b.q))
        rem.remove(b0)
        cur, es = [b0], set(b0.entries)
        while rem:
            cand = sorted(rem, key=lambda b: (len(set(b.entries) - es), -len(b.ops), b.q))[:RTAN_CANDIDATES]
            nb = next((b for b in cand if _rtan_live(_locality_order(cur + [b])) <= budget), None)
            if nb is None:
                break
            cur.append(nb)
            rem.remove(nb)
            es |= set(nb.entries)
        parts.append(_locality_order(cur))
    return parts


def _emit_components_reverse_tangent(w: _W, prog: Program, parts):
    """One function per part: the forward tangent of each of its blocks again, then the block
    read backwards, accumulating the tangents of the moment adjoints of the entries the part
    touches.  The part that touches an entry first stores it, later parts add to it, and the
    first part stores zero for entries no block reads, so running the parts in order leaves
    out[e * ld] = d(mbar_e) for every entry."""
    first = {}
    for pi, part in enumerate(parts):
        for blk in part:
            for e in blk.entries:
                first.setdefault(e, pi)
    for pi, part in enumerate(parts):
        entries = sorted(set(e for b in part for e in b.entries))
        slot = {e: k for k, e in enumerate(entries)}
        w("template <class R, class MA, class CB, class OUT>")
        w(f"static __device__ __forceinline__ void rev_tan_p{pi}(const MA& M, const MA& Md, const CB& Cb,")
        w("    const CB& Cbd, const OUT& out, long ld) {")
        w.push()
        last = {}
        for bi, blk in enumerate(part):
            for e in blk.entries:
                last[e] = bi
        started = set()
        w(f"R mbd[{len(entries)}];")
        # every load of the program in order (moments, their tangents, then the block's adjoint
        # pair), kept TAN_PREFETCH_DEPTH ahead across the fenced blocks
        seq = []
        for blk in part:
            seq += [(f"me{e}", f"M({e})") for e in blk.entries] + [(f"mde{e}", f"Md({e})") for e in blk.entries]
            seq += [("cb", f"Cb[{blk.q}]"), ("cbd", f"Cbd[{blk.q}]")]
        depth = max(1, min(TAN_PREFETCH_DEPTH, len(seq)))
        for k in range(depth):
            w(f"R pf{k} = {seq[k][1]};")
        pos = 0
        for bi, blk in enumerate(part):
            w(f"{{  // contraction {blk.q}")
            w.push()
            w("MTP_BLOCK_FENCE();")
            for _ in range(2 * len(blk.entries) + 2):
                sl = pos % depth
                w(f"const R {seq[pos][0]} = pf{sl};")
                if pos + depth < len(seq):
                    w(f"pf{sl} = {seq[pos + depth][1]};")
                pos += 1
            for e in blk.entries:
                if e not in started:
                    started.add(e)
                    w(f"mbd[{slot[e]}] = R(0);")
            _emit_block_forward_tangent(w, blk, with_output=False)
            for k in range(blk.n_temp):
                w(f"R tb{k} = R(0), tbd{k} = R(0);")
            # entries the part touches for the last time here are stored after their last update
            flush = {e: f"out[{e} * ld] {'=' if first[e] == pi else '+='} double(mbd[{slot[e]}]);"
                     for e in blk.entries if last[e] == bi}
            _emit_block_reverse_tangent(w, blk, slot, flush)
            w.pop()
            w("}")
        if pi == 0:
            for e in range(prog.n_mom):
                if e not in first:
                    w(f"out[{e} * ld] = 0.0;")
        w.pop()
        w("}")


def _emit_products_tangent(w: _W, prog: Program):
    children = defaultdict(list)
    roots = []
    for a, (parent, comp) in enumerate(prog.trie):
        if parent < 0:
            roots.append(a)
        else:
            children[parent].append(a)
    w("// Basis values and tangents; writes out[alpha * ld] = ebar B_alpha - dB_alpha, and the")
    w("// adjoints Cb_q = dE_i/dC_q with their tangents Cbd_q.")
    w("template <class R>")
    w("static __device__ __forceinline__ void products_tan(const R* __restrict__ C, const R* __restrict__ Cd,")
    w("    const double* __restrict__ xi, double ebar, R* __restrict__ Cb, R* __restrict__ Cbd,")
    w("    double* __restrict__ out, long ld) {")
    w.push()
    for q in range(prog.n_comp):
        w(f"Cb[{q}] = R(0); Cbd[{q}] = R(0);")

    def node(a, pv, pdv):
        parent, comp = prog.trie[a]
        w(f"R bb{a}, bbd{a};")
        w("{")
        w.push()
        if pv is None:
            w(f"const R b = C[{comp}], bd = Cd[{comp}];")
        else:
            w(f"const R b = {pv} * C[{comp}];")
            w(f"const R bd = fma({pdv}, C[{comp}], {pv} * Cd[{comp}]);")
        w(f"out[{a} * ld] = fma(ebar, double(b), -double(bd));")
        w(f"bb{a} = R(xi[{a}]); bbd{a} = R(0);")
        if children[a]:
            w(f"const R p{a} = b, pd{a} = bd;")
            for ch in children[a]:
                node(ch, f"p{a}", f"pd{a}")
                _, cc = prog.trie[ch]
                w(f"bbd{a} = fma(bbd{ch}, C[{cc}], fma(bb{ch}, Cd[{cc}], bbd{a}));")
                w(f"bb{a} = fma(bb{ch}, C[{cc}], bb{a});")
        w.pop()
        w("}")
        if pv is None:
            w(f"Cb[{comp}] += bb{a}; Cbd[{comp}] += bbd{a};")
        else:
            w(f"Cbd[{comp}] = fma(bbd{a}, {pv}, fma(bb{a}, {pdv}, Cbd[{comp}]));")
            w(f"Cb[{comp}] = fma(bb{a}, {pv}, Cb[{comp}]);")

    for a in roots:
        node(a, None, None)
    w.pop()
    w("}")


def _emit_tangent_dispatchers(w: _W, n_rtparts: int, n_agroups: int, n_tgroups: int):
    sigs = (
        ("tan_moments", "R* __restrict__ md, const R* __restrict__ f, const R* __restrict__ fp, R x, R y, R z, "
                        "R ex, R ey, R ez, R rdot", "md, f, fp, x, y, z, ex, ey, ez, rdot", "class R", "<R>"),
        ("adj_pair", "const R* __restrict__ mb, const R* __restrict__ mbd, R x, R y, R z, R ex, R ey, R ez, "
                     "R* __restrict__ S, R* __restrict__ A", "mb, mbd, x, y, z, ex, ey, ez, S, A", "class R", "<R>"),
        ("rev_tan", "const MA& M, const MA& Md, const CB& Cb, const CB& Cbd, "
                    "const OUT& out, long ld", "M, Md, Cb, Cbd, out, ld", "class R, class MA, class CB, class OUT",
         "<R, MA, CB>"),
    )
    for name, params, args, tparams, targs in sigs:
        w(f"template <int G, {tparams}>")
        w(f"static __device__ __forceinline__ void {name}({params}) {{")
        w.push()
        count = {"adj_pair": n_agroups, "tan_moments": n_tgroups, "rev_tan": n_rtparts}[name]
        tag = "p" if name == "rev_tan" else "g"
        for g in range(count):
            kw = "if constexpr" if g == 0 else "else if constexpr"
            w(f"{kw} (G == {g}) {name}_{tag}{g}{targs}({args});")
        w.pop()
        w("}")


# Extra cuts of the chain's groups for the moment-tangent kernel, by level.  Measured at level
# 20: the second group (entries 98-196, the higher-order moments) spilled 208 bytes per lane
# in that kernel and took 2.6 ms of the batch step; cut at entry 148, its two passes take 1.85.
TANGENT_EXTRA_CUTS = {20: (148,)}


def tangent_moment_groups(groups, agroups, level=None):
    """Ranges of the moment-tangent kernel: the adjoint ranges where the chain has one group
    (its whole layout does not fit in registers next to the tangent monomials), else the
    chain's groups (measured faster at level 20 than seven passes over the pairs), cut further
    at the level's extra cuts."""
    if len(groups) == 1:
        return agroups
    cuts = TANGENT_EXTRA_CUTS.get(level, ())
    out = []
    for lo, hi in groups:
        inner = sorted(c for c in cuts if lo < c < hi)
        bounds = [lo] + inner + [hi]
        out += [(bounds[k], bounds[k + 1]) for k in range(len(bounds) - 1)]
    return out


def emit_tangent_parts(w: _W, prog: Program, groups, agroups, rparts):
    tgroups = tangent_moment_groups(groups, agroups, prog.level)
    _emit_tangent_pair_functions(w, prog, tgroups)
    _emit_adj_pair_functions(w, prog, agroups)
    _emit_components_forward_tangent(w, prog)
    _emit_components_reverse_tangent(w, prog, rparts)
    _emit_products_tangent(w, prog)
    _emit_tangent_dispatchers(w, len(rparts), len(agroups), len(tgroups))
