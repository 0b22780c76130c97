"""Oracle: plain float64 CPU evaluation of the Moment Tensor Potential.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library never
does, and it shares no code, table or helper with it.

What is computed (the paper defines the MTP by reference to its original
formulation and MLIP-3, Section 1; Section 2.1 states that inference yields
energies, forces and stresses and that active learning adds an extrapolation
grade).  Readings taken where the paper is silent are listed in the design
notes of the repository and repeated briefly here:

  u        = (2 r - (r_min + r_cut)) / (r_cut - r_min)
  Q_beta   = T_beta(u) (r_cut - r)^2               Chebyshev T, beta < n_cheb, no clamping
  f_mu     = sum_beta c[z_i, z_j, mu, beta] Q_beta  (ordered species pair)
  M_mu,nu  = sum_j f_mu(r_ij) d_ij^(x nu)          full displacement d_ij (not unit)
  B_alpha  = full contraction of the moments of basis function alpha
  E_i      = s[z_i] + sum_alpha xi_alpha B_alpha(i);   E = sum_i E_i
  F_k      = -dE/dR_k;   W = -sum_pairs d_ij (x) dE_i/dd_ij  (xx, yy, zz, xy, xz, yz)
  grade_i  = max_k |(B_i A^-1)_k|                  neighbourhood mode
  grade    = max_k |((sum_i B_i) A^-1)_k|          configuration mode (b = dE/dxi)

Everything is evaluated the plain way: dense 3^nu tensors, one einsum per
basis function, derivatives by PyTorch autograd (a library primitive), no
blocking or reuse beyond that.
"""
from __future__ import annotations

import functools

import numpy as np
import torch

from . import basis as _basis
from . import neighbors as _nb

VIRIAL_ORDER = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


@functools.lru_cache(maxsize=None)
def basis_for(level: int):
    return tuple(_basis.enumerate_basis(level))


class Model:
    """Hyper-parameters and coefficients of one potential (float64)."""

    def __init__(self, level, n_species, n_cheb, r_min, r_cut, radial, linear, shift):
        self.level = int(level)
        self.n_species = int(n_species)
        self.n_cheb = int(n_cheb)
        self.r_min = float(r_min)
        self.r_cut = float(r_cut)
        self.basis = basis_for(self.level)
        self.n_alpha = len(self.basis)
        self.n_mu = _basis.radial_count(self.level, self.basis)
        self.moments = _basis.used_moments(self.basis)
        self.radial = torch.as_tensor(np.asarray(radial, dtype=np.float64))
        self.linear = torch.as_tensor(np.asarray(linear, dtype=np.float64))
        self.shift = torch.as_tensor(np.asarray(shift, dtype=np.float64))
        assert self.radial.shape == (self.n_species, self.n_species, self.n_mu, self.n_cheb)
        assert self.linear.shape == (self.n_alpha,)
        assert self.shift.shape == (self.n_species,)

    @classmethod
    def from_params(cls, p):
        return cls(p.level, p.n_species, p.n_cheb, p.r_min, p.r_cut, p.radial, p.linear, p.shift)


# ----------------------------------------------------------------------------- radial part


def chebyshev(u, n):
    """[..., n] values T_0(u) .. T_{n-1}(u) by the three-term recurrence."""
    out = [torch.ones_like(u)]
    if n > 1:
        out.append(u)
    for b in range(2, n):
        out.append(2.0 * u * out[b - 1] - out[b - 2])
    return torch.stack(out[:n], dim=-1)


def radial_basis(r, r_min, r_cut, n_cheb):
    """Q_beta(r) = T_beta(u) (r_cut - r)^2 with u mapping [r_min, r_cut] onto [-1, 1]."""
    u = (2.0 * r - (r_min + r_cut)) / (r_cut - r_min)
    return chebyshev(u, n_cheb) * ((r_cut - r) ** 2)[..., None]


def radial_functions(model, r, zi, zj, radial=None):
    """f[p, mu] = sum_beta c[z_i, z_j, mu, beta] Q_beta(r_p)."""
    c = model.radial if radial is None else radial
    q = radial_basis(r, model.r_min, model.r_cut, model.n_cheb)
    return torch.einsum("pmb,pb->pm", c[zi, zj], q)


# ----------------------------------------------------------------------------- moments + basis


def moment_tensors(model, d, centre, n_centres, f):
    """Dense moments {(mu, nu): [n_centres, 3, ..., 3]} = sum_j f_mu d^(x nu)."""
    out = {}
    by_nu = {}
    for mu, nu in model.moments:
        by_nu.setdefault(nu, []).append(mu)
    power = torch.ones(d.shape[0], dtype=d.dtype)          # d^(x 0)
    for nu in range(max(by_nu) + 1):
        if nu > 0:
            power = power[..., None] * d.reshape((d.shape[0],) + (1,) * (nu - 1) + (3,))
        for mu in by_nu.get(nu, []):
            contrib = f[:, mu].reshape((-1,) + (1,) * nu) * power
            acc = torch.zeros((n_centres,) + (3,) * nu, dtype=d.dtype)
            out[(mu, nu)] = acc.index_add(0, centre, contrib)
    return out


_LETTERS = "abcdefghijklmnopqrstuvwxy"


def einsum_spec(bf):
    """Subscripts contracting the tensors of one basis function (batch letter z)."""
    k = len(bf.labels)
    m = bf.matrix()
    subs = [[] for _ in range(k)]
    nxt = 0
    for a in range(k):
        for b in range(a + 1, k):
            for _ in range(m[a][b]):
                ch = _LETTERS[nxt]
                nxt += 1
                subs[a].append(ch)
                subs[b].append(ch)
    return ",".join("z" + "".join(s) for s in subs) + "->z"


def basis_values(model, mom):
    """B [n_centres, n_alpha]: one dense contraction per basis function."""
    cols = []
    for bf in model.basis:
        ops = [mom[lab] for lab in bf.labels]
        cols.append(torch.einsum(einsum_spec(bf), *ops))
    return torch.stack(cols, dim=1)


def site_quantities(model, d, centre, zc, zn, n_centres, radial=None, linear=None, shift=None):
    """(E_i [n_centres], B [n_centres, n_alpha]) for the centres owning pairs d."""
    r = torch.sqrt((d * d).sum(dim=1))
    f = radial_functions(model, r, zc[centre], zn, radial)
    mom = moment_tensors(model, d, centre, n_centres, f)
    b = basis_values(model, mom)
    xi = model.linear if linear is None else linear
    s = model.shift if shift is None else shift
    e = s[zc] + b @ xi
    return e, b


# ----------------------------------------------------------------------------- whole system


def _pairs(struct, nl):
    i = torch.as_tensor(nl["i"].astype(np.int64))
    j = torch.as_tensor(nl["j"].astype(np.int64))
    d = _nb.displacements(struct.pos, struct.cell, nl["i"], nl["j"], nl["n"])
    return i, j, torch.as_tensor(d)


def energy_forces_virial(model, struct, nl=None, radial=None, linear=None, shift=None,
                         create_graph=False):
    """Return dict(E, E_i, F [N,3], W [6], B [N, n_alpha], g [P,3]) as torch float64."""
    if nl is None:
        nl = _nb.neighbor_csr(struct.pos, struct.cell, model.r_cut)
    n = struct.n_atoms
    i, j, d = _pairs(struct, nl)
    d = d.clone().requires_grad_(True)
    z = torch.as_tensor(struct.species.astype(np.int64))
    e_i, b = site_quantities(model, d, i, z, z[j], n, radial, linear, shift)
    e = e_i.sum()
    (g,) = torch.autograd.grad(e, d, create_graph=create_graph)
    f = torch.zeros((n, 3), dtype=d.dtype).index_add(0, i, g).index_add(0, j, -g)
    w = torch.stack([-(d[:, a] * g[:, c]).sum() for a, c in VIRIAL_ORDER])
    return dict(E=e, E_i=e_i, F=f, W=w, B=b, g=g, d=d, nl=nl)


def energy_from_positions(model, pos, struct, nl, cell=None):
    """E as a function of (possibly perturbed) positions and cell on a fixed pair list."""
    cell = struct.cell if cell is None else cell
    d = torch.as_tensor(_nb.displacements(pos, cell, nl["i"], nl["j"], nl["n"]))
    i = torch.as_tensor(nl["i"].astype(np.int64))
    z = torch.as_tensor(struct.species.astype(np.int64))
    e_i, _ = site_quantities(model, d, i, z, z[torch.as_tensor(nl["j"].astype(np.int64))],
                             struct.n_atoms)
    return float(e_i.sum())


def grade(b, ainv):
    """Neighbourhood-mode grade per atom: max_k |sum_alpha B[i, alpha] Ainv[alpha, k]|."""
    b = np.asarray(b, dtype=np.float64)
    return np.abs(b @ np.asarray(ainv, dtype=np.float64)).max(axis=1)


def config_descriptor(b):
    """Configuration-mode descriptor: sum over atoms of B_i (equal to dE/dxi)."""
    return np.asarray(b, dtype=np.float64).sum(axis=0)


def config_grade(b, ainv):
    """Configuration-mode grade (Section 2.1 names the mode; the MLIP-3 definition it follows):
    max_k |(sum_i B_i) A^-1|_k for one configuration."""
    return float(np.abs(config_descriptor(b) @ np.asarray(ainv, dtype=np.float64)).max())


def param_vjp(model, struct, ebar, fbar, nl=None):
    """(d_xi, d_c, d_s) = ebar dE/dtheta + sum_k fbar_k . dF_k/dtheta (vector-Jacobian product)."""
    radial = model.radial.clone().requires_grad_(True)
    linear = model.linear.clone().requires_grad_(True)
    shift = model.shift.clone().requires_grad_(True)
    out = energy_forces_virial(model, struct, nl, radial, linear, shift, create_graph=True)
    fbar_t = torch.as_tensor(np.asarray(fbar, dtype=np.float64))
    target = float(ebar) * out["E"] + (out["F"] * fbar_t).sum()
    grads = torch.autograd.grad(target, [linear, radial, shift], allow_unused=True)
    grads = [torch.zeros_like(p) if g is None else g for g, p in zip(grads, [linear, radial, shift])]
    return tuple(g.detach().numpy() for g in grads)


# ----------------------------------------------------------------------------- sampled atoms


def sampled_site_values(model, struct, centres):
    """Neighbour rows, E_i and B_i for selected centres of a large structure."""
    rows = _nb.neighbor_rows(struct.pos, struct.cell, model.r_cut, centres)
    js = np.concatenate([r[0] for r in rows])
    ns = np.concatenate([r[1] for r in rows])
    ci = np.repeat(np.arange(len(centres)), [len(r[0]) for r in rows])
    gi = np.asarray(centres)[ci]
    d = torch.as_tensor(_nb.displacements(struct.pos, struct.cell, gi, js, ns))
    z = torch.as_tensor(struct.species.astype(np.int64))
    zc = z[torch.as_tensor(np.asarray(centres, dtype=np.int64))]
    e, b = site_quantities(model, d, torch.as_tensor(ci), zc, z[torch.as_tensor(js)], len(centres))
    return rows, e.detach().numpy(), b.detach().numpy()


def sampled_forces(model, struct, atoms):
    """F_k for a few atoms k of a large structure, from the site energies of k and of
    every atom that has k as a neighbour (the neighbour relation is symmetric)."""
    out = []
    for k in atoms:
        (row,) = _nb.neighbor_rows(struct.pos, struct.cell, model.r_cut, [k])
        owners = sorted(set([int(k)] + [int(x) for x in row[0]]))
        rows = _nb.neighbor_rows(struct.pos, struct.cell, model.r_cut, owners)
        js = np.concatenate([r[0] for r in rows])
        ns = np.concatenate([r[1] for r in rows])
        ci = np.repeat(np.arange(len(owners)), [len(r[0]) for r in rows])
        gi = np.asarray(owners)[ci]
        d = torch.as_tensor(_nb.displacements(struct.pos, struct.cell, gi, js, ns))
        d.requires_grad_(True)
        z = torch.as_tensor(struct.species.astype(np.int64))
        zc = z[torch.as_tensor(np.asarray(owners, dtype=np.int64))]
        e, _ = site_quantities(model, d, torch.as_tensor(ci), zc, z[torch.as_tensor(js)], len(owners))
        (g,) = torch.autograd.grad(e.sum(), d)
        g = g.numpy()
        fk = g[gi == k].sum(axis=0) - g[js == k].sum(axis=0)
        out.append(fk)
    return np.array(out)


def param_vjp_chunked(model, struct, ebar, fbar, nl=None, chunk=512):
    """The same vector-Jacobian product, accumulated over chunks of centre atoms.

    With D = sum_k fbar_k . dE/dR_k = sum_i sum_j g_ij . (fbar_j - fbar_i), where g_ij is the
    derivative of E_i by the pair displacement, ebar dE/dtheta + sum_k fbar_k . dF_k/dtheta =
    d/dtheta sum_i (ebar E_i - D_i), and each bracket depends only on centre i's pairs; so the
    chunks add up to the whole.  Used where the system is too large for one autograd graph.
    """
    if nl is None:
        nl = _nb.neighbor_csr(struct.pos, struct.cell, model.r_cut)
    fbar = np.asarray(fbar, dtype=np.float64)
    z = torch.as_tensor(struct.species.astype(np.int64))
    radial = model.radial.clone().requires_grad_(True)
    linear = model.linear.clone().requires_grad_(True)
    shift = model.shift.clone().requires_grad_(True)
    acc = [torch.zeros_like(linear), torch.zeros_like(radial), torch.zeros_like(shift)]
    off = nl["off"]
    n = struct.n_atoms
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        p0, p1 = int(off[c0]), int(off[c1])
        i = nl["i"][p0:p1]
        j = nl["j"][p0:p1]
        d = torch.as_tensor(_nb.displacements(struct.pos, struct.cell, i, j, nl["n"][p0:p1]))
        d.requires_grad_(True)
        ci = torch.as_tensor((i - c0).astype(np.int64))
        zc = z[c0:c1]
        e_i, _ = site_quantities(model, d, ci, zc, z[torch.as_tensor(j.astype(np.int64))], c1 - c0,
                                 radial, linear, shift)
        (g,) = torch.autograd.grad(e_i.sum(), d, create_graph=True)
        delta = torch.as_tensor(fbar[j] - fbar[i])
        target = float(ebar) * e_i.sum() - (g * delta).sum()
        grads = torch.autograd.grad(target, [linear, radial, shift], allow_unused=True)
        for a, gr in zip(acc, grads):
            if gr is not None:
                a += gr.detach()
    return tuple(a.numpy() for a in acc)
