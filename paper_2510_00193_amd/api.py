"""PyTorch-facing wrapper of libmtp.so.

PyTorch supplies device memory and the stream; every computation runs in the
library's HIP kernels.  Tensors passed in must already live on the GPU with
the documented dtypes (float64 positions, int32 species); nothing is
converted or computed on the host here besides argument packing.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import MtpNlist, MtpParams, MtpSystem, check


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, shape=None, name=""):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


@dataclass
class NeighborList:
    """Canonical CSR list (device int32 tensors).

    checked is True for a list returned by Potential.neighbors (the library uses it as is); a
    list assembled by the caller keeps the default False and is validated by the library on
    every use (one pass over the list and one synchronization).
    """

    off: torch.Tensor
    j: torch.Tensor
    shift: torch.Tensor
    rev: torch.Tensor
    checked: bool = False

    @property
    def n_pairs(self) -> int:
        return int(self.j.shape[0])

    def _c(self):
        for name in ("off", "j", "shift", "rev"):
            _dev(getattr(self, name), torch.int32, name=name)
        return MtpNlist(self.off.data_ptr(), self.j.data_ptr() if self.n_pairs else None,
                        self.shift.data_ptr() if self.n_pairs else None,
                        self.rev.data_ptr() if self.n_pairs else None, self.n_pairs, 1 if self.checked else 0)


def compiled_levels():
    lib = _lib.load()
    n = ctypes.c_int()
    buf = (ctypes.c_int * 64)()
    check(lib.mtp_levels(ctypes.byref(n), buf))
    return [buf[k] for k in range(n.value)]


LEVEL_INFO_KEYS = ("n_alpha", "n_mu", "n_moments", "n_components", "n_products", "max_nu", "n_groups")


def level_info(level):
    """Sizes of a compiled level (no GPU needed)."""
    lib = _lib.load()
    buf = (ctypes.c_int * len(LEVEL_INFO_KEYS))()
    check(lib.mtp_level_info(int(level), buf, len(LEVEL_INFO_KEYS)))
    return dict(zip(LEVEL_INFO_KEYS, list(buf)))


class Potential:
    """One MTP model on the current GPU."""

    def __init__(self, level, n_species, n_cheb, r_min, r_cut, radial, linear, shift, precision="fp64",
                 chunk_atoms=0, grade_select=0.0, grade_break=0.0, lanes_per_atom=0):
        self._lib = _lib.load()
        self._h = None
        radial = np.ascontiguousarray(radial, dtype=np.float64)
        linear = np.ascontiguousarray(linear, dtype=np.float64)
        shift = np.ascontiguousarray(shift, dtype=np.float64)
        prec = {"fp64": _lib.MTP_FP64, "fp32": _lib.MTP_FP32_MOMENTS}[precision]
        p = MtpParams(int(level), int(n_species), int(n_cheb), float(r_min), float(r_cut),
                      radial.ctypes.data_as(_lib.c_double_p), linear.ctypes.data_as(_lib.c_double_p),
                      shift.ctypes.data_as(_lib.c_double_p), prec, int(chunk_atoms), float(grade_select),
                      float(grade_break), int(lanes_per_atom))
        h = ctypes.c_void_p()
        check(self._lib.mtp_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self.level, self.n_species, self.n_cheb = int(level), int(n_species), int(n_cheb)
        self.r_min, self.r_cut = float(r_min), float(r_cut)
        a, mu, nm, nc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(self._lib.mtp_sizes(h, ctypes.byref(a), ctypes.byref(mu), ctypes.byref(nm), ctypes.byref(nc)))
        self.n_alpha, self.n_mu, self.n_moments, self.n_components = a.value, mu.value, nm.value, nc.value

    @classmethod
    def from_params(cls, p, **kw):
        return cls(p.level, p.n_species, p.n_cheb, p.r_min, p.r_cut, p.radial, p.linear, p.shift, **kw)

    def close(self):
        if self._h is not None:
            self._lib.mtp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ profiling
    def profile(self, enable=True):
        check(self._lib.mtp_profile(self._h, 1 if enable else 0))

    def profile_reset(self):
        check(self._lib.mtp_profile_reset(self._h))

    def profile_read(self):
        """{kernel class: (total ms, launches)} accumulated since the last reset (synchronizes)."""
        out = {}
        k = 0
        while True:
            name = ctypes.c_char_p()
            ms = ctypes.c_double()
            n = ctypes.c_longlong()
            code = self._lib.mtp_profile_read(self._h, k, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(n))
            if code != _lib.MTP_OK:
                break
            out[name.value.decode()] = (ms.value, n.value)
            k += 1
        return out

    # ------------------------------------------------------------------ helpers
    def _system(self, pos, species, cell):
        n = int(pos.shape[0])
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(species, torch.int32, (n,), "species")
        cell = np.ascontiguousarray(cell, dtype=np.float64).reshape(9)
        s = MtpSystem(n, pos.data_ptr() if n else None, species.data_ptr() if n else None,
                      (ctypes.c_double * 9)(*cell.tolist()))
        return s, n

    def set_params(self, radial=None, linear=None, shift=None):
        """Replace coefficients in place (device tensors, float64)."""
        args = []
        for t in (radial, linear, shift):
            args.append(_ptr(_dev(t, torch.float64, name="coefficients")) if t is not None else None)
        check(self._lib.mtp_set_params(self._h, *args, 1, _stream()))

    def neighbors(self, pos, species, cell, cap=None):
        sysc, n = self._system(pos, species, cell)
        dev = pos.device
        off = torch.empty(n + 1, dtype=torch.int32, device=dev)
        total = ctypes.c_longlong()
        if cap is None:
            check(self._lib.mtp_neighbors(self._h, ctypes.byref(sysc), _ptr(off), None, None, None, 0,
                                          ctypes.byref(total), _stream()), (_lib.MTP_OK, _lib.MTP_ERR_CAPACITY))
            cap = total.value
        j = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        sh = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        rev = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        check(self._lib.mtp_neighbors(self._h, ctypes.byref(sysc), _ptr(off), _ptr(j), _ptr(sh), _ptr(rev),
                                      int(cap), ctypes.byref(total), _stream()))
        p = total.value
        return NeighborList(off, j[:p], sh[:p], rev[:p], checked=True)

    def compute(self, pos, species, cell, nlist=None, forces=True, virial=True, e_atom=False):
        return self._compute(self._lib.mtp_compute, pos, species, cell, nlist, forces, virial, e_atom)

    def compute_static(self, pos, species, cell, nlist, forces=True, virial=True, e_atom=False):
        """compute() through mtp_compute_static: the library's fixed scratch area instead of its
        workspace (the caller's list is required; outputs are still allocated here by torch)."""
        if nlist is None:
            raise ValueError("compute_static needs a neighbour list")
        return self._compute(self._lib.mtp_compute_static, pos, species, cell, nlist, forces, virial, e_atom)

    def _compute(self, entry, pos, species, cell, nlist, forces, virial, e_atom):
        sysc, n = self._system(pos, species, cell)
        dev = pos.device
        e = torch.empty(1, dtype=torch.float64, device=dev)
        ea = torch.empty(n, dtype=torch.float64, device=dev) if e_atom else None
        f = torch.empty((n, 3), dtype=torch.float64, device=dev) if forces else None
        w = torch.empty(6, dtype=torch.float64, device=dev) if virial else None
        nl = ctypes.byref(nlist._c()) if nlist is not None else None
        check(entry(self._h, ctypes.byref(sysc), nl, _ptr(e), _ptr(ea), _ptr(f), _ptr(w), _stream()))
        out = {"energy": e[0]}
        if forces:
            out["forces"] = f
        if virial:
            out["virial"] = w
        if e_atom:
            out["e_atom"] = ea
        return out

    def grade(self, pos, species, cell, ainv, nlist=None, mode="fp64"):
        sysc, n = self._system(pos, species, cell)
        dev = pos.device
        _dev(ainv, torch.float64, (self.n_alpha, self.n_alpha), "ainv")
        g = torch.empty(n, dtype=torch.float64, device=dev)
        gm = torch.empty(1, dtype=torch.float64, device=dev)
        md = {"fp64": _lib.MTP_GRADE_FP64, "fp32split": _lib.MTP_GRADE_FP32SPLIT}[mode]
        nl = ctypes.byref(nlist._c()) if nlist is not None else None
        code = check(self._lib.mtp_grade(self._h, ctypes.byref(sysc), nl, _ptr(ainv), md, _ptr(g), _ptr(gm),
                                         _stream()),
                     (_lib.MTP_OK, _lib.MTP_GRADE_SELECT, _lib.MTP_GRADE_BREAK))
        return {"grade": g, "grade_max": gm[0], "status": code}

    def grade_config(self, pos, species, cell, ainv, nlist=None):
        """Configuration-mode grade: {'grade': max_k |(sum_i B_i) Ainv|_k (device scalar),
        'descriptor': sum_i B_i [n_alpha], 'status'}."""
        sysc, n = self._system(pos, species, cell)
        dev = pos.device
        _dev(ainv, torch.float64, (self.n_alpha, self.n_alpha), "ainv")
        g = torch.empty(1, dtype=torch.float64, device=dev)
        desc = torch.empty(self.n_alpha, dtype=torch.float64, device=dev)
        nl = ctypes.byref(nlist._c()) if nlist is not None else None
        code = check(self._lib.mtp_grade_config(self._h, ctypes.byref(sysc), nl, _ptr(ainv), _ptr(desc), _ptr(g),
                                                _stream()),
                     (_lib.MTP_OK, _lib.MTP_GRADE_SELECT, _lib.MTP_GRADE_BREAK))
        return {"grade": g[0], "descriptor": desc, "status": code}

    def maxvol(self, cand, active, ainv, tol=1e-3, max_swaps=100):
        """MaxVol active-set update in place (device float64 tensors cand [m][n], active [n][n],
        ainv [n][n]); returns the list of swaps (i, k, g)."""
        n = int(active.shape[0])
        m = int(cand.shape[0])
        _dev(cand, torch.float64, (m, n), "cand")
        _dev(active, torch.float64, (n, n), "active")
        _dev(ainv, torch.float64, (n, n), "ainv")
        sw = (ctypes.c_int * max(2 * max_swaps, 1))()
        gr = (ctypes.c_double * max(max_swaps, 1))()
        ns = ctypes.c_int()
        check(self._lib.mtp_maxvol(self._h, _ptr(cand), m, n, _ptr(active), _ptr(ainv), float(tol), int(max_swaps),
                                   sw, gr, ctypes.byref(ns), _stream()))
        return [(sw[2 * t], sw[2 * t + 1], gr[t]) for t in range(ns.value)]

    def param_grad(self, pos, species, cell, ebar, fbar, nlist=None):
        sysc, n = self._system(pos, species, cell)
        dev = pos.device
        _dev(fbar, torch.float64, (n, 3), "fbar")
        dl = torch.empty(self.n_alpha, dtype=torch.float64, device=dev)
        dr = torch.empty((self.n_species, self.n_species, self.n_mu, self.n_cheb), dtype=torch.float64, device=dev)
        ds = torch.empty(self.n_species, dtype=torch.float64, device=dev)
        nl = ctypes.byref(nlist._c()) if nlist is not None else None
        check(self._lib.mtp_param_grad(self._h, ctypes.byref(sysc), nl, float(ebar), _ptr(fbar), _ptr(dl),
                                       _ptr(dr), _ptr(ds), _stream()))
        return dl, dr, ds


class Batch:
    """Many small periodic configurations evaluated together (training sets).

    positions [N, 3] float64 and species [N] int32 live on the GPU and are referenced by the
    library for the batch's lifetime (this object keeps them alive); atom_off [n_cfg + 1]
    and cells [n_cfg, 3, 3] are host arrays.  The neighbour lists are built once here.
    """

    def __init__(self, pot: Potential, atom_off, pos, species, cells):
        self._lib = pot._lib
        self._pot = pot
        self._h = None
        n = int(pos.shape[0])
        _dev(pos, torch.float64, (n, 3), "pos")
        _dev(species, torch.int32, (n,), "species")
        self.atom_off = np.ascontiguousarray(atom_off, dtype=np.int32)
        self.cells = np.ascontiguousarray(cells, dtype=np.float64).reshape(-1, 9)
        self.n_cfg = int(self.cells.shape[0])
        if self.atom_off.shape != (self.n_cfg + 1,):
            raise ValueError("atom_off must have n_cfg + 1 entries")
        self.pos, self.species = pos, species
        h = ctypes.c_void_p()
        off_c = self.atom_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        check(self._lib.mtp_batch_create(pot._h, self.n_cfg, off_c, _ptr(pos), _ptr(species),
                                         self.cells.ctypes.data_as(_lib.c_double_p), ctypes.byref(h), _stream()))
        self._h = h
        self.n_atoms = n
        self.n_alpha, self.n_mu = pot.n_alpha, pot.n_mu

    def close(self):
        if self._h is not None:
            self._lib.mtp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self):
        n, p, so, ch, pe = ctypes.c_int(), ctypes.c_longlong(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(self._lib.mtp_batch_sizes(self._h, ctypes.byref(n), ctypes.byref(p), ctypes.byref(so), ctypes.byref(ch),
                                        ctypes.byref(pe)))
        return {"n_atoms": n.value, "n_pairs": p.value, "sorted": so.value, "chunk_atoms": ch.value,
                "persistent": pe.value}

    def schedule(self, sorted=False, chunk_atoms=0, persistent=False):
        check(self._lib.mtp_batch_schedule(self._h, 1 if sorted else 0, int(chunk_atoms), 1 if persistent else 0))

    def tune(self, cache_path=None):
        choice = (ctypes.c_int * 3)()
        path = cache_path.encode() if cache_path else None
        check(self._lib.mtp_batch_tune(self._h, path, choice, _stream()))
        return {"sorted": choice[0], "chunk_atoms": choice[1], "persistent": choice[2]}

    def vjp(self, ebar, fbar, use_graph=False):
        """sum_c ebar_c dE_c/dtheta + sum_i fbar_i . dF_i/dtheta for device cotangents ebar [n_cfg]
        and fbar [N, 3]: (d_linear, d_radial, d_shift) as new device tensors."""
        _dev(ebar, torch.float64, (self.n_cfg,), "ebar")
        _dev(fbar, torch.float64, (self.n_atoms, 3), "fbar")
        p = self._pot
        dev = self.pos.device
        if getattr(self, "_vjp_out", None) is None or not use_graph:
            self._vjp_out = (torch.empty(p.n_alpha, dtype=torch.float64, device=dev),
                             torch.empty((p.n_species, p.n_species, p.n_mu, p.n_cheb), dtype=torch.float64,
                                         device=dev),
                             torch.empty(p.n_species, dtype=torch.float64, device=dev))
        dl, dr, ds = self._vjp_out
        check(self._lib.mtp_batch_vjp(self._h, _ptr(ebar), _ptr(fbar), _ptr(dl), _ptr(dr), _ptr(ds),
                                      1 if use_graph else 0, _stream()))
        return (dl.clone(), dr.clone(), ds.clone()) if use_graph else (dl, dr, ds)

    def neighbors(self):
        ptrs = [ctypes.c_void_p() for _ in range(4)]
        check(self._lib.mtp_batch_neighbors(self._h, *[ctypes.byref(x) for x in ptrs]))
        return [p.value for p in ptrs]

    def outputs(self, loss=True):
        dev = self.pos.device
        out = {"energy": torch.empty(self.n_cfg, dtype=torch.float64, device=dev),
               "forces": torch.empty((self.n_atoms, 3), dtype=torch.float64, device=dev),
               "virial": torch.empty((self.n_cfg, 6), dtype=torch.float64, device=dev)}
        if loss:
            p = self._pot
            out.update({"loss": torch.empty(1, dtype=torch.float64, device=dev),
                        "d_linear": torch.empty(p.n_alpha, dtype=torch.float64, device=dev),
                        "d_radial": torch.empty((p.n_species, p.n_species, p.n_mu, p.n_cheb), dtype=torch.float64,
                                                device=dev),
                        "d_shift": torch.empty(p.n_species, dtype=torch.float64, device=dev)})
        return out

    def run(self, out, e_target=None, f_target=None, use_graph=False):
        """Fill the preallocated dict from outputs(); with targets also the loss gradient."""
        if (e_target is None) != (f_target is None):
            raise ValueError("give both targets or neither")
        if e_target is not None:
            _dev(e_target, torch.float64, (self.n_cfg,), "e_target")
            _dev(f_target, torch.float64, (self.n_atoms, 3), "f_target")
        g = lambda k: _ptr(out[k]) if k in out else None  # noqa: E731
        check(self._lib.mtp_batch_run(self._h, _ptr(e_target), _ptr(f_target), g("energy"), g("forces"),
                                      g("virial"), g("loss"), g("d_linear"), g("d_radial"), g("d_shift"),
                                      1 if use_graph else 0, _stream()))
        return out
