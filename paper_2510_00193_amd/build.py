"""Build libmtp.so for gfx950: generate the per-level programs, compile with hipcc, link.

Usage: python -m paper_2510_00193_amd.build [--levels 10,16] [--jobs 8]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "gen")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmtp.so")
INCLUDE = os.path.join(ROOT, "include")

# level -> moment-entry groups of the lane-per-atom kernels (register budget): a count of
# equal ranges, or a tuple of interior boundaries of the flat moment layout
LEVELS = {2: 1, 4: 1, 6: 1, 8: 1, 10: 1, 12: 1, 14: 1, 16: 1, 18: 2, 20: 3}
if os.environ.get("MTP_GROUPS_L16"):
    LEVELS[16] = tuple(int(x) for x in os.environ["MTP_GROUPS_L16"].split(","))
# levels that also get the binary32-moment chain
FP32_LEVELS = {2, 4, 6, 8, 10, 12, 14, 16}
DEFAULT_LEVELS = (2, 4, 6, 8, 10, 12, 14, 16, 20)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=on",
    # no packed fp32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _write_if_changed(path, text):
    if os.path.exists(path):
        with open(path) as fh:
            if fh.read() == text:
                return
    with open(path, "w") as fh:
        fh.write(text)


def _unit(lv, body):
    return (f'// Generated: part of level {lv}.\n#include "mtp_device.h"\n#include "gen/mtp_L{lv}.inc"\n'
            f'#include "mtp_level_impl.h"\n{body}\n')


def _ngroups(lv):
    g = LEVELS[lv]
    return len(g) + 1 if isinstance(g, tuple) else g


def _nrtparts(lv):
    """Number of reverse-tangent parts of a generated level (read from its program header)."""
    with open(os.path.join(GEN, f"mtp_L{lv}.inc")) as fh:
        for line in fh:
            if "static constexpr int NRTPART" in line:
                return int(line.split("=")[1].strip().rstrip(";"))
    raise RuntimeError(f"level {lv}: no NRTPART in the generated program")


def _assembly(lv):
    """Translation unit that assembles the launcher table of one level."""
    fp32 = lv in FP32_LEVELS
    lines = ['#include "mtp_device.h"', f'#include "gen/mtp_L{lv}.inc"', '#include "mtp_internal.h"',
             "namespace mtp {", f"ChainOps chain_ops_{lv}_f64();", f"ChainOps chain_ops_{lv}_b64();"]
    if fp32:
        lines.append(f"ChainOps chain_ops_{lv}_f32();")
    lines.append(f"AdjOps adj_ops_{lv}();")
    lines.append(f"void adj_fwd_{lv}(const SysArgs&, const double*, const double*, long, int, int, const double*, "
                 "double, double*, double*, hipStream_t);")
    for g in range(_nrtparts(lv)):
        lines.append(f"void adj_rev_{lv}_{g}(const double*, const double*, long, int, const double*, "
                     "const double*, double*, hipStream_t);")
    lines += [f"LevelOps level_ops_{lv}() {{", "  LevelOps o{};", f"  using L = Lv{lv};",
              "  o.level = L::LEVEL; o.nmom = L::NMOM; o.ncomp = L::NCOMP; o.nalpha = L::NALPHA;",
              "  o.nmu = L::NMU; o.maxnu = L::MAXNU; o.ngroup = L::NGROUP; o.triples = L::TRIPLES;",
              f"  o.chain[0] = chain_ops_{lv}_f64();", f"  o.chain[2] = chain_ops_{lv}_b64();"]
    if fp32:
        lines.append(f"  o.chain[1] = chain_ops_{lv}_f32();")
    lines.append(f"  o.adj = adj_ops_{lv}();")
    lines.append(f"  o.adj.tan_forward = &adj_fwd_{lv};")
    for g in range(_nrtparts(lv)):
        lines.append(f"  o.adj.tan_reverse[{g}] = &adj_rev_{lv}_{g};")
    lines += ["  return o;", "}", "}  // namespace mtp", ""]
    return f"// Generated: launcher table of level {lv}.\n" + "\n".join(lines)


def level_units(lv):
    """(file name, text) of the translation units of one level."""
    units = [(f"mtp_L{lv}.hip", _assembly(lv)),
             (f"mtp_L{lv}_f64.hip", _unit(lv, f"MTP_DEFINE_CHAIN(Lv{lv}, {lv}, double, false, f64)")),
             (f"mtp_L{lv}_b64.hip", _unit(lv, f"MTP_DEFINE_CHAIN(Lv{lv}, {lv}, double, true, b64)")),
             (f"mtp_L{lv}_adj.hip", _unit(lv, f"MTP_DEFINE_ADJ(Lv{lv}, {lv})")),
             (f"mtp_L{lv}_tfw.hip", _unit(lv, f"MTP_DEFINE_ADJ_FWD(Lv{lv}, {lv})"))]
    for g in range(_nrtparts(lv)):
        units.append((f"mtp_L{lv}_rev{g}.hip", _unit(lv, f"MTP_DEFINE_ADJ_REV(Lv{lv}, {lv}, {g})")))
    if lv in FP32_LEVELS:
        units.append((f"mtp_L{lv}_f32.hip", _unit(lv, f"MTP_DEFINE_CHAIN(Lv{lv}, {lv}, float, false, f32)")))
    return units


def generate(levels):
    from .codegen.emit import write_level
    os.makedirs(GEN, exist_ok=True)
    for lv in levels:
        write_level(lv, GEN, LEVELS[lv])
        units = level_units(lv)
        for name, text in units:
            _write_if_changed(os.path.join(GEN, name), text)
        # reverse-tangent units of an earlier, finer cut of the program
        keep = {name for name, _ in units}
        for name in os.listdir(GEN):
            if name.startswith(f"mtp_L{lv}_rev") and name.endswith(".hip") and name not in keep:
                os.remove(os.path.join(GEN, name))
    _write_if_changed(os.path.join(GEN, "levels.inc"),
                      "".join(f"MTP_LEVEL({lv})\n" for lv in levels))


def _compile(src, obj):
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj, time.time() - t0


def sources(levels):
    out = [os.path.join(CSRC, f) for f in ("mtp_api.cpp", "mtp_batch.cpp", "mtp_nbr.hip", "mtp_common.hip",
                                           "mtp_grade.hip", "mtp_static.hip", "mtp_maxvol.hip")]
    for lv in levels:
        out += [os.path.join(GEN, name) for name, _ in level_units(lv)]
    return out


def _level_of(src):
    """Level number of a generated level unit (mtp_L16_f64.hip -> 16), else None."""
    base = os.path.basename(src)
    if not base.startswith("mtp_L"):
        return None
    return int(base[5:].split(".")[0].split("_")[0])


def _work_estimate(src):
    lv = _level_of(src)
    inc = os.path.join(GEN, f"mtp_L{lv}.inc") if lv is not None else None
    return os.path.getsize(inc) if inc and os.path.exists(inc) else 0


def _deps_mtime(src):
    """Newest mtime among a source, the shared headers and (for a level unit) its program."""
    paths = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    paths.append(os.path.join(INCLUDE, "mtp.h"))
    base = os.path.basename(src)
    lv = _level_of(src)
    if lv is not None:
        paths.append(os.path.join(GEN, f"mtp_L{lv}.inc"))
    if base == "mtp_api.cpp":
        paths.append(os.path.join(GEN, "levels.inc"))
    return max(os.path.getmtime(p) for p in paths if os.path.exists(p))


def build(levels=DEFAULT_LEVELS, jobs=None, verbose=True, incremental=False):
    """Compile every source (incremental=True skips objects newer than their inputs)."""
    levels = tuple(sorted(levels))
    generate(levels)
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(sources(levels), key=lambda p: -_work_estimate(p))  # big level units first
    jobs = jobs or min(8, os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {}
        for src in srcs:
            obj = os.path.join(OBJ, os.path.basename(src) + ".o")
            if incremental and os.path.exists(obj) and os.path.getmtime(obj) >= _deps_mtime(src):
                objs.append(obj)
                continue
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            futs[ex.submit(_compile_lang, src, obj, lang)] = src
        for fut in cf.as_completed(futs):
            obj, dt = fut.result()
            objs.append(obj)
            if verbose:
                print(f"  compiled {os.path.basename(futs[fut])} in {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *sorted(objs)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    shutil.move(tmp, LIB)
    if verbose:
        print(f"  linked {LIB}", flush=True)
    return LIB


def _compile_lang(src, obj, lang):
    cmd = [HIPCC, *FLAGS, *lang, "-c", src, "-o", obj]
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout[-4000:]}\n{res.stderr[-8000:]}")
    return obj, time.time() - t0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", default=",".join(str(l) for l in DEFAULT_LEVELS))
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true", help="reuse objects newer than their inputs")
    args = ap.parse_args(argv)
    levels = [int(x) for x in args.levels.split(",") if x]
    build(levels, args.jobs, incremental=args.incremental)


if __name__ == "__main__":
    sys.exit(main())
