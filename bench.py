"""Benchmark of the MTP hot path on one MI355X.

One step = one pass of the hot path over the 1,024,000-atom level-16 bcc
workload: canonical neighbour-list rebuild, then energy, forces and virial
(float64).  Prints one JSON line.  Extra fields report the evaluation on a
prebuilt list, per-kernel times and the roofline of the dominant kernel.

  python bench.py [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64 (256 CUs x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
METRIC = "atom-steps/s (E+F+virial) at 1M atoms; batched param-grad configs/s vs plain"


def flop_model(info, n_cheb):
    """Algorithmic flops per unit of each kernel class (FMA = 2), from the model tables."""
    C, nmu, T, nalpha, maxnu = (info["n_moments"], info["n_mu"], info["n_products"], info["n_alpha"],
                                info["max_nu"])
    mono = (maxnu + 1) * (maxnu + 2) * (maxnu + 3) // 6 - 1
    return {
        "moments": ("pair", 3 * n_cheb + 2 * nmu * n_cheb + mono + 2 * C),
        "program_forward": ("atom", 3 * T + 2 * nalpha),
        "program_reverse": ("atom", 6 * T),
        "program": ("atom", 9 * T + 2 * nalpha),   # forward + reverse fused
        "pair_backward": ("pair", 6 * n_cheb + 2 * nmu * n_cheb + 8 * C + 10 * nmu + 22),
    }


# sources that determine the per-atom kernels; counters taken on other sources are stale
KERNEL_SOURCES = ("paper_2510_00193_amd/codegen", "paper_2510_00193_amd/csrc/mtp_level_impl.h",
                  "paper_2510_00193_amd/csrc/mtp_device.h", "paper_2510_00193_amd/csrc/mtp_internal.h",
                  "paper_2510_00193_amd/build.py")
TRAFFIC_FILE = os.path.join("profiles", "hbm_traffic_bcc80_L16.md")


def kernel_source_hash():
    h = hashlib.sha256()
    files = []
    for rel in KERNEL_SOURCES:
        path = os.path.join(ROOT, rel)
        if os.path.isdir(path):
            files += sorted(os.path.join(rel, f) for f in os.listdir(path) if f.endswith(".py"))
        else:
            files.append(rel)
    for rel in files:
        h.update(rel.encode())
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_class, n_atoms):
    """HBM bytes per launch of a kernel class from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by the copy-kernel calibration), or None when the summary is missing,
    was taken on another workload size, or the kernel sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    meta = dict(re.findall(r"^- (\w+): (\S+)", text, re.M))
    if meta.get("source_hash") != kernel_source_hash() or meta.get("atoms") != str(n_atoms):
        return None
    for row in re.findall(r"^\| `?(\w+)`? \|(.*)$", text, re.M):
        if row[0] == kernel_class:
            cells = [c.strip() for c in row[1].split("|")]
            return float(cells[2]) * 1e6   # column "total MB per launch"
    return None


def _cpu_model():
    """CPU model name of the host (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(params, target_s=10.0, single_s=8.0):
    """The oracle on a bounded sample of the same workload: 10x10x10 bcc cells (2000 atoms)
    drawn with the same recipe, neighbour list + E + F + virial, repeated to ~target_s with
    all host threads, then to ~single_s with one thread."""
    import torch
    from oracle import mtp as om
    from oracle import neighbors as onb
    rng = np.random.default_rng(3)
    sites, cell = wl.bcc_sites(10, 10, 10, 3.16)
    pos = wl.jitter_wrap(sites, cell, 0.1, rng)
    s = wl.Structure(pos, np.zeros(len(pos), np.int32), cell)
    model = om.Model.from_params(params)

    def run(budget):
        reps, t0 = 0, time.perf_counter()
        while True:
            nl = onb.neighbor_csr(s.pos, s.cell, params.r_cut)
            om.energy_forces_virial(model, s, nl)
            reps += 1
            if time.perf_counter() - t0 >= budget:
                break
        return reps, time.perf_counter() - t0

    threads = torch.get_num_threads()
    reps, dt = run(target_s)
    torch.set_num_threads(1)
    try:
        reps1, dt1 = run(single_s)
    finally:
        torch.set_num_threads(threads)
    return {"value": s.n_atoms * reps / dt, "unit": "atom-steps/s", "cores": threads,
            "kind": "oracle", "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "one_thread": {"value": s.n_atoms * reps1 / dt1, "unit": "atom-steps/s", "cores": 1,
                           "sample": f"{reps1} x the same step, {dt1:.1f} s"},
            "sample": f"{reps} x (neighbour list + E/F/virial) of a 2000-atom 10x10x10 bcc cell, "
                      f"same recipe and level-16 coefficients, {dt:.1f} s with {threads} threads"}


def _timeit(fn, steps, warmup=1):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def section_fp32(s, params, pos, sp, ref, steps):
    """FP32-moment form on the same workload: rate, and error against the float64 path."""
    import torch
    from paper_2510_00193_amd import Potential
    pot = Potential.from_params(params, precision="fp32")
    nl = pot.neighbors(pos, sp, s.cell)
    dt_eval = _timeit(lambda: pot.compute(pos, sp, s.cell, nlist=nl), steps)
    pot.profile(True)
    pot.profile_reset()
    dt_full = _timeit(lambda: pot.compute(pos, sp, s.cell), steps, warmup=0)
    prof = pot.profile_read()
    pot.profile(False)
    out = pot.compute(pos, sp, s.cell, nlist=nl)
    torch.cuda.synchronize()

    def rel(a, b):
        a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
        return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))

    return {"value": s.n_atoms / dt_full, "unit": "atom-steps/s", "ms_per_step": dt_full * 1e3,
            "eval_only_atom_steps_per_s": s.n_atoms / dt_eval,
            "kernels_ms_per_step": {k: v[0] / steps for k, v in prof.items() if v[1]},
            "rel_err_vs_fp64": {"E": rel(out["energy"].reshape(1), ref["energy"].reshape(1)),
                                "F": rel(out["forces"], ref["forces"]), "W": rel(out["virial"], ref["virial"])}}


def section_grade(steps):
    """Neighbourhood grade on the 250,000-atom fcc workload (prebuilt list), FP64 and FP32-split,
    and the configuration-mode grade of the same configuration."""
    import torch
    from paper_2510_00193_amd import Potential, level_info
    info = level_info(16)
    w = wl.workload(4, info["n_alpha"], info["n_mu"])
    (s,) = w["structures"]
    pot = Potential.from_params(w["params"])
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    ainv = torch.as_tensor(w["extra"]["active_set_inv"], device="cuda")
    nl = pot.neighbors(pos, sp, s.cell)
    out = {}
    for mode in ("fp64", "fp32split"):
        pot.grade(pos, sp, s.cell, ainv, nlist=nl, mode=mode)
        pot.profile(True)
        pot.profile_reset()
        dt = _timeit(lambda: pot.grade(pos, sp, s.cell, ainv, nlist=nl, mode=mode), steps, warmup=0)
        prof = pot.profile_read()
        pot.profile(False)
        ms, launches = prof["grade_gemm"]
        flops = 2.0 * info["n_alpha"] ** 2 * s.n_atoms  # B . Ainv per evaluation
        gemm_tf = flops / (ms * 1e-3 / steps) / 1e12
        peak = 78.6 if mode == "fp64" else 157.3
        out[mode] = {"value": s.n_atoms / dt, "unit": "atom-steps/s", "ms_per_step": dt * 1e3,
                     "gemm_ms_per_step": ms / steps, "gemm_tflops": gemm_tf,
                     "gemm_roofline": {"bound": "mfma", "achieved": gemm_tf, "peak": peak, "unit": "TFLOP/s",
                                       "frac": gemm_tf / peak}}
    g64 = pot.grade(pos, sp, s.cell, ainv, nlist=nl, mode="fp64")["grade"]
    g32 = pot.grade(pos, sp, s.cell, ainv, nlist=nl, mode="fp32split")["grade"]
    torch.cuda.synchronize()
    out["fp32split"]["rel_err_vs_fp64"] = float(((g32 - g64).abs() / g64.clamp(min=1.0)).max().cpu())
    # configuration mode on the same configuration: descriptor sum_i B_i, then one product
    pot.grade_config(pos, sp, s.cell, ainv, nlist=nl)
    dt = _timeit(lambda: pot.grade_config(pos, sp, s.cell, ainv, nlist=nl), steps, warmup=0)
    out["config_mode"] = {"value": s.n_atoms / dt, "unit": "atom-steps/s", "ms_per_step": dt * 1e3}
    out["workload"] = f"fcc-50x50x25-3sp-L16: {s.n_atoms} atoms, n_alpha {info['n_alpha']}"
    return out


def section_adjoint(steps):
    """Parameter VJP on the 16,000-atom two-species workload (prebuilt list)."""
    import torch
    from paper_2510_00193_amd import Potential, level_info
    info = level_info(16)
    w = wl.workload(2, info["n_alpha"], info["n_mu"])
    (s,) = w["structures"]
    pot = Potential.from_params(w["params"])
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    fbar = torch.as_tensor(np.random.default_rng(2).normal(size=(s.n_atoms, 3)), device="cuda")
    nl = pot.neighbors(pos, sp, s.cell)
    dt = _timeit(lambda: pot.param_grad(pos, sp, s.cell, 0.5, fbar, nlist=nl), steps)
    dt_e = _timeit(lambda: pot.compute(pos, sp, s.cell, nlist=nl), steps)
    return {"value": s.n_atoms / dt, "unit": "atom-steps/s", "ms_per_step": dt * 1e3,
            "eval_ms_per_step": dt_e * 1e3,
            "workload": f"bcc-20x20x20-2sp-L16: {s.n_atoms} atoms, VJP of (E, F) w.r.t. xi, c, s"}


def section_small(reps=200):
    """Small systems: latency of one E/F/virial evaluation of the 128-atom level-10 workload
    (prebuilt list, synchronized per call; also as a captured graph of the allocation-free
    entry point, replayed), and the throughput of the 16,000-atom level-16
    two-species workload (prebuilt list) with the library's lanes-per-atom choice and with each
    setting forced."""
    import torch
    from paper_2510_00193_amd import Potential, level_info
    out = {}
    info = level_info(10)
    w = wl.workload(1, info["n_alpha"], info["n_mu"])
    (s,) = w["structures"]
    pot = Potential.from_params(w["params"])
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    nl = pot.neighbors(pos, sp, s.cell)
    for _ in range(10):
        pot.compute(pos, sp, s.cell, nlist=nl)
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        t0 = time.perf_counter()
        pot.compute(pos, sp, s.cell, nlist=nl)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    dt = _timeit(lambda: pot.compute(pos, sp, s.cell, nlist=nl), reps)
    out["bcc-4x4x4-L10"] = {"atoms": s.n_atoms, "latency_us_median": float(np.median(lat) * 1e6),
                            "latency_us_best": float(np.min(lat) * 1e6),
                            "pipelined_us_per_eval": dt * 1e6}
    # the same evaluation captured once (the allocation-free entry point) and replayed; a
    # failure here is reported in the line instead of ending the run
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            pot.compute_static(pos, sp, s.cell, nl)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            pot.compute_static(pos, sp, s.cell, nl)
        for _ in range(10):
            graph.replay()
        torch.cuda.synchronize()
        glat = []
        for _ in range(reps):
            t0 = time.perf_counter()
            graph.replay()
            torch.cuda.synchronize()
            glat.append(time.perf_counter() - t0)
        out["bcc-4x4x4-L10"]["graph_replay_latency_us_median"] = float(np.median(glat) * 1e6)
    except Exception as exc:  # noqa: BLE001
        out["bcc-4x4x4-L10"]["graph_replay_error"] = str(exc)[:200]
    info = level_info(16)
    w = wl.workload(2, info["n_alpha"], info["n_mu"])
    (s,) = w["structures"]
    pos = torch.as_tensor(s.pos, device="cuda")
    sp = torch.as_tensor(s.species, device="cuda")
    rates = {}
    for lanes in (0, 1, 2, 4, 8):  # 0: the library's choice for this size
        pot = Potential.from_params(w["params"], lanes_per_atom=lanes)
        nl = pot.neighbors(pos, sp, s.cell)
        dt = _timeit(lambda: pot.compute(pos, sp, s.cell, nlist=nl), 50, warmup=5)
        rates[lanes] = dt
    dt = rates[0]
    out["bcc-20x20x20-2sp-L16"] = {"atoms": s.n_atoms, "ms_per_eval": dt * 1e3,
                                   "value": s.n_atoms / dt, "unit": "atom-steps/s",
                                   "ms_per_eval_by_lanes_per_atom": {str(k): v * 1e3 for k, v in rates.items()
                                                                     if k}}
    return out


def section_batch(steps, plain_sample=128):
    """4096 triclinic configurations at level 20: batched forward + loss gradient (tuned
    schedule, graph replay) against plain per-configuration launches."""
    import torch
    from paper_2510_00193_amd import Batch, Potential, level_info
    info = level_info(20)
    t0 = time.perf_counter()
    w = wl.workload(5, info["n_alpha"], info["n_mu"])
    t_gen = time.perf_counter() - t0
    structs, params = w["structures"], w["params"]
    off, pos, species, cells = wl.batch_arrays(structs)
    pot = Potential.from_params(params)
    dpos = torch.as_tensor(pos, device="cuda")
    dsp = torch.as_tensor(species, device="cuda")
    rng = np.random.default_rng(55)
    e0_host = rng.normal(size=len(structs))
    e0 = torch.as_tensor(e0_host, device="cuda")
    f0 = torch.as_tensor(rng.normal(size=(len(pos), 3)), device="cuda")
    b = Batch(pot, off, dpos, dsp, cells)
    choice = b.tune()
    out = b.outputs()
    dt = _timeit(lambda: b.run(out, e0, f0, use_graph=True), steps)
    # plain: one configuration at a time through mtp_compute and mtp_param_grad, each with its
    # own model and a neighbour list built before the timed region; the forward of every
    # configuration is enqueued first, the energies come back in one synchronization (the VJP
    # takes the energy cotangent on the host), then every VJP is enqueued
    sample = structs[:plain_sample]
    plain = []
    for x in sample:
        p1 = Potential.from_params(params)
        ps = torch.as_tensor(x.pos, device="cuda")
        ss = torch.as_tensor(x.species, device="cuda")
        plain.append((p1, ps, ss, x.cell, p1.neighbors(ps, ss, x.cell)))
    torch.cuda.synchronize()

    def plain_pass():
        outs = [p1.compute(ps, ss, cell, nlist=nl) for (p1, ps, ss, cell, nl) in plain]
        energies = torch.stack([r["energy"] for r in outs]).cpu()
        for k, (p1, ps, ss, cell, nl) in enumerate(plain):
            fb = 2.0 * (outs[k]["forces"] - f0[off[k]:off[k + 1]])
            p1.param_grad(ps, ss, cell, 2.0 * float(energies[k] - e0_host[k]), fb.contiguous(), nlist=nl)

    dt_plain = _timeit(plain_pass, 1)
    # flops by the model: forward and backward of every pair and atom, and the parameter
    # adjoint estimated at 2.5 times that work (its tangent passes over the same program)
    fm = flop_model(info, params.n_cheb)
    n_pairs = b.sizes()["n_pairs"]
    fwd_bwd = n_pairs * (fm["moments"][1] + fm["pair_backward"][1]) + int(off[-1]) * fm["program"][1]
    model = 3.5 * fwd_bwd
    flops = {"forward_backward_gflop": fwd_bwd / 1e9, "with_adjoint_gflop": model / 1e9,
             "tflops": model / dt / 1e12, "frac_fp64": model / dt / 1e12 / PEAK_FP64_TFLOPS,
             "adjoint_model": "2.5 x forward + backward"}
    return {"value": len(structs) / dt, "unit": "configs/s", "ms_per_step": dt * 1e3, "flop_model": flops,
            "atoms": int(off[-1]), "pairs": b.sizes()["n_pairs"], "schedule": choice,
            "plain": {"value": len(sample) / dt_plain, "unit": "configs/s", "sample_configs": len(sample),
                      "method": "mtp_compute + mtp_param_grad per configuration, prebuilt lists, one host "
                                "synchronization per pass"},
            "speedup_vs_plain": (len(structs) / dt) / (len(sample) / dt_plain),
            "generation_s": t_gen,
            "workload": "4096 triclinic cells, N ~ U{8..256}, 3 species, level 20, n_cheb 10, r_cut 5.5: "
                        "forward E/F/virial + loss gradient w.r.t. xi, c, s per step"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--rep", type=int, default=80, help="bcc repeat (80 -> 1,024,000 atoms)")
    ap.add_argument("--sections", default="fp32,grade,adjoint,small,batch",
                    help="extra sections after the headline (comma list, or 'none')")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        return 2

    import torch
    from paper_2510_00193_amd import Potential, level_info

    level = 16
    info = level_info(level)
    w = wl.workload(3, info["n_alpha"], info["n_mu"], small={"rep": (args.rep,) * 3})
    (s,) = w["structures"]
    params = w["params"]
    n = s.n_atoms
    dev = torch.device("cuda:0")
    pos = torch.as_tensor(s.pos, device=dev)
    sp = torch.as_tensor(s.species, device=dev)
    pot = Potential.from_params(params)
    print(f"# workload bcc {args.rep}^3 x2 = {n} atoms, level {level}", file=sys.stderr, flush=True)

    def step():
        return pot.compute(pos, sp, s.cell)

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    pot.profile(True)
    pot.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = pot.profile_read()
    pot.profile(False)
    ms_step = dt * 1e3 / args.steps
    value = n * args.steps / dt
    print(f"# full step {ms_step:.3f} ms", file=sys.stderr, flush=True)

    # evaluation on a prebuilt list (the list is reused, as between rebuilds in MD)
    nl = pot.neighbors(pos, sp, s.cell)
    torch.cuda.synchronize()
    n_pairs = nl.n_pairs
    for _ in range(2):
        ref64 = pot.compute(pos, sp, s.cell, nlist=nl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pot.compute(pos, sp, s.cell, nlist=nl)
    torch.cuda.synchronize()
    dt_eval = time.perf_counter() - t0
    eval_rate = n * args.steps / dt_eval

    # roofline of the dominant compute kernel (algorithmic flops / average launch time)
    fm = flop_model(info, params.n_cheb)
    kernels = {}
    for name, (ms, launches) in prof.items():
        if launches:
            kernels[name] = {"avg_ms": ms / launches, "launches_per_step": launches / args.steps,
                             "ms_per_step": ms / args.steps}
    dom = max((k for k in kernels if k in fm), key=lambda k: kernels[k]["ms_per_step"])
    unit, per_unit = fm[dom]
    units_per_step = n_pairs if unit == "pair" else n
    flops_per_launch = per_unit * units_per_step / kernels[dom]["launches_per_step"]
    achieved = flops_per_launch / (kernels[dom]["avg_ms"] * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(dom, n), "kernel": dom,
                "flops_per_unit": per_unit, "unit_of_work": unit, "launch_avg_ms": kernels[dom]["avg_ms"]}
    # algorithmic flops of one evaluation: the kernel classes that ran
    total_flops = sum(fm[k][1] * (n_pairs if fm[k][0] == "pair" else n) for k in fm if k in kernels)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"bcc-{args.rep}x{args.rep}x{args.rep}-L16: {n} atoms, level 16, 1 species, "
                               "8 Chebyshev functions, r_cut 5.0; step = neighbour rebuild + E/F/virial",
                   "atoms": n, "pairs": n_pairs, "level": level},
        "roofline": roofline,
        "eval_only": {"value": eval_rate, "unit": "atom-steps/s", "ms_per_step": dt_eval * 1e3 / args.steps,
                      "flops_per_step": total_flops,
                      "fp64_tflops": total_flops / (dt_eval / args.steps) / 1e12},
        "kernels": kernels,
    }
    sections = [x for x in args.sections.split(",") if x and x != "none"]
    if "fp32" in sections:
        print("# section fp32", file=sys.stderr, flush=True)
        out["fp32_form"] = section_fp32(s, params, pos, sp, ref64, args.steps)
    del nl, ref64
    if "grade" in sections:
        print("# section grade", file=sys.stderr, flush=True)
        out["grade"] = section_grade(max(3, args.steps // 2))
    if "adjoint" in sections:
        print("# section adjoint", file=sys.stderr, flush=True)
        out["adjoint"] = section_adjoint(args.steps)
    if "small" in sections:
        print("# section small", file=sys.stderr, flush=True)
        out["small_systems"] = section_small()
    if "batch" in sections:
        print("# section batch", file=sys.stderr, flush=True)
        out["batch"] = section_batch(max(3, args.steps // 2))
    if not args.no_cpu:
        print("# cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(params)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
