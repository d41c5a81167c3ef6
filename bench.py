#!/usr/bin/env python3
"""Benchmark of the CRK-SPH pair passes and short-range gravity on one MI355X.

One step = one pass of the hot path over one synthetic particle set already
resident in HBM: for the CRK workloads the position packing, the volume pass,
the corrections pass (40 moments + FP64 solve), the fused acceleration /
energy pass with FP64 totals, and the backward (force, moments and volume
adjoints, with the moments recomputed); for the gravity workload one
short-range gravity evaluation.  The tree and the neighbour lists are built
once before the timed region (reported separately as build time); particles
are held in tree order.  The launch/tiling choices are autotuned first.

The default run measures the CRK step on C2 (the headline line) and then the
gravity step on its own workload (C3, gas + dark matter), reported in the same
JSON line under ``sr_gravity``; ``--config`` runs one workload alone.

Prints ONE JSON line.  ``value`` is pair interactions per second: ordered
pairs j != i inside each pass's radius (2h_i for volume and moments,
max(2h_i, 2h_j) for forces, r_c for gravity), counted exactly in FP64 on the
device, summed over the passes of a step, divided by the step time.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CRK-SPH pair interactions/s & % FP32 VALU peak; fwd+bwd ms vs FP64 GPU form"

# Algorithmic FP32 work per ordered pair inside the pass radius (FMA = 2 FLOP,
# square root / reciprocal square root = 1), per-particle constants hoisted;
# compensation arithmetic excluded.
FLOP_PER_PAIR = {"volume": 21, "moments": 112, "accel": 141, "gravity": 19,
                 "accel_adj": 520, "moments_adj": 365, "volume_adj": 40}
HYDRO_KERNELS = ("volume", "moments", "accel", "accel_adj", "moments_adj", "volume_adj")
PEAK_FP32_VALU_TFLOPS = 157.3  # 256 CUs x 2.4 GHz x 256 FLOP/clk/CU

WORKLOADS = {
    "C2": "128^3 clustered gas (lognormal, P(k)~k^-2, sigma_ln=1), h for 64+-8 neighbours, "
          "leaf 128; FP32 pairs + compensated sums, FP64 solve/totals",
    "C5": "256^3 clustered gas, 32..256 neighbours over a 16x density contrast; FP32 mixed",
    "C3": "128^3 gas + 128^3 dark matter, Plummer-softened short-range gravity, r_c = 3 spacing, "
          "uneven RCB leaves 16..512; FP32 + compensated sums",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(step, steps, warmup, torch):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def sampled(run, k0, n, budget_s):
    """Time run(k) on a sample of k targets sized to take about budget_s seconds
    (one small warm-up call first: library load and thread start-up)."""
    run(min(8, k0))
    k = k0
    dt, inter = run(k)
    for _ in range(3):
        if dt >= budget_s / 2 or k >= n:
            break
        k = int(min(k * budget_s / max(dt, 1e-3), n))
        dt, inter = run(k)
    return k, dt, inter


def cpu_baseline_hydro(cfg, budget_s):
    """The oracle (brute-force FP64 passes) on a sample of target particles of the workload."""
    import numpy as np

    import oracle
    import synth

    n = cfg["n"]
    # Brute force costs the same whatever the field values; the pass inputs the
    # sample needs for all particles (V, rho, corrections) are placeholders.
    V = np.full(n, 1.0 / n)
    rho = cfg["m"] / V
    corr = (np.ones(n), np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3, 3)))

    def run(k):
        t = synth.sample_targets(n, k, seed=123)
        t0 = time.perf_counter()
        oracle.volume(cfg, t)
        oracle.corrections(cfg, V, t)
        oracle.accel(cfg, V, rho, corr, t)
        dt = time.perf_counter() - t0
        inter = 2 * oracle.count_pairs(cfg, 0, t)[0] + oracle.count_pairs(cfg, 1, t)[0]
        return dt, inter

    k, dt, inter = sampled(run, 64, n, budget_s)
    return {"value": inter / dt, "unit": "interactions/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{k} sampled particles of the {n}-particle workload through the oracle's "
                      f"brute-force volume, corrections and accel/energy passes (each scans all "
                      f"{n} particles per target); {dt:.1f} s"}


def cpu_baseline_gravity(cfg, budget_s):
    import oracle
    import synth

    n = cfg["n"]

    def run(k):
        t = synth.sample_targets(n, k, seed=123)
        t0 = time.perf_counter()
        oracle.gravity(cfg, t)
        dt = time.perf_counter() - t0
        return dt, oracle.count_pairs(cfg, 2, t, r_fixed=cfg["r_cut"])[0]

    k, dt, inter = sampled(run, 256, n, budget_s)
    return {"value": inter / dt, "unit": "interactions/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{k} sampled particles of the {n}-particle workload through the oracle's "
                      f"brute-force gravity (all {n} particles scanned per target); {dt:.1f} s"}


# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs, calibrated
# against a device copy of known size (profiles/*_hbm_traffic.json, written by
# paper_2310_16122_amd.profiling); used only while the kernel sources are the
# ones the counters were taken on.
TRAFFIC_FILES = {"C2": "crk_passes_C2_hbm_traffic.json", "C5": "crk_passes_C5_hbm_traffic.json",
                 "C3": "sr_gravity_C3_hbm_traffic.json"}
PROFILE_NAMES = {k: f"void k_{k}<float>" for k in ("volume", "moments", "accel", "accel_adj",
                                                   "moments_adj", "volume_adj", "gravity")}


def measured_counters(config, kind):
    """The kernel's counter readings from the committed profile, or None when
    there is none or the kernel sources changed since it was taken."""
    from paper_2310_16122_amd import profiling

    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES.get(config, ""))
    if not os.path.isfile(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_digest") != profiling.source_digest():
        return None  # kernels changed since the counters were taken
    # the FP32 instantiation (template arguments after the precision allowed)
    name = PROFILE_NAMES[kind]
    hits = [v for k, v in rec["kernels"].items() if k == name or k.startswith(name[:-1] + ",")]
    return max(hits, key=lambda v: v.get("dispatches", 0)) if hits else None


def roofline(kind, ms_total, launches, units, config):
    avg_ms = ms_total / max(launches, 1)
    achieved = FLOP_PER_PAIR[kind] * units / (avg_ms * 1e-3) / 1e12
    k = measured_counters(config, kind)
    out = {"bound": "alu", "kernel": kind, "achieved": round(achieved, 3),
           "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
           "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 4),
           "traffic": None if k is None else round(k["hbm_bytes"]),
           "avg_launch_ms": round(avg_ms, 4), "flop_per_unit": FLOP_PER_PAIR[kind],
           "units_per_launch": units}
    if k is not None and "SQ_INSTS_VALU_FLOPS_FP32" in k:
        # executed FP32 FLOP (counter: per wave instruction, FMA = 2; x 64 lanes),
        # padding, compensation and masked lanes included
        ex = 64.0 * k["SQ_INSTS_VALU_FLOPS_FP32"] / (avg_ms * 1e-3) / 1e12
        out["executed_counter"] = round(ex, 3)
        out["executed_frac"] = round(ex / PEAK_FP32_VALU_TFLOPS, 4)
    return out


def bench_hydro(args, torch, crk):
    import numpy as np

    import synth

    t0 = time.perf_counter()
    cfg = synth.make_config(args.config)
    log(f"[bench] generated {args.config}: n={cfg['n']} in {time.perf_counter() - t0:.1f}s")
    # Particles are kept in tree order, as a simulation keeps them: build once
    # on the generated (random) order, reorder the arrays along the tree and
    # rebuild, which gives the identity permutation (coalesced particle I/O).
    g_rand = crk.gas_to_device(cfg, "f32")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    L_rand = crk.crk_build_leaf_pairs(g_rand["x"], g_rand["y"], g_rand["z"], g_rand["h"],
                                      leaf_max=args.leaf_max, prec="f32")
    build_ms = (time.perf_counter() - tb) * 1e3
    cull = L_rand.kernel_times()["cull"]
    perm = L_rand.perm().cpu().numpy()
    cfg_t = {k: (v[perm] if isinstance(v, np.ndarray) and v.shape == (cfg["n"],) else v)
             for k, v in cfg.items()}
    g32 = crk.gas_to_device(cfg_t, "f32")
    L = crk.crk_build_leaf_pairs(g32["x"], g32["y"], g32["z"], g32["h"], leaf_max=args.leaf_max,
                                 prec="f32")
    identity = bool((L.perm().cpu().numpy() == np.arange(cfg["n"])).all())
    if args.tuning:
        L.set_tuning(**json.loads(args.tuning))
        L_rand.set_tuning(**json.loads(args.tuning))
    st = L.stats()
    G, F = st["pairs_gather"], st["pairs_force"]
    log(f"[bench] build {build_ms:.0f} ms (list build on GPU {cull[0]:.2f} ms); identity order "
        f"after rebuild: {identity}; stats {st}")
    inter_fwd = 2 * G + F
    inter = inter_fwd + (G + 3 * F if not args.no_backward else 0)
    dev = g32["x"].device

    def adjoints(g, prec):
        dt = torch.float32 if prec == "f32" else torch.float64
        w = torch.as_tensor(cfg_t["w"]).to(dt).to(dev)
        c = torch.as_tensor(cfg_t["c"]).to(dt).to(dev)
        o = crk.forward(L, g, cfg["gamma"], prec)
        return (2.0 * w[:, None] * o["a"]).contiguous(), c

    def make_step(Lh, g, prec, ga, gdu):
        # the forward keeps its per-particle moment sums for the backward
        # (30 doubles per particle); pair terms are recomputed, never stored
        def step():
            o = crk.forward(Lh, g, cfg["gamma"], prec, store_sums=not args.no_backward)
            if not args.no_backward:
                crk.crk_accel_energy_backward(Lh, g, o["V"], o["rho"],
                                              (o["A"], o["B"], o["dA"], o["dB"], o["M"]),
                                              ga, gdu, cfg["gamma"], prec)
        return step

    ga32, gdu32 = adjoints(g32, "f32")
    step32 = make_step(L, g32, "f32", ga32, gdu32)
    tuned = None
    if not args.no_autotune and not args.tuning:
        from paper_2310_16122_amd import tune

        best, best_ms, tried = tune.autotune(L, step32, repeats=2)
        L_rand.set_tuning(**best)
        tuned = {"tried": len(tried), "best_ms": round(best_ms, 3)}
        log(f"[bench] autotuned over {len(tried)} settings: {best} ({best_ms:.3f} ms)")
    L.timing(False)
    timed_steps(step32, 2, args.warmup, torch)
    L.timing(True)
    ms32 = timed_steps(step32, args.steps, 0, torch)
    kt = L.kernel_times()
    L.timing(False)
    log(f"[bench] f32 step {ms32:.3f} ms; kernels {kt}")
    units = {"volume": G, "moments": G, "accel": F, "accel_adj": F, "moments_adj": F, "volume_adj": F}
    ran = [k for k in HYDRO_KERNELS if kt[k][1] > 0]
    dom = max(ran, key=lambda k: kt[k][0])
    rl = roofline(dom, kt[dom][0], kt[dom][1], units[dom], args.config)
    per_kernel = {k: {"avg_ms": round(kt[k][0] / kt[k][1], 4), "launches_per_step": kt[k][1] / args.steps,
                      "tflops": round(FLOP_PER_PAIR[k] * units[k] / (kt[k][0] / kt[k][1]) * 1e-9, 3)}
                  for k in ran}
    per_kernel["pack_ms_per_step"] = round(kt["pack"][0] / args.steps, 4)
    per_kernel["solve_adj_ms_per_step"] = round(kt["solve_adj"][0] / args.steps, 4)
    flop_step = sum(FLOP_PER_PAIR[k] * units[k] * kt[k][1] / args.steps for k in ran)

    # the same step with particle arrays in the generated (random) order
    ms_rand = None
    if not args.no_random_order:
        inv = torch.as_tensor(np.argsort(perm)).to(dev)  # tree position of each generated particle
        ms_rand = timed_steps(make_step(L_rand, g_rand, "f32", ga32[inv].contiguous(),
                                        gdu32[inv].contiguous()), max(2, args.steps // 4), 1, torch)
        log(f"[bench] f32 step, random particle order: {ms_rand:.3f} ms")

    ms64 = None
    acc = None
    if not args.no_f64:
        g64 = crk.gas_to_device(cfg_t, "f64")
        ga64, gdu64 = adjoints(g64, "f64")
        ms64 = timed_steps(make_step(L, g64, "f64", ga64, gdu64), max(2, args.steps // 4), 1, torch)
        log(f"[bench] f64 step {ms64:.3f} ms")
        # the FP32 mixed path against the FP64 GPU form, every particle, per output
        o32 = crk.forward(L, g32, cfg["gamma"], "f32")
        o64 = crk.forward(L, g64, cfg["gamma"], "f64")
        acc = {}
        for k in ("V", "rho", "A", "B", "dA", "dB", "a", "dudt"):
            d = (o32[k].double() - o64[k]).abs().max().item()
            acc[k] = float(f"{d / o64[k].abs().max().item():.3e}")
        log(f"[bench] FP32 vs FP64 normwise errors {acc}")
        del g64, o32, o64

    out = {
        "metric": METRIC, "value": inter / (ms32 * 1e-3), "unit": "interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms32, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "n": cfg["n"],
                   "leaf_max": args.leaf_max,
                   "passes": "volume+corrections+accel_energy" +
                             ("" if args.no_backward else "+backward(accel,moments,volume adjoints)"),
                   "particle_order": "tree order (identity permutation)" if identity else "tree-built",
                   "interactions_per_step": inter, "pairs_gather": G, "pairs_force": F,
                   "list_entries": st["list_entries"], "tuning": L.get_tuning(), "autotune": tuned},
        "roofline": rl,
        "kernels": per_kernel,
        "fp32_frac_step": round(flop_step / (ms32 * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS, 4),
        "fp64_gpu_ms_per_step": None if ms64 is None else round(ms64, 4),
        "fp64_over_fp32_time": None if ms64 is None else round(ms64 / ms32, 3),
        "fp32_vs_fp64_normwise": acc,
        "random_order_ms_per_step": None if ms_rand is None else round(ms_rand, 4),
        "build_ms": round(build_ms, 1), "list_build_gpu_ms": round(cull[0], 3),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_hydro(cfg, args.cpu_budget)
    return out


def bench_gravity(args, torch, crk):
    import synth

    import numpy as np

    cfg = synth.make_config("C3")
    log(f"[bench] generated C3: n={cfg['n']}")
    x, y, z = (torch.as_tensor(cfg[k]).cuda() for k in ("x", "y", "z"))

    def build(leaf_max, xx, yy, zz):
        return crk.crk_build_leaf_pairs(xx, yy, zz, None, r_fixed=cfg["r_cut"], leaf_max=leaf_max,
                                        leaf_min=16, split_extent=cfg["r_cut"], prec="f32")

    # particles in tree order (as a simulation holds them): build, reorder, rebuild
    tb = time.perf_counter()
    L0 = build(512, x, y, z)
    build_ms = (time.perf_counter() - tb) * 1e3
    perm = L0.perm().long()
    L0.free()
    x, y, z = x[perm].contiguous(), y[perm].contiguous(), z[perm].contiguous()
    m = torch.as_tensor(cfg["m"]).float().cuda()[perm].contiguous()

    def make_step(Lh):
        def step():
            crk.sr_gravity(Lh, x, y, z, m, cfg["G"], cfg["eps"], cfg["r_cut"], prec="f32")
        return step

    tuned = None
    if args.tuning or args.no_autotune:
        L = build(args.leaf_max if args.leaf_max != 128 else 512, x, y, z)
        if args.tuning:
            L.set_tuning(**json.loads(args.tuning))
    else:
        from paper_2310_16122_amd import tune

        leaf, L, tun, best_ms, per_leaf = tune.autotune_leaf_size(
            lambda lm: build(lm, x, y, z), make_step, leaf_values=(128, 256, 512), log=log, repeats=2)
        tuned = {"leaf_max": leaf, "ms_by_leaf": {str(k): round(v, 3) for k, v in per_leaf.items()},
                 "best_ms": round(best_ms, 3)}
        log(f"[bench] autotuned gravity: leaf {leaf}, {tun} ({best_ms:.3f} ms)")
    st = L.stats()
    step = make_step(L)

    timed_steps(step, 2, args.warmup, torch)
    L.timing(True)
    ms = timed_steps(step, args.steps, 0, torch)
    kt = L.kernel_times()
    inter = st["pairs_force"]
    out = {
        "metric": METRIC, "value": inter / (ms * 1e-3), "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"C3: {WORKLOADS['C3']}", "n": cfg["n"],
                   "interactions_per_step": inter, "candidate_pairs": st["candidate_pairs"],
                   "leaves": st["leaves"], "particle_order": "tree order",
                   "tuning": L.get_tuning(), "autotune": tuned},
        "roofline": roofline("gravity", kt["gravity"][0], kt["gravity"][1], inter, "C3"),
        "build_ms": round(build_ms, 1),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_gravity(cfg, args.cpu_budget)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C2", choices=("C2", "C5", "C3"))
    ap.add_argument("--leaf-max", type=int, default=128)
    ap.add_argument("--tuning", default=None, help="JSON dict of crk_tuning fields")
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default tuning")
    ap.add_argument("--no-gravity", action="store_true", help="C2 only: skip the gravity workload")
    ap.add_argument("--no-random-order", action="store_true",
                    help="skip the comparison step on randomly ordered particle arrays")
    ap.add_argument("--gravity-tuning", default=None, help="JSON crk_tuning for the gravity workload")
    ap.add_argument("--gravity-leaf-max", type=int, default=512,
                    help="gravity leaf size when its tuning is given")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-backward", action="store_true", help="forward passes only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy a buffer of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path "
              "(the passes would shard by spatial domain with halo exchange; not built)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2310_16122_amd as crk

    crk.load_library()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.config == "C3":
        out = bench_gravity(args, torch, crk)
    else:
        out = bench_hydro(args, torch, crk)
        if args.config == "C2" and not args.no_gravity:
            # the gravity pass on its own workload, in the same JSON line
            import gc

            gc.collect()
            torch.cuda.empty_cache()
            gargs = argparse.Namespace(**vars(args))
            gargs.config, gargs.tuning, gargs.leaf_max = "C3", args.gravity_tuning, args.gravity_leaf_max
            out["sr_gravity"] = bench_gravity(gargs, torch, crk)
    if args.calibrate_copy:
        # a plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counter
        # readings calibrate the counters of the pair kernels
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = nbytes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
