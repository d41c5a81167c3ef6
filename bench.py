#!/usr/bin/env python3
"""Benchmark of the CRK-SPH pair passes (and short-range gravity) on one MI355X.

One step = one pass of the hot path over one synthetic particle set already
resident in HBM: for the CRK workloads the position packing, the volume pass,
the corrections pass (40 moments + FP64 solve) and the fused acceleration /
energy pass with FP64 totals; for the gravity workload one short-range
gravity evaluation.  The tree and the neighbour lists are built once before
the timed region (reported separately as build time).

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
# compensation arithmetic excluded.  Derivation in the design doc.
FLOP_PER_PAIR = {"volume": 21, "moments": 112, "accel": 141, "gravity": 19}
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

    k = 64
    dt, inter = run(k)
    if dt < budget_s / 4:
        k = int(min(k * budget_s / max(dt, 1e-3), n))
        dt, inter = run(k)
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

    k = 256
    dt, inter = run(k)
    if dt < budget_s / 4:
        k = int(min(k * budget_s / max(dt, 1e-3), n))
        dt, inter = run(k)
    return {"value": inter / dt, "unit": "interactions/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{k} sampled particles of the {n}-particle workload through the oracle's "
                      f"brute-force gravity (all {n} particles scanned per target); {dt:.1f} s"}


def roofline(kind, ms_total, launches, units):
    avg_ms = ms_total / max(launches, 1)
    achieved = FLOP_PER_PAIR[kind] * units / (avg_ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": kind, "achieved": round(achieved, 3),
            "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 4), "traffic": None,
            "avg_launch_ms": round(avg_ms, 4), "flop_per_unit": FLOP_PER_PAIR[kind],
            "units_per_launch": units}


def bench_hydro(args, torch, crk):
    import synth

    t0 = time.perf_counter()
    cfg = synth.make_config(args.config)
    log(f"[bench] generated {args.config}: n={cfg['n']} in {time.perf_counter() - t0:.1f}s")
    g32 = crk.gas_to_device(cfg, "f32")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    L = crk.crk_build_leaf_pairs(g32["x"], g32["y"], g32["z"], g32["h"], leaf_max=args.leaf_max,
                                 prec="f32")
    build_ms = (time.perf_counter() - tb) * 1e3
    if args.tuning:
        L.set_tuning(**json.loads(args.tuning))
    cull = L.kernel_times()["cull"]
    st = L.stats()
    log(f"[bench] build {build_ms:.0f} ms (list build on GPU {cull[0]:.2f} ms); stats {st}")
    inter = 2 * st["pairs_gather"] + st["pairs_force"]

    def step32():
        crk.forward(L, g32, cfg["gamma"], "f32")

    L.timing(False)
    ms32 = timed_steps(step32, 2, args.warmup, torch)  # warm-up outside the timed region
    L.timing(True)
    ms32 = timed_steps(step32, args.steps, 0, torch)
    kt = L.kernel_times()
    log(f"[bench] f32 step {ms32:.3f} ms; kernels {kt}")
    units = {"volume": st["pairs_gather"], "moments": st["pairs_gather"], "accel": st["pairs_force"]}
    dom = max(("volume", "moments", "accel"), key=lambda k: kt[k][0])
    rl = roofline(dom, kt[dom][0], kt[dom][1], units[dom])
    per_kernel = {k: {"avg_ms": round(kt[k][0] / max(kt[k][1], 1), 4),
                      "tflops": round(FLOP_PER_PAIR[k] * units[k] / (kt[k][0] / max(kt[k][1], 1)) * 1e-9, 3)}
                  for k in ("volume", "moments", "accel")}
    per_kernel["pack_ms_per_step"] = round(kt["pack"][0] / args.steps, 4)

    ms64 = None
    if not args.no_f64:
        g64 = crk.gas_to_device(cfg, "f64")

        def step64():
            crk.forward(L, g64, cfg["gamma"], "f64")

        L.timing(False)
        ms64 = timed_steps(step64, max(2, args.steps // 4), 1, torch)
        log(f"[bench] f64 step {ms64:.3f} ms")
        del g64

    out = {
        "metric": METRIC, "value": inter / (ms32 * 1e-3), "unit": "interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms32, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "n": cfg["n"],
                   "leaf_max": args.leaf_max, "passes": "pack+volume+corrections+accel_energy",
                   "interactions_per_step": inter, "pairs_gather": st["pairs_gather"],
                   "pairs_force": st["pairs_force"], "list_entries": st["list_entries"],
                   "tuning": L.get_tuning()},
        "roofline": rl,
        "kernels": per_kernel,
        "fp32_frac_step": round(sum(FLOP_PER_PAIR[k] * units[k] for k in units) /
                                (ms32 * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS, 4),
        "fp64_gpu_ms_per_step": None if ms64 is None else round(ms64, 4),
        "fp64_over_fp32_time": None if ms64 is None else round(ms64 / ms32, 3),
        "build_ms": round(build_ms, 1), "list_build_gpu_ms": round(cull[0], 3),
        "backward": "not built yet",
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_hydro(cfg, args.cpu_budget)
    return out


def bench_gravity(args, torch, crk):
    import synth

    cfg = synth.make_config("C3")
    x, y, z = (torch.as_tensor(cfg[k]).cuda() for k in ("x", "y", "z"))
    m = torch.as_tensor(cfg["m"]).float().cuda()
    tb = time.perf_counter()
    L = crk.crk_build_leaf_pairs(x, y, z, None, r_fixed=cfg["r_cut"], leaf_max=512, leaf_min=16,
                                 split_extent=cfg["r_cut"], prec="f32")
    build_ms = (time.perf_counter() - tb) * 1e3
    if args.tuning:
        L.set_tuning(**json.loads(args.tuning))
    st = L.stats()

    def step():
        crk.sr_gravity(L, x, y, z, m, cfg["G"], cfg["eps"], cfg["r_cut"], prec="f32")

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
                   "tuning": L.get_tuning()},
        "roofline": roofline("gravity", kt["gravity"][0], kt["gravity"][1], inter),
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
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
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
    out = bench_gravity(args, torch, crk) if args.config == "C3" else bench_hydro(args, torch, crk)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
