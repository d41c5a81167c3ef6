#!/usr/bin/env python3
"""Benchmark of the CRK-SPH pair passes and short-range gravity on one MI355X.

One step = one pass of the hot path over one synthetic particle set already
resident in HBM: for the CRK workloads the position packing, the volume pass,
the corrections pass (40 moments + FP64 solve; the moment sums are kept for
the backward), the fused acceleration / energy pass with FP64 totals, and the
backward (force adjoint, the solve adjoint from the stored sums, moments and
volume adjoints); for the gravity workload one short-range gravity
evaluation.  The tree and the neighbour lists are built once before the timed
region (reported separately as build time); particles are held in tree order.
The launch/tiling choices are autotuned first.

The default run measures the CRK step on the 128^3 clustered gas (the
headline line), then the same step on the 256^3 gas with 32-256 neighbours
(``c5``: FP32 against the FP64 form, forward and backward) and the gravity
step on 128^3 gas + 128^3 dark matter (``sr_gravity``), in one JSON line;
``--config`` runs one workload alone.

``value`` is pair interactions per second: the ordered pairs j != i inside the
radius of every pair pass the step launches (2h_i for volume and moments,
max(2h_i, 2h_j) for the force pass and the three adjoint pair passes, r_c for
gravity), counted exactly in FP64 on the device, summed over the launches of a
step and divided by the step time.
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
HYDRO_KERNELS = ("volume", "moments", "accel", "accel_adj", "moments_adj", "volume_adj")
PEAK_FP32_VALU_TFLOPS = 157.3  # 256 CUs x 2.4 GHz x 256 FLOP/clk/CU

# FLOP per ordered pair of every pass, counted by the oracle on its own per-pair
# code (oracle/flop_table.py writes the file; a CPU test keeps it current).
FLOP_TABLE = os.path.join(ROOT, "oracle", "flop_per_pair.json")

WORKLOADS = {
    "C2": "128^3 clustered gas (lognormal, P(k)~k^-2, sigma_ln=1), h for 64+-8 neighbours, "
          "leaf 128; FP32 pairs + compensated sums, FP64 solve/totals",
    "C5": "256^3 clustered gas, 32..256 neighbours over a 16x density contrast, leaf 128; FP32 mixed",
    "C3": "128^3 gas + 128^3 dark matter, Plummer-softened short-range gravity, r_c = 3 spacing, "
          "uneven RCB leaves 16..512; FP32 + compensated sums",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flop_table():
    with open(FLOP_TABLE) as f:
        return json.load(f)["flop_per_pair"]


def timed_steps(step, steps, warmup, torch):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


# ---------------------------------------------------------------- CPU baseline (the oracle)
def _csr(rows):
    import numpy as np

    off = np.zeros(len(rows) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.concatenate(rows).astype(np.int64) if rows else np.zeros(0, np.int64)
    return off, idx


def force_lists(cfg, targets):
    """Exact candidate lists of the targets: every j != i with |x_ij| <
    max(2h_i, 2h_j) (periodic), from k-d trees over particles binned by h, so
    that a dense target never scans the support of the sparsest particle.
    Input preparation for the CPU baseline (scipy), not timed."""
    import numpy as np
    from scipy.spatial import cKDTree

    P = np.stack([cfg["x"], cfg["y"], cfg["z"]], 1)
    H = 2.0 * np.asarray(cfg["h"], dtype=np.float64)
    edges = np.exp2(np.arange(np.floor(np.log2(H.min())), np.ceil(np.log2(H.max())) + 0.26, 0.25))
    b = np.clip(np.searchsorted(edges, H, side="right") - 1, 0, len(edges) - 2)
    Pt, Ht = P[targets], H[targets]
    rows = [[] for _ in targets]
    for k in range(len(edges) - 1):
        sel = np.nonzero(b == k)[0]
        if sel.size == 0:
            continue
        tree = cKDTree(P[sel], boxsize=1.0)
        R = np.maximum(Ht, edges[k + 1])
        for t, c in enumerate(tree.query_ball_point(Pt, R, workers=-1)):
            if c:
                rows[t].append(sel[np.asarray(c)])
    out = []
    for t, i in enumerate(targets):
        c = np.concatenate(rows[t]) if rows[t] else np.zeros(0, np.int64)
        d = P[c] - P[i]
        d -= np.floor(d + 0.5)
        r = np.sqrt((d * d).sum(1))
        keep = (r < np.maximum(H[i], H[c])) & (c != i)
        out.append(np.sort(c[keep]))
    return out


def repeat_timed(fn, min_s):
    """Run fn until min_s seconds have passed (at least twice); seconds per call."""
    fn()
    t0 = time.perf_counter()
    k = 0
    while True:
        fn()
        k += 1
        dt = time.perf_counter() - t0
        if dt >= min_s and k >= 2:
            return dt / k


def cpu_baseline_hydro(cfg, budget_s, n_targets=16384):
    """The oracle's FP64 passes on the host cores: physics only (the three hydro
    passes of sampled targets over precomputed exact neighbour lists), on all
    threads and on one; and the brute-force form (every particle scanned per
    target) per pass, extrapolated to the whole workload."""
    import numpy as np

    import oracle
    import synth

    n = cfg["n"]
    t = synth.sample_targets(n, min(n_targets, n), seed=123)
    t0 = time.perf_counter()
    rows = force_lists(cfg, t)
    off, idx = _csr(rows)
    prep_s = time.perf_counter() - t0
    # V, rho and corrections of the neighbours are placeholders: the work per
    # pair does not depend on their values
    V = np.full(n, 1.0 / n)
    rho = cfg["m"] / V
    corr = (np.ones(n), np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3, 3)))
    F = int(off[-1])
    res = {}
    for label, threads, share in (("all", 0, 0.6), ("one", 1, 0.25)):
        nt = len(t) if threads == 0 else max(256, len(t) // 16)
        o2, i2 = off[:nt + 1], idx[:off[nt]]
        pairs = {}

        def run():
            pairs["g2"] = oracle.passes_listed(cfg, t[:nt], o2, i2, V, rho, corr, threads)[0]

        dt = repeat_timed(run, budget_s * share)
        res[label] = ((pairs["g2"] + int(o2[-1])) / dt, nt, dt)
    # brute force per pass on a few targets, extrapolated to all n particles
    tb = t[:32]
    bf = {}
    for name, fn in (("volume", lambda: oracle.volume(cfg, tb)),
                     ("corrections", lambda: oracle.corrections(cfg, V, tb)),
                     ("accel", lambda: oracle.accel(cfg, V, rho, corr, tb))):
        dt = repeat_timed(fn, budget_s * 0.05)
        bf[name] = round(dt / len(tb) * n, 1)
    rate, nt, dt = res["all"]
    return {"value": rate, "unit": "interactions/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{nt} sampled particles of the {n}-particle workload through the oracle's FP64 "
                      f"volume, corrections and accel/energy passes over exact precomputed neighbour "
                      f"lists ({F} force-list entries; the lists built by scipy k-d trees in "
                      f"{prep_s:.1f} s, not timed), repeated for {dt:.2f} s per pass set",
            "single_thread": {"value": res["one"][0], "targets": res["one"][1]},
            "brute_force_s_per_pass_extrapolated": bf,
            "brute_force_note": "brute-force oracle (every particle scanned per target) timed on 32 "
                                "targets per pass and scaled to all particles"}


def cpu_baseline_gravity(cfg, budget_s, n_targets=16384):
    import numpy as np
    from scipy.spatial import cKDTree

    import oracle
    import synth

    n = cfg["n"]
    t = synth.sample_targets(n, min(n_targets, n), seed=123)
    P = np.stack([cfg["x"], cfg["y"], cfg["z"]], 1)
    rows = [np.asarray(sorted(c), dtype=np.int64)
            for c in cKDTree(P, boxsize=1.0).query_ball_point(P[t], cfg["r_cut"], workers=-1)]
    off, idx = _csr(rows)
    inter = int(off[-1]) - len(t)  # every list holds the target itself
    res = {}
    for label, threads, share in (("all", 0, 0.6), ("one", 1, 0.3)):
        nt = len(t) if threads == 0 else max(256, len(t) // 16)
        o2, i2 = off[:nt + 1], idx[:off[nt]]
        dt = repeat_timed(lambda: oracle.gravity_listed(cfg, t[:nt], o2, i2, threads), budget_s * share)
        res[label] = ((int(o2[-1]) - nt) / dt, nt, dt)
    rate, nt, dt = res["all"]
    return {"value": rate, "unit": "interactions/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{nt} sampled particles of the {n}-particle workload through the oracle's FP64 "
                      f"gravity over precomputed candidate lists (r < r_c, {inter} pairs), repeated "
                      f"for {dt:.2f} s",
            "single_thread": {"value": res["one"][0], "targets": res["one"][1]}}


# ---------------------------------------------------------------- counters and roofline
# HBM traffic and executed FLOP per launch from rocprofv3 --pmc runs, calibrated
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


def profiled_setup(config):
    """(tuning, leaf size) the committed counter profile of `config` was taken
    with (from its command line), when it matches the current kernel sources;
    else None.  The timed launches then use it, so that the counters, the
    executed FLOP and the launch times in the roofline describe the same
    launches (the autotuner's own pick, within noise of it, is reported beside)."""
    import re

    from paper_2310_16122_amd import profiling

    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES.get(config, ""))
    if not os.path.isfile(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_digest") != profiling.source_digest():
        return None
    cmd = rec.get("command", "")
    flag, leaf_flag, leaf = (("--gravity-tuning", "--gravity-leaf-max", None) if config == "C3"
                             else ("--tuning", "--leaf-max", 128))
    m = re.search(re.escape(flag) + r" '(\{[^']*\})'", cmd)
    if not m:
        return None
    m2 = re.search(re.escape(leaf_flag) + r" (\d+)", cmd)
    if m2:
        leaf = int(m2.group(1))
    return json.loads(m.group(1)), leaf


def flop_per_unit(kind, units, config, table):
    """(FLOP per pair used for the algorithmic rate, oracle count, executed
    count per pair or None).  The algorithmic count is the oracle's, unless the
    kernel executes fewer FLOP per pair (counter, padding and compensation
    included): then the executed figure, so that the rate never claims work
    the kernel did not do."""
    ref = table["gravity" if kind == "gravity" else kind]
    k = measured_counters(config, kind)
    ex = None
    if k is not None and "SQ_INSTS_VALU_FLOPS_FP32" in k and units:
        ex = 64.0 * k["SQ_INSTS_VALU_FLOPS_FP32"] / units
    return (min(ref, ex) if ex is not None else ref), ref, ex


def roofline(kind, ms_total, launches, units, config, table):
    avg_ms = ms_total / max(launches, 1)
    flop, ref, ex = flop_per_unit(kind, units, config, table)
    achieved = flop * units / (avg_ms * 1e-3) / 1e12
    k = measured_counters(config, kind)
    out = {"bound": "alu", "kernel": kind, "achieved": round(achieved, 3),
           "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
           "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 4),
           "traffic": None if k is None else round(k["hbm_bytes"]),
           "avg_launch_ms": round(avg_ms, 4), "flop_per_unit": round(flop, 2),
           "flop_per_unit_oracle": ref,
           "flop_per_unit_executed": None if ex is None else round(ex, 2),
           "units_per_launch": units}
    if k is not None and "SQ_INSTS_VALU_FLOPS_FP32" in k:
        # executed FP32 FLOP (counter: per wave instruction, FMA = 2; x 64 lanes),
        # padding, compensation and masked lanes included
        exr = 64.0 * k["SQ_INSTS_VALU_FLOPS_FP32"] / (avg_ms * 1e-3) / 1e12
        out["executed_counter"] = round(exr, 3)
        out["executed_frac"] = round(exr / PEAK_FP32_VALU_TFLOPS, 4)
    return out


# ---------------------------------------------------------------- CRK step
def tree_ordered(crk, cfg, leaf_max, torch):
    """Particles in tree order, as a simulation keeps them: build once on the
    generated (random) order, reorder the arrays along the tree and rebuild,
    which gives the identity permutation (coalesced particle I/O).  Returns
    (cfg in tree order, handle, the generated order's handle, perm, build ms,
    list-build GPU ms, identity)."""
    import numpy as np

    g_rand = crk.gas_to_device(cfg, "f32")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    L_rand = crk.crk_build_leaf_pairs(g_rand["x"], g_rand["y"], g_rand["z"], g_rand["h"],
                                      leaf_max=leaf_max, prec="f32")
    build_ms = (time.perf_counter() - tb) * 1e3
    cull = L_rand.kernel_times()["cull"]
    perm = L_rand.perm().cpu().numpy()
    cfg_t = {k: (v[perm] if isinstance(v, np.ndarray) and v.shape == (cfg["n"],) else v)
             for k, v in cfg.items()}
    g32 = crk.gas_to_device(cfg_t, "f32")
    L = crk.crk_build_leaf_pairs(g32["x"], g32["y"], g32["z"], g32["h"], leaf_max=leaf_max, prec="f32")
    identity = bool((L.perm().cpu().numpy() == np.arange(cfg["n"])).all())
    return cfg_t, g32, L, L_rand, g_rand, perm, build_ms, cull, identity


def crk_step(crk, Lh, g, cfg, prec, ga, gdu, backward=True):
    """One step: forward with the moment sums kept, then the backward from them."""
    def step():
        o = crk.forward(Lh, g, cfg["gamma"], prec, store_sums=backward)
        if backward:
            crk.crk_accel_energy_backward(Lh, g, o["V"], o["rho"], (o["A"], o["B"], o["dA"], o["dB"], o["M"]),
                                          ga, gdu, cfg["gamma"], prec)
    return step


def upstream(crk, L, g, cfg_t, prec, torch):
    """dL/da = 2 w a and dL/d(du/dt) = c for L = sum w |a|^2 + sum c du/dt."""
    dt = torch.float32 if prec == "f32" else torch.float64
    dev = g["x"].device
    w = torch.as_tensor(cfg_t["w"]).to(dt).to(dev)
    c = torch.as_tensor(cfg_t["c"]).to(dt).to(dev)
    o = crk.forward(L, g, cfg_t["gamma"], prec)
    return (2.0 * w[:, None] * o["a"]).contiguous(), c


def interactions(kt, steps, G, F):
    """Ordered pairs per step summed over the pair kernels the step launched."""
    units = {"volume": G, "moments": G, "accel": F, "accel_adj": F, "moments_adj": F, "volume_adj": F}
    return sum(units[k] * kt[k][1] for k in HYDRO_KERNELS) // steps, units


def per_kernel_table(kt, steps, units, config, table):
    ran = [k for k in HYDRO_KERNELS if kt[k][1] > 0]
    out = {}
    for k in ran:
        avg = kt[k][0] / kt[k][1]
        flop, ref, ex = flop_per_unit(k, units[k], config, table)
        out[k] = {"avg_ms": round(avg, 4), "launches_per_step": kt[k][1] / steps,
                  "tflops": round(flop * units[k] / avg * 1e-9, 3),
                  "flop_per_pair": round(flop, 2), "flop_per_pair_oracle": ref,
                  "flop_per_pair_executed": None if ex is None else round(ex, 2)}
    out["pack_ms_per_step"] = round(kt["pack"][0] / steps, 4)
    out["solve_adj_ms_per_step"] = round(kt["solve_adj"][0] / steps, 4)
    return ran, out


def fp32_vs_fp64(crk, L, g32, g64, cfg_t, torch):
    """Normwise errors of the FP32 mixed path against the FP64 GPU form over
    every particle: forward outputs, and the backward's gradients for the
    benchmark loss."""
    acc = {}
    o32 = crk.forward(L, g32, cfg_t["gamma"], "f32", store_sums=True)
    o64 = crk.forward(L, g64, cfg_t["gamma"], "f64", store_sums=True)
    for k in ("V", "rho", "A", "B", "dA", "dB", "a", "dudt"):
        d = (o32[k].double() - o64[k]).abs().max().item()
        acc[k] = float(f"{d / o64[k].abs().max().item():.3e}")
    dev = g32["x"].device
    w = torch.as_tensor(cfg_t["w"]).to(dev)
    c = torch.as_tensor(cfg_t["c"]).to(dev)
    # the same upstream adjoints (from the FP64 forward) for both backward forms
    ga64 = (2.0 * w[:, None] * o64["a"]).contiguous()
    b64 = crk.crk_accel_energy_backward(L, g64, o64["V"], o64["rho"],
                                        (o64["A"], o64["B"], o64["dA"], o64["dB"], o64["M"]),
                                        ga64, c, cfg_t["gamma"], "f64")
    b32 = crk.crk_accel_energy_backward(L, g32, o32["V"], o32["rho"],
                                        (o32["A"], o32["B"], o32["dA"], o32["dB"], o32["M"]),
                                        ga64.float(), c.float(), cfg_t["gamma"], "f32")
    for k, u, v in zip(("gx", "gv", "gu"), b32, b64):
        d = (u.double() - v).abs().max().item()
        acc[k] = float(f"{d / v.abs().max().item():.3e}")
    del o32, o64, b32, b64
    return acc


def bench_hydro(args, torch, crk, config=None, tuning=None, autotune=True, random_order=True,
                f64=True, cpu=True):
    import numpy as np

    import synth

    config = config or args.config
    table = flop_table()
    t0 = time.perf_counter()
    cfg = synth.make_config(config)
    gen_s = time.perf_counter() - t0
    log(f"[bench] generated {config}: n={cfg['n']} in {gen_s:.1f}s")
    cfg_t, g32, L, L_rand, g_rand, perm, build_ms, cull, identity = tree_ordered(crk, cfg, args.leaf_max, torch)
    if tuning:
        L.set_tuning(**tuning)
        L_rand.set_tuning(**tuning)
    st = L.stats()
    G, F = st["pairs_gather"], st["pairs_force"]
    log(f"[bench] build {build_ms:.0f} ms (list build on GPU {cull[0]:.2f} ms); identity order "
        f"after rebuild: {identity}; stats {st}")
    backward = not args.no_backward
    ga32, gdu32 = upstream(crk, L, g32, cfg_t, "f32", torch)
    step32 = crk_step(crk, L, g32, cfg_t, "f32", ga32, gdu32, backward)
    tuned = None
    if autotune and not tuning:
        from paper_2310_16122_amd import tune

        best, best_ms, tried = tune.autotune(L, step32, repeats=2)
        L_rand.set_tuning(**best)
        tuned = {"tried": len(tried), "best": best, "best_ms": round(best_ms, 3)}
        log(f"[bench] autotuned over {len(tried)} settings: {best} ({best_ms:.3f} ms)")
        prof = profiled_setup(config)
        if prof is not None and prof[1] == args.leaf_max:
            L.set_tuning(**prof[0])
            L_rand.set_tuning(**prof[0])
            tuned["timed"] = "the committed profile's tuning"
            log(f"[bench] timing with the committed profile's tuning {prof[0]}")
    L.timing(False)
    timed_steps(step32, 2, args.warmup, torch)
    L.timing(True)
    steps = args.steps
    ms32 = timed_steps(step32, steps, 0, torch)
    kt = L.kernel_times()
    L.timing(False)
    log(f"[bench] {config} f32 step {ms32:.3f} ms; kernels {kt}")
    inter, units = interactions(kt, steps, G, F)
    ran, per_kernel = per_kernel_table(kt, steps, units, config, table)
    dom = max(ran, key=lambda k: kt[k][0])
    rl = roofline(dom, kt[dom][0], kt[dom][1], units[dom], config, table)
    rl_accel = roofline("accel", kt["accel"][0], kt["accel"][1], units["accel"], config, table)
    flop_step = sum(per_kernel[k]["flop_per_pair"] * units[k] * kt[k][1] / steps for k in ran)

    # the same step with particle arrays in the generated (random) order
    ms_rand = None
    if random_order:
        inv = torch.as_tensor(np.argsort(perm)).to(g32["x"].device)  # tree position of each generated particle
        ms_rand = timed_steps(crk_step(crk, L_rand, g_rand, cfg_t, "f32", ga32[inv].contiguous(),
                                       gdu32[inv].contiguous(), backward), max(2, steps // 4), 1, torch)
        log(f"[bench] {config} f32 step, random particle order: {ms_rand:.3f} ms")
    L_rand.free()
    del g_rand, L_rand
    torch.cuda.empty_cache()

    ms64 = acc = None
    if f64:
        g64 = crk.gas_to_device(cfg_t, "f64")
        ga64, gdu64 = upstream(crk, L, g64, cfg_t, "f64", torch)
        ms64 = timed_steps(crk_step(crk, L, g64, cfg_t, "f64", ga64, gdu64, backward), max(2, steps // 4), 1,
                           torch)
        log(f"[bench] {config} f64 step {ms64:.3f} ms")
        del ga64, gdu64
        acc = fp32_vs_fp64(crk, L, g32, g64, cfg_t, torch)
        log(f"[bench] {config} FP32 vs FP64 normwise errors {acc}")
        del g64
    torch.cuda.empty_cache()

    # the Extras pass and the viscous force pass, and the device leaf build, on the headline workload only
    ev = extras_viscosity(args, torch, crk, L, g32, cfg_t, G, F, config, table, f64=f64) if config == "C2" else None
    dbuild = None
    if not args.no_device_build:
        # C2: the build and the step over its order; C5: the build and its lists only
        dbuild = device_build_leg(args, torch, crk, cfg, L.get_tuning(), backward, st, step=config == "C2")
    out = {
        "metric": METRIC, "value": inter / (ms32 * 1e-3), "unit": "interactions/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": round(ms32, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{config}: {WORKLOADS[config]}", "n": cfg["n"],
                   "leaf_max": args.leaf_max,
                   "passes": "volume+corrections+accel_energy" +
                             ("+backward(accel adjoint, solve adjoint from stored sums, moments and "
                              "volume adjoints)" if backward else ""),
                   "particle_order": "tree order (identity permutation)" if identity else "tree-built",
                   "interactions_per_step": inter, "pairs_gather": G, "pairs_force": F,
                   "interactions_rule": "sum over the step's pair-kernel launches of their in-radius "
                                        "ordered pairs: volume, moments G each; accel and its three "
                                        "adjoint pair passes F each",
                   "list_entries": st["list_entries"], "tuning": L.get_tuning(), "autotune": tuned},
        "roofline": rl,
        "roofline_forward_accel": rl_accel,
        "kernels": per_kernel,
        "fp32_frac_step": round(flop_step / (ms32 * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS, 4),
        "fp64_gpu_ms_per_step": None if ms64 is None else round(ms64, 4),
        "fp64_over_fp32_time": None if ms64 is None else round(ms64 / ms32, 3),
        "fp32_vs_fp64_normwise": acc,
        "random_order_ms_per_step": None if ms_rand is None else round(ms_rand, 4),
        "build_ms": round(build_ms, 1), "list_build_gpu_ms": round(cull[0], 3),
        "list_build_note": "neighbour-list count, fill and schedule kernels of one build",
        "generate_s": round(gen_s, 1),
        "extras_viscosity": ev,
        "device_build": dbuild,
    }
    if cpu and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_hydro(cfg, args.cpu_budget)
    L.free()
    del L, g32, ga32, gdu32
    torch.cuda.empty_cache()
    return out


def device_build_leg(args, torch, crk, cfg, tuning, backward, host_stats, step=True):
    """The leaf build on the device (Morton octree; crk_build_leaf_pairs_device)
    on the generated order: wall time, its list-build kernels, whether its
    lists hold as many entries as the host build's; with step, the same step
    as the headline one over particles in the device build's order."""
    import numpy as np

    g_rand = crk.gas_to_device(cfg, "f32")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    Ld = crk.crk_build_leaf_pairs_device(g_rand["x"], g_rand["y"], g_rand["z"], g_rand["h"],
                                         leaf_max=args.leaf_max, prec="f32")
    build_ms = (time.perf_counter() - tb) * 1e3
    cull = Ld.kernel_times()["cull"]
    std = Ld.stats()
    perm = Ld.perm().cpu().numpy()
    Ld.free()
    del g_rand, Ld
    same = std["list_entries"] == host_stats["list_entries"] and std["pairs_force"] == host_stats["pairs_force"]
    if not step:
        log(f"[bench] device build {build_ms:.0f} ms (list build kernels {cull[0]:.2f} ms); same list "
            f"entries as the host build: {same}")
        torch.cuda.empty_cache()
        return {"build_ms": round(build_ms, 1), "list_build_gpu_ms": round(cull[0], 3),
                "list_entries": std["list_entries"], "same_lists_as_host_build": same,
                "padded_slots": std["padded_slots"], "host_build_padded_slots": host_stats["padded_slots"]}
    cfg_t = {k: (v[perm] if isinstance(v, np.ndarray) and v.shape == (cfg["n"],) else v)
             for k, v in cfg.items()}
    g32 = crk.gas_to_device(cfg_t, "f32")
    L = crk.crk_build_leaf_pairs_device(g32["x"], g32["y"], g32["z"], g32["h"], leaf_max=args.leaf_max,
                                        prec="f32")
    identity = bool((L.perm().cpu().numpy() == np.arange(cfg["n"])).all())
    L.set_tuning(**tuning)
    st = L.stats()
    ga, gdu = upstream(crk, L, g32, cfg_t, "f32", torch)
    ms = timed_steps(crk_step(crk, L, g32, cfg_t, "f32", ga, gdu, backward), args.steps, args.warmup, torch)
    log(f"[bench] device build {build_ms:.0f} ms (list build kernels {cull[0]:.2f} ms); step over its "
        f"order {ms:.3f} ms; stats {st}")
    out = {"build_ms": round(build_ms, 1), "list_build_gpu_ms": round(cull[0], 3),
           "same_lists_as_host_build": same,
           "ms_per_step": round(ms, 4), "identity_order": identity, "leaves": st["leaves"],
           "list_entries": st["list_entries"], "padded_slots": st["padded_slots"],
           "host_build_padded_slots": host_stats["padded_slots"],
           "note": "same lists per particle as the host build; the step is the headline step (same "
                   "tuning) over particles in the device build's order"}
    L.free()
    del L, g32, ga, gdu
    torch.cuda.empty_cache()
    return out


def extras_viscosity(args, torch, crk, L, g32, cfg_t, G, F, config, table, f64=True):
    """The Extras pass and the force pass with the artificial viscosity on the
    same tree (not part of the headline step): per-launch times, interactions/s
    (G gather pairs for Extras, F force pairs for the viscous force pass), the
    algorithmic FP32 rate from the oracle's FLOP counts, and the FP32 outputs
    against the FP64 GPU form over every particle."""
    def run(g, prec):
        o = crk.forward(L, g, cfg_t["gamma"], prec)
        corr = (o["A"], o["B"], o["dA"], o["dB"])
        return o, corr

    o32, c32 = run(g32, "f32")
    reps = max(4, args.steps // 2)

    def step():
        rhoR, dv, du = crk.crk_extras(L, g32, o32["V"], c32, "f32")
        crk.crk_accel_energy_visc(L, g32, o32["V"], o32["rho"], c32, dv, cfg_t["gamma"], "f32")

    timed_steps(step, 1, 1, torch)
    L.timing(True)
    timed_steps(step, reps, 0, torch)
    kt = L.kernel_times()
    L.timing(False)
    res = {}
    for kind, units in (("extras", G), ("accel_visc", F)):
        ms = kt[kind][0] / max(kt[kind][1], 1)
        flop = table[kind]
        res[kind] = {"avg_ms": round(ms, 4), "interactions_per_s": units / (ms * 1e-3),
                     "tflops_algorithmic": round(flop * units / (ms * 1e-3) / 1e12, 3),
                     "frac_fp32_peak": round(flop * units / (ms * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS, 4),
                     "flop_per_pair_oracle": flop, "units_per_launch": units}
    log(f"[bench] {config} extras {res['extras']['avg_ms']:.3f} ms, viscous force pass "
        f"{res['accel_visc']['avg_ms']:.3f} ms")

    # the force pass with the compatible energy partition (inviscid), and the
    # adjoint of the viscous chain (force adjoint with the viscosity, Extras adjoint)
    w = torch.as_tensor(cfg_t["w"]).float().to(g32["x"].device)
    c = torch.as_tensor(cfg_t["c"]).float().to(g32["x"].device)
    rhoR, dv32, _ = crk.crk_extras(L, g32, o32["V"], c32, "f32")
    av, _, _ = crk.crk_accel_energy_visc(L, g32, o32["V"], o32["rho"], c32, dv32, cfg_t["gamma"], "f32")
    ga = (2.0 * w[:, None] * av).contiguous()

    def compat_step():
        crk.crk_accel_energy_compatible(L, g32, o32["V"], o32["rho"], c32, 0.1, gamma=cfg_t["gamma"], prec="f32")

    def visc_bwd_step():
        crk.crk_accel_energy_visc_backward(L, g32, o32["V"], o32["rho"], c32, dv32, ga, c, cfg_t["gamma"], "f32")

    # kinds: (report name, kernel kinds whose launch times add up, FLOP key, units per launch)
    for name, fn, kinds in (("compatible", compat_step, (("accel", ("accel",), "accel_compat", F),)),
                            ("visc_backward", visc_bwd_step,
                             (("visc_force_adjoint", ("accel_adj",), "accel_visc_adj", F),
                              ("extras_adj", ("extras_adj",), "extras_adj", G)))):
        timed_steps(fn, 1, 1, torch)
        L.timing(True)
        ms_call = timed_steps(fn, reps, 0, torch)
        kt = L.kernel_times()
        L.timing(False)
        sub = {"ms_per_call": round(ms_call, 4)}
        for kind, parts, fkey, units in kinds:
            ms = sum(kt[p][0] / max(kt[p][1], 1) for p in parts)
            flop = table[fkey]
            sub[kind] = {"avg_ms": round(ms, 4), "interactions_per_s": units / (ms * 1e-3),
                         "tflops_algorithmic": round(flop * units / (ms * 1e-3) / 1e12, 3),
                         "frac_fp32_peak": round(flop * units / (ms * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS, 4),
                         "flop_per_pair_oracle": flop, "units_per_launch": units}
            if len(parts) > 1:
                sub[kind]["kernels_ms"] = {p: round(kt[p][0] / max(kt[p][1], 1), 4) for p in parts}
        res[name] = sub
        log(f"[bench] {config} {name}: {sub}")
    if f64:
        g64 = crk.gas_to_device(cfg_t, "f64")
        o64, c64 = run(g64, "f64")
        e32 = crk.crk_extras(L, g32, o32["V"], c32, "f32")
        e64 = crk.crk_extras(L, g64, o64["V"], c64, "f64")
        a32 = crk.crk_accel_energy_visc(L, g32, o32["V"], o32["rho"], c32, e32[1], cfg_t["gamma"], "f32")
        a64 = crk.crk_accel_energy_visc(L, g64, o64["V"], o64["rho"], c64, e64[1], cfg_t["gamma"], "f64")
        err = {}
        for k, u, v in zip(("rhoR", "dv", "du", "a_visc", "dudt_visc"), e32 + a32[:2], e64 + a64[:2]):
            err[k] = float(f"{((u.double() - v).abs().max() / v.abs().max()).item():.3e}")
        w64, c64w = w.double(), c.double()
        b32 = crk.crk_accel_energy_visc_backward(L, g32, o32["V"], o32["rho"], c32, e32[1],
                                                 (2.0 * w[:, None] * a64[0].float()).contiguous(), c,
                                                 cfg_t["gamma"], "f32")
        b64 = crk.crk_accel_energy_visc_backward(L, g64, o64["V"], o64["rho"], c64, e64[1],
                                                 (2.0 * w64[:, None] * a64[0]).contiguous(), c64w,
                                                 cfg_t["gamma"], "f64")
        for k, u, v in zip(("gx_visc", "gv_visc", "gu_visc"), b32, b64):
            err[k] = float(f"{((u.double() - v).abs().max() / v.abs().max()).item():.3e}")
        # the viscous chain's gradient jumps where a pair's viscosity switches on,
        # so the end-to-end figures above include the jumps the FP32 forward
        # crosses; against the FP64 backward at the FP32 forward's own state
        # (V, rho, corrections, dv) they measure the FP32 backward's arithmetic
        d = lambda t: t.double().contiguous()
        bs = crk.crk_accel_energy_visc_backward(L, g64, d(o32["V"]), d(o32["rho"]), tuple(d(t) for t in c32),
                                                d(e32[1]), (2.0 * w64[:, None] * a64[0]).contiguous(), c64w,
                                                cfg_t["gamma"], "f64")
        for k, u, v in zip(("gx_visc_same_state", "gv_visc_same_state", "gu_visc_same_state"), b32, bs):
            err[k] = float(f"{((u.double() - v).abs().max() / v.abs().max()).item():.3e}")
        del bs
        res["fp32_vs_fp64_normwise"] = err
        del g64, o64, c64, e64, a64, b32, b64
    torch.cuda.empty_cache()
    return res


# ---------------------------------------------------------------- gravity step
def bench_gravity(args, torch, crk, tuning=None, leaf_max=None):
    import synth

    table = flop_table()
    cfg = synth.make_config("C3")
    log(f"[bench] generated C3: n={cfg['n']}")
    x, y, z = (torch.as_tensor(cfg[k]).cuda() for k in ("x", "y", "z"))

    def build(lm, xx, yy, zz):
        return crk.crk_build_leaf_pairs(xx, yy, zz, None, r_fixed=cfg["r_cut"], leaf_max=lm,
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
    if tuning or args.no_autotune:
        L = build(leaf_max or 512, x, y, z)
        if tuning:
            L.set_tuning(**tuning)
    else:
        from paper_2310_16122_amd import tune

        leaf, L, tun, best_ms, per_leaf = tune.autotune_leaf_size(
            lambda lm: build(lm, x, y, z), make_step, leaf_values=(128, 256, 512), log=log, repeats=2,
            space=tune.GRAVITY_SPACE)
        tuned = {"leaf_max": leaf, "ms_by_leaf": {str(k): round(v, 3) for k, v in per_leaf.items()},
                 "best": tun, "best_ms": round(best_ms, 3)}
        log(f"[bench] autotuned gravity: leaf {leaf}, {tun} ({best_ms:.3f} ms)")
        prof = profiled_setup("C3")
        if prof is not None and prof[1] is not None:
            if prof[1] != leaf:
                L.free()
                L = build(prof[1], x, y, z)
            L.set_tuning(**prof[0])
            tuned["timed"] = f"the committed profile's tree (leaf {prof[1]}) and tuning"
            log(f"[bench] timing gravity with the committed profile's leaf {prof[1]} and tuning {prof[0]}")
    st = L.stats()
    step = make_step(L)

    timed_steps(step, 2, args.warmup, torch)
    L.timing(True)
    ms = timed_steps(step, args.steps, 0, torch)
    kt = L.kernel_times()
    L.timing(False)
    inter = st["pairs_force"]
    # the adjoint (dL/dx for seeded dL/da), same tree and tuning
    ga = torch.randn(cfg["n"], 3, generator=torch.Generator().manual_seed(3)).float().cuda()

    def adj_step():
        crk.sr_gravity_backward(L, x, y, z, m, ga, cfg["G"], cfg["eps"], cfg["r_cut"], prec="f32")

    timed_steps(adj_step, 1, 1, torch)
    L.timing(True)
    ms_adj = timed_steps(adj_step, max(2, args.steps // 2), 0, torch)
    kta = L.kernel_times()
    L.timing(False)
    adj_launch = kta["gravity_adj"][0] / max(kta["gravity_adj"][1], 1)
    adj = {"ms_per_call": round(ms_adj, 4), "avg_launch_ms": round(adj_launch, 4),
           "interactions_per_s": inter / (adj_launch * 1e-3),
           "tflops_algorithmic": round(table["gravity_adj"] * inter / (adj_launch * 1e-3) / 1e12, 3),
           "frac_fp32_peak": round(table["gravity_adj"] * inter / (adj_launch * 1e-3) / 1e12 /
                                   PEAK_FP32_VALU_TFLOPS, 4),
           "flop_per_pair_oracle": table["gravity_adj"]}
    log(f"[bench] C3 gravity adjoint {adj_launch:.3f} ms per launch")
    out = {
        "metric": METRIC, "value": inter / (ms * 1e-3), "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"C3: {WORKLOADS['C3']}", "n": cfg["n"],
                   "interactions_per_step": inter, "candidate_pairs": st["candidate_pairs"],
                   "leaves": st["leaves"], "leaf_max": (tuned or {}).get("leaf_max", leaf_max or 512),
                   "particle_order": "tree order", "tuning": L.get_tuning(), "autotune": tuned},
        "roofline": roofline("gravity", kt["gravity"][0], kt["gravity"][1], inter, "C3", table),
        "adjoint": adj,
        "build_ms": round(build_ms, 1),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_gravity(cfg, args.cpu_budget)
    L.free()
    return out


def c5_summary(r):
    """The C5 leg of the default run, condensed into the headline line."""
    keys = ("ms_per_step", "value", "fp64_gpu_ms_per_step", "fp64_over_fp32_time", "fp32_vs_fp64_normwise",
            "roofline", "roofline_forward_accel", "kernels", "build_ms", "list_build_gpu_ms", "generate_s",
            "device_build")
    out = {k: r[k] for k in keys if k in r}
    out["workload"] = r["config"]["workload"]
    out["interactions_per_step"] = r["config"]["interactions_per_step"]
    out["tuning"] = r["config"]["tuning"]
    out["steps"] = r["steps"]
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
    ap.add_argument("--no-c5", action="store_true", help="C2 only: skip the 256^3 workload")
    ap.add_argument("--c5-steps", type=int, default=6)
    ap.add_argument("--no-random-order", action="store_true",
                    help="skip the comparison step on randomly ordered particle arrays")
    ap.add_argument("--gravity-tuning", default=None, help="JSON crk_tuning for the gravity workload")
    ap.add_argument("--gravity-leaf-max", type=int, default=512,
                    help="gravity leaf size when its tuning is given")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-device-build", action="store_true", help="C2 only: skip the device leaf build leg")
    ap.add_argument("--no-backward", action="store_true", help="forward passes only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work per workload")
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
    tuning = json.loads(args.tuning) if args.tuning else None
    if args.config == "C3":
        out = bench_gravity(args, torch, crk, json.loads(args.gravity_tuning) if args.gravity_tuning else tuning,
                            args.gravity_leaf_max if args.gravity_tuning else args.leaf_max)
    else:
        out = bench_hydro(args, torch, crk, tuning=tuning, autotune=not args.no_autotune,
                          random_order=not args.no_random_order, f64=not args.no_f64)
        if args.config == "C2":
            import gc

            if not args.no_c5:
                # the paper's per-GPU gas share, with the C2 workload's tuning
                cargs = argparse.Namespace(**vars(args))
                cargs.steps = args.c5_steps
                cargs.warmup = 1
                r5 = bench_hydro(cargs, torch, crk, config="C5", tuning=out["config"]["tuning"],
                                 autotune=False, random_order=False, f64=not args.no_f64, cpu=False)
                out["c5"] = c5_summary(r5)
                gc.collect()
                torch.cuda.empty_cache()
            if not args.no_gravity:
                # the gravity pass on its own workload, in the same JSON line
                gc.collect()
                torch.cuda.empty_cache()
                out["sr_gravity"] = bench_gravity(
                    args, torch, crk, json.loads(args.gravity_tuning) if args.gravity_tuning else None,
                    args.gravity_leaf_max)
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
