"""Autotuner for the launch and tiling choices of a ``crk_leaves`` handle.

The search space is the ``crk_tuning`` struct of ``include/crk.h`` --
persistent work queue or one tile per wave, persistent grid size, waves per
workgroup, number of XCD chunks of tile order, tree order or longest-first
order, compensation chunk of the FP32 pair sums -- plus the leaf size of the
tree (which needs a rebuild).  Candidates are timed with the library's own
per-kernel HIP-event timing on the caller's step (a closure that runs the
passes), by coordinate descent from the current setting.  Results are cached
in a JSON file keyed by device, workload name, particle count, precision and
leaf size.
"""

from __future__ import annotations

import json
import os

import torch

SPACE = {
    "xcd_groups": (1, 8),
    "tile_order": (0, 1),
    "persistent": (0, 1),
    "waves_per_cu": (8, 16, 32),
    "block_waves": (1, 2, 4),
    "kahan_chunk": (1, 4, 8, 16),
    "stage16": (0, 1),
}
# short-range gravity also chooses how candidates are exchanged between lanes
# (LDS broadcast, scalar-register broadcast, cross-lane permute)
GRAVITY_SPACE = dict(SPACE, exchange=(0, 1, 2))


def _sync():
    if torch.cuda.is_available():
        torch.cuda.synchronize()


def _time_step(leaves, step, repeats):
    step()
    _sync()
    leaves.timing(True)
    for _ in range(repeats):
        step()
    kt = leaves.kernel_times()
    leaves.timing(False)
    return sum(ms for ms, _ in kt.values()) / repeats


def cache_key(name, n, prec, leaf_max):
    if not torch.cuda.is_available():
        return f"cpu|{name}|n={n}|{prec}|leaf={leaf_max}"
    dev = torch.cuda.get_device_properties(0)
    arch = getattr(dev, "gcnArchName", dev.name)
    return f"{arch}|{name}|n={n}|{prec}|leaf={leaf_max}"


def load_cache(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(path, cache):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(leaves, step, space=None, repeats=3, rounds=2, cache_path=None, key=None, log=None):
    """Coordinate descent over ``space``; leaves the best setting on the handle.

    Returns (best tuning dict, best ms per step, list of (tuning, ms) tried).
    A cached entry for ``key`` is applied without timing.
    """
    cache = load_cache(cache_path)
    if key and key in cache:
        leaves.set_tuning(**cache[key]["tuning"])
        return cache[key]["tuning"], cache[key]["ms"], []
    space = space or SPACE
    best = leaves.get_tuning()
    best_ms = _time_step(leaves, step, repeats)
    tried = [(dict(best), best_ms)]
    for _ in range(rounds):
        improved = False
        for field, values in space.items():
            for v in values:
                if best[field] == v:
                    continue
                cand = dict(best, **{field: v})
                if not cand["persistent"] and field == "waves_per_cu":
                    continue  # only used by the persistent grid
                leaves.set_tuning(**cand)
                ms = _time_step(leaves, step, repeats)
                tried.append((cand, ms))
                if log:
                    log(f"[tune] {cand} -> {ms:.3f} ms")
                if ms < best_ms * 0.995:
                    best, best_ms, improved = cand, ms, True
            leaves.set_tuning(**best)
        if not improved:
            break
    leaves.set_tuning(**best)
    if key:
        cache[key] = {"tuning": best, "ms": best_ms}
        save_cache(cache_path, cache)
    return best, best_ms, tried


def autotune_leaf_size(build, make_step, leaf_values=(32, 64, 128, 256), log=None, **kw):
    """Pick the leaf size: ``build(leaf_max)`` returns a handle, ``make_step(handle)``
    its step closure; every size is tuned with ``autotune``.  Returns
    (best leaf size, its handle, its tuning, ms per step, {leaf: ms})."""
    results = {}
    best = None
    for leaf in leaf_values:
        L = build(leaf)
        tun, ms, _ = autotune(L, make_step(L), log=log, **kw)
        results[leaf] = ms
        if log:
            log(f"[tune] leaf {leaf}: {ms:.3f} ms with {tun}")
        if best is None or ms < best[3]:
            if best is not None:
                best[1].free()
            best = (leaf, L, tun, ms)
        else:
            L.free()
    return best + (results,)
