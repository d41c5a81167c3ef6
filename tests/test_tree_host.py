"""Host tree and tile candidate lists (CPU only, no GPU).

The RCB tree and the per-tile candidate ranges are plain host C++; they are
compiled here with g++ through a test shim and checked by brute force: every
ordered pair inside the interaction radius must fall into its tile's
candidate ranges, and tree order must be a permutation.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_16122_amd", "csrc")
_lib = None


def shim():
    global _lib
    if _lib is None:
        out = os.path.join(ROOT, "tests", "_tree_shim.so")
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-I", CSRC, os.path.join(ROOT, "tests", "tree_shim.cpp"),
                               os.path.join(CSRC, "tree.cpp"), "-o", out])
        _lib = ctypes.CDLL(out)
    return _lib


def build(cfg, H=None, r_fixed=0.0, leaf_max=32, leaf_min=1, split_extent=0.0, weight=None,
          leaves=False):
    n = len(cfg["x"])
    q = [np.ascontiguousarray(synth.to_u32(cfg[k])) for k in ("x", "y", "z")]
    perm = np.empty(n, np.int32)
    nt = (n + 63) // 64
    rng_off = np.empty(nt + 1, np.int32)
    cap = 64 * nt * 64
    rng = np.empty(cap, np.int32)
    nl = ctypes.c_int()
    cp = ctypes.c_longlong()
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    Hc = None if H is None else np.ascontiguousarray(H, np.float64)
    W = None if weight is None else np.ascontiguousarray(weight, np.int32)
    lb = np.empty(n + 1, np.int32)
    rc = shim().tree_shim(ctypes.c_longlong(n), P(q[0]), P(q[1]), P(q[2]),
                          None if Hc is None else P(Hc), ctypes.c_double(r_fixed),
                          leaf_max, leaf_min, ctypes.c_double(split_extent), P(perm),
                          ctypes.byref(nl), P(rng_off), P(rng), cap, ctypes.byref(cp),
                          None if W is None else P(W), P(lb))
    assert rc >= 0
    res = (perm, nl.value, rng_off, rng[:rc].reshape(-1, 2), cp.value)
    return res + (lb[:nl.value],) if leaves else res


def brute_pairs(cfg, radius_fn):
    P = np.stack([cfg["x"], cfg["y"], cfg["z"]], 1)
    d = P[:, None, :] - P[None, :, :]
    d -= np.floor(d + 0.5)
    r = np.sqrt((d * d).sum(-1))
    R = radius_fn()
    m = r < R
    np.fill_diagonal(m, False)
    return m


def covered(perm, rng_off, rng, need):
    n = len(perm)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    cover = np.zeros((n, n), bool)  # in tree order: (i, j) candidate?
    for t in range(len(rng_off) - 1):
        rows = slice(64 * t, min(n, 64 * t + 64))
        for b, e in rng[rng_off[t]:rng_off[t + 1]]:
            cover[rows, b:e] = True
    need_s = need[np.ix_(perm, perm)]
    return np.all(cover[need_s])


@pytest.mark.parametrize("leaf_max", [8, 32, 128])
def test_hydro_candidates_cover_all_pairs(leaf_max):
    cfg = synth.make_config("C2", n_side=12)
    H = 2.0 * cfg["h"]
    perm, nl, off, rng, cp = build(cfg, H=H, leaf_max=leaf_max)
    assert sorted(perm.tolist()) == list(range(cfg["n"]))
    need = brute_pairs(cfg, lambda: np.maximum(H[:, None], H[None, :]))
    assert covered(perm, off, rng, need)
    assert cp >= need.sum()


def test_fixed_radius_candidates_and_extent_rule():
    cfg = synth.make_gravity(n_side=10)
    rc = cfg["r_cut"] * 2.5
    perm, nl, off, rng, cp = build(cfg, r_fixed=rc, leaf_max=64, leaf_min=4, split_extent=rc)
    need = brute_pairs(cfg, lambda: rc)
    assert covered(perm, off, rng, need)


def test_leaf_sizes_and_lattice_edges():
    cfg = synth.make_lattice(n_side=16, jitter=0.0)
    H = 2.0 * cfg["h"]
    perm, nl, off, rng, _ = build(cfg, H=H, leaf_max=100)
    # median splits: every leaf holds between 50 and 100 particles
    assert 4096 / 100 <= nl <= 4096 / 50
    need = brute_pairs(cfg, lambda: np.maximum(H[:, None], H[None, :]))
    assert covered(perm, off, rng, need)


def test_tiny_and_ragged_inputs():
    rng_ = np.random.default_rng(1)
    for n in (1, 2, 63, 65, 130):
        cfg = dict(x=synth.grid_round(rng_.random(n)), y=synth.grid_round(rng_.random(n)),
                   z=synth.grid_round(rng_.random(n)))
        H = np.full(n, 0.3)
        perm, nl, off, rng, _ = build(cfg, H=H, leaf_max=16)
        assert sorted(perm.tolist()) == list(range(n))
        need = brute_pairs(cfg, lambda: np.maximum(H[:, None], H[None, :]))
        assert covered(perm, off, rng, need)


def test_rebuild_on_tree_order_is_identity():
    """Median splits keep the current order, so particles already in tree order stay put."""
    cfg = synth.make_config("C2", n_side=16)
    H = 2.0 * cfg["h"]
    perm, *_ = build(cfg, H=H, leaf_max=32)
    cfg2 = {k: cfg[k][perm] for k in ("x", "y", "z")}
    perm2, *_ = build(cfg2, H=H[perm], leaf_max=32)
    assert np.array_equal(perm2, np.arange(cfg["n"]))
    lat = synth.make_lattice(n_side=16, jitter=0.0)  # many equal keys
    p, *_ = build(lat, H=2.0 * lat["h"], leaf_max=64)
    lat2 = {k: lat[k][p] for k in ("x", "y", "z")}
    p2, *_ = build(lat2, H=2.0 * lat["h"], leaf_max=64)
    assert np.array_equal(p2, np.arange(lat["n"]))


def test_weighted_leaves_keep_sets_and_sort_by_work():
    """With a work weight, each leaf holds the same particles, ordered by
    decreasing weight (stable), and the new tiles' candidates still cover
    every pair; rebuilding on that order with the same weights is the identity."""
    cfg = synth.make_config("C2", n_side=14)
    n = cfg["n"]
    H = 2.0 * cfg["h"]
    w = np.random.default_rng(4).integers(40, 120, n).astype(np.int32)
    p0, nl0, _, _, _, lb0 = build(cfg, H=H, leaf_max=128, leaves=True)
    p1, nl1, off, rng, _, lb1 = build(cfg, H=H, leaf_max=128, weight=w, leaves=True)
    assert nl0 == nl1 and np.array_equal(lb0, lb1)
    ends = np.append(lb1[1:], n)
    for b, e in zip(lb1, ends):
        assert set(p0[b:e]) == set(p1[b:e])
        ww = w[p1[b:e]]
        assert np.all(ww[:-1] >= ww[1:])
        # stable: equal weights keep the unweighted order
        for v in np.unique(ww):
            sel = p1[b:e][ww == v]
            pos0 = {x: k for k, x in enumerate(p0[b:e])}
            assert [pos0[x] for x in sel] == sorted(pos0[x] for x in sel)
    need = brute_pairs(cfg, lambda: np.maximum(H[:, None], H[None, :]))
    assert covered(p1, off, rng, need)
    cfg2 = {k: cfg[k][p1] for k in ("x", "y", "z")}
    p2, *_ = build(cfg2, H=H[p1], leaf_max=128, weight=w[p1])
    assert np.array_equal(p2, np.arange(n))
