"""Parity of the HIP passes with the FP64 oracle, through the C ABI (GPU only).

Error metric per output array (normwise): max_i |y_i - y_ref_i| / max_i |y_ref_i|.
Bars: FP64 path <= 1e-12, FP32 path (FP32 pairs + compensated sums, FP64
solve and totals) <= 1e-5.  Small configurations are compared element by
element with the full brute-force oracle; the full-size configuration is
compared on sampled particles, each evaluated by the oracle inside its
three-hop closure.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.cases import dense_case, fallback_case, planar_case

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
# C5 backward, FP32 mixed path against the FP64 form, normwise over all 2^24
# particles (measured values in the test's output)
C5_BACKWARD_TOL = {"gx": 1e-4, "gv": 1e-4, "gu": 1e-4}
KEYS = ("V", "rho", "A", "B", "dA", "dB", "a", "dudt")


@pytest.fixture(scope="module")
def crk():
    import paper_2310_16122_amd as crk

    crk.load_library()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return crk


def normwise(y, ref):
    """max |y - ref| / max |ref|; the absolute error where ref is identically zero."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    err = np.abs(y - ref).max()
    return float(err / scale) if scale > 0 else float(err)


def run_gpu(crk, cfg, prec, leaf_max=64, tuning=None):
    g = crk.gas_to_device(cfg, prec)
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=leaf_max, prec=prec)
    if tuning:
        L.set_tuning(**tuning)
    out = crk.forward(L, g, cfg["gamma"], prec)
    torch.cuda.synchronize()
    host = {k: v.double().cpu().numpy() for k, v in out.items()}
    return host, L


_cache = {}


def oracle_full(name, n_side):
    key = (name, n_side)
    if key not in _cache:
        cfg = synth.make_config(name, n_side)
        _cache[key] = (cfg, oracle.hydro(cfg))
    return _cache[key]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,n_side", [("C1", None), ("C2", 21), ("C5", 24)])
def test_forward_chain_parity(crk, name, n_side, prec):
    cfg, ref = oracle_full(name, n_side)
    print(f"case {name} n_side={n_side} prec={prec} n={cfg['n']}", flush=True)
    got, L = run_gpu(crk, cfg, prec)
    errs = {k: normwise(got[k], ref[k]) for k in KEYS}
    print(errs, flush=True)
    for k in KEYS:
        assert errs[k] <= TOL[prec], (k, errs[k])
    assert int(got["n_fallback"][0]) == 0 == ref["n_fallback"]
    # FP64 totals: momentum and energy conserved to the precision of the path
    T = got["totals"]
    lim = 1e-13 if prec == "f64" else 2e-6
    assert np.abs(T[:3]).max() <= lim * T[4]
    assert abs(T[3]) <= lim * T[5]
    assert np.allclose(T[4], ref["totals"][4], rtol=1e-5)


def moments_from_stored_sums(S):
    """The oracle's 40 raw moments per particle rebuilt from crk_corrections'
    stored output ([30][n]: the 29 independent sums, then the neighbour count)."""
    n = S.shape[1]
    sym = [[0, 1, 2], [1, 3, 4], [2, 4, 5]]
    cub = {}
    k = 0
    for a in range(3):
        for b in range(a, 3):
            for c in range(b, 3):
                for p in {(a, b, c), (a, c, b), (b, a, c), (b, c, a), (c, a, b), (c, b, a)}:
                    cub[p] = k
                k += 1
    M = np.zeros((n, 40))
    M[:, :13] = S[:13].T
    for a in range(3):
        for c in range(3):
            M[:, 13 + 3 * a + c] = (S[0] if a == c else 0.0) + S[13 + sym[a][c]]
    for a in range(3):
        for b in range(a, 3):
            for c in range(3):
                t = S[19 + cub[(a, b, c)]].copy()
                if a == c:
                    t += S[1 + b]
                if b == c:
                    t += S[1 + a]
                M[:, 22 + 3 * sym[a][b] + c] = t
    return M


MOMENT_BLOCKS = ((0, 1), (1, 4), (4, 10), (10, 13), (13, 22), (22, 40))


def test_stored_moment_sums_match_oracle_moments(crk):
    """crk_corrections' optional output: the 29 independent sums and the
    neighbour count, rebuilt here into the 40 moments of the oracle."""
    cfg, ref = oracle_full("C2", 21)
    g = crk.gas_to_device(cfg, "f64")
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec="f64")
    V, _ = crk.crk_volume(L, g, "f64")
    A, B, dA, dB, S = crk.crk_corrections(L, g, V, "f64", store_sums=True)
    A0, B0, dA0, dB0 = crk.crk_corrections(L, g, V, "f64")
    for u, v in ((A, A0), (B, B0), (dA, dA0), (dB, dB0)):
        assert torch.equal(u, v)
    S = S.cpu().numpy()
    M_ref, nnb_ref = oracle.moments(cfg, ref["V"])
    M = moments_from_stored_sums(S)
    for lo, hi in MOMENT_BLOCKS:
        assert normwise(M[:, lo:hi], M_ref[:, lo:hi]) <= 1e-12, (lo, hi)
    assert np.array_equal(S[29].astype(np.int64), nnb_ref)


def test_fp32_against_fp64_all_particles_c2(crk):
    """C2 at 128^3: every output of the FP32 mixed path against the FP64 GPU
    path over all 2,097,152 particles (the oracle checks both on samples)."""
    cfg = synth.make_config("C2")
    print(f"case C2 full f32 vs f64 n={cfg['n']}", flush=True)
    g64, _ = run_gpu(crk, cfg, "f64", leaf_max=128)
    g32, _ = run_gpu(crk, cfg, "f32", leaf_max=128)
    for k in KEYS:
        assert normwise(g32[k], g64[k]) <= TOL["f32"], k


def test_interaction_counts_exact(crk):
    cfg, _ = oracle_full("C2", 21)
    got, L = run_gpu(crk, cfg, "f64")
    st = L.stats()
    assert st["pairs_gather"] == oracle.count_pairs(cfg, 0)[0]
    assert st["pairs_force"] == oracle.count_pairs(cfg, 1)[0]
    assert st["list_entries"] >= st["pairs_force"]


@pytest.mark.parametrize("leaf_max", [16, 128, 512])
def test_leaf_size_and_scheduling_do_not_change_results(crk, leaf_max):
    cfg, _ = oracle_full("C2", 21)
    base, _ = run_gpu(crk, cfg, "f32", leaf_max=64)
    for tun in ({"persistent": 0}, {"persistent": 1, "waves_per_cu": 3, "block_waves": 1}):
        got, _ = run_gpu(crk, cfg, "f32", leaf_max=leaf_max, tuning=tun)
        for k in KEYS:
            # the per-particle arithmetic does not depend on tree or schedule,
            # only the neighbour order does (compensated sums: tiny differences)
            assert normwise(got[k], base[k]) <= 2e-6, k


def test_bitwise_reproducible(crk):
    cfg, _ = oracle_full("C2", 21)
    a, _ = run_gpu(crk, cfg, "f32")
    b, _ = run_gpu(crk, cfg, "f32", tuning={"persistent": 0})
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_wide_record_addressing_is_bitwise_identical(crk, prec):
    """Record arrays beyond 4 GiB are addressed with 64-bit pointers instead of
    32-bit offsets; forcing that form on a small input changes no bit."""
    cfg, _ = oracle_full("C2", 21)
    a, _ = run_gpu(crk, cfg, prec)
    b, L = run_gpu(crk, cfg, prec, tuning={"addr64": 1})
    assert L.get_tuning()["addr64"] == 1
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_staged_16_byte_records_are_bitwise_identical(crk, prec):
    """Staging the volume and moments passes' neighbour records through LDS
    (one fetch per distinct particle of a slot) instead of gathering them lane
    by lane changes no bit, with and without the 64-bit record addressing."""
    cfg, _ = oracle_full("C2", 21)
    a, _ = run_gpu(crk, cfg, prec)
    for extra in ({}, {"addr64": 1}):
        b, L = run_gpu(crk, cfg, prec, tuning={"stage16": 1, **extra})
        assert L.get_tuning()["stage16"] == 1
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), (k, extra)
        L.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dense_neighbourhoods(crk, prec):
    """About 600 neighbours per particle: most tiles' neighbour sets overflow
    the list schedule's table and keep one-per-lane staging, the others fill it
    almost to the brim; every output against the oracle."""
    cfg = dense_case()
    print(f"case dense n={cfg['n']} prec={prec}", flush=True)
    ref = oracle.hydro(cfg)
    got, _ = run_gpu(crk, cfg, prec, leaf_max=64)
    for k in KEYS:
        assert normwise(got[k], ref[k]) <= TOL[prec], k


def test_kahan_chunk_within_tolerance(crk):
    cfg, ref = oracle_full("C2", 21)
    for chunk in (1, 8, 32, 64):
        got, _ = run_gpu(crk, cfg, "f32", tuning={"kahan_chunk": chunk})
        for k in KEYS:
            assert normwise(got[k], ref[k]) <= TOL["f32"], (chunk, k)


def test_lattice_zero_acceleration_gpu(crk):
    cfg = synth.make_lattice(n_side=16, jitter=0.0)
    ref = oracle.hydro(cfg)
    for prec, lim in (("f64", 1e-12), ("f32", 1e-5)):
        got, _ = run_gpu(crk, cfg, prec)
        scale = np.abs(oracle.hydro(synth.make_lattice())["a"]).max()
        assert np.abs(got["a"]).max() <= lim * scale, prec
        assert normwise(got["V"], ref["V"]) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_full_size_sampled_closure(crk, prec):
    """C2 at 128^3: 48 sampled particles against the oracle's per-target closure."""
    cfg = synth.make_config("C2")
    print(f"case C2 full n={cfg['n']} prec={prec}", flush=True)
    got, L = run_gpu(crk, cfg, prec, leaf_max=128)
    t = synth.sample_targets(cfg["n"], 48, seed=11)
    ref = oracle.hydro_targets(cfg, t)
    for k in KEYS:
        # normalised by the full GPU array's max (the oracle sees only the sample)
        scale = np.abs(got[k]).max()
        err = np.abs(got[k][t] - ref[k]).max() / scale
        assert err <= TOL[prec], (k, err)
    T = got["totals"]
    lim = 1e-13 if prec == "f64" else 2e-6
    assert np.abs(T[:3]).max() <= lim * T[4]


_listed = {}


def oracle_listed(name):
    """The oracle's full chain over exact neighbour lists (equal to its
    brute-force chain bit for bit, pinned on the CPU), cached per workload."""
    if name not in _listed:
        cfg = synth.make_config(name)
        off, idx = oracle.neighbour_lists(cfg)
        _listed[name] = (cfg, oracle.hydro_listed(cfg, off, idx))
    return _listed[name]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["C4", "C2"])
def test_full_size_every_particle(crk, name, prec):
    """C4 (64^3) and C2 (128^3) at full size, leaf 128: every output of every
    particle against the oracle's FP64 chain, element by element."""
    cfg, ref = oracle_listed(name)
    print(f"case {name} full every particle n={cfg['n']} prec={prec}", flush=True)
    got, L = run_gpu(crk, cfg, prec, leaf_max=128)
    errs = {k: normwise(got[k], ref[k]) for k in KEYS}
    print(errs, flush=True)
    for k in KEYS:
        assert errs[k] <= TOL[prec], (k, errs[k])
    assert int(got["n_fallback"][0]) == 0 == ref["n_fallback"]
    T = got["totals"]
    lim = 1e-13 if prec == "f64" else 2e-6
    assert np.abs(T[:3]).max() <= lim * T[4]
    assert abs(T[3]) <= lim * T[5]
    st = L.stats()
    if name == "C4":
        assert st["pairs_gather"] == oracle.count_pairs(cfg, 0)[0]
        assert st["pairs_force"] == oracle.count_pairs(cfg, 1)[0]
    L.free()


def test_c5_full_size_sampled(crk):
    """C5 at 256^3 (32-256 neighbours over a 16x density contrast), leaf 128, the
    benchmarked tuning: 128 sampled particles of the FP32 and FP64 forward chains
    against the oracle's per-target closure, and the momentum totals; then the
    FP32 mixed path against the FP64 GPU form over every particle, forward and
    backward (gradients of L = sum w |a|^2 + sum c du/dt)."""
    cfg = synth.make_config("C5")
    print(f"case C5 full n={cfg['n']}", flush=True)
    t = synth.sample_targets(cfg["n"], 128, seed=17)
    ref = oracle.hydro_targets(cfg, t)
    assert ref["n_fallback"] == 0
    res = {}
    for prec in ("f64", "f32"):
        got, L = run_gpu(crk, cfg, prec, leaf_max=128,
                         tuning={"persistent": 0, "block_waves": 4, "xcd_groups": 8, "kahan_chunk": 8})
        for k in KEYS:
            scale = np.abs(got[k]).max()
            err = np.abs(got[k][t] - ref[k]).max() / scale
            assert err <= TOL[prec], (prec, k, err)
        assert int(got["n_fallback"][0]) == 0
        T = got["totals"]
        assert np.abs(T[:3]).max() <= (1e-13 if prec == "f64" else 2e-6) * T[4]
        res[prec] = {k: got[k] for k in KEYS}
        # the backward with the same upstream adjoints (from the FP64 forward's a)
        if prec == "f64":
            a64 = torch.as_tensor(got["a"]).cuda()
        g = crk.gas_to_device(cfg, prec)
        o = crk.forward(L, g, cfg["gamma"], prec, store_sums=True)
        dt = o["a"].dtype
        ga = (2.0 * torch.as_tensor(cfg["w"]).cuda()[:, None] * a64).to(dt).contiguous()
        gdu = torch.as_tensor(cfg["c"]).to(dt).cuda()
        grads = crk.crk_accel_energy_backward(L, g, o["V"], o["rho"], (o["A"], o["B"], o["dA"], o["dB"], o["M"]),
                                              ga, gdu, cfg["gamma"], prec)
        res[prec].update({k: v.double().cpu().numpy() for k, v in zip(("gx", "gv", "gu"), grads)})
        L.free()
        del got, g, o, grads
        torch.cuda.empty_cache()
    # the FP32 mixed path against the FP64 GPU path over every particle
    errs = {k: normwise(res["f32"][k], res["f64"][k]) for k in KEYS + ("gx", "gv", "gu")}
    print("C5 FP32 vs FP64", errs, flush=True)
    for k in KEYS:
        assert errs[k] <= TOL["f32"], k
    for k in ("gx", "gv", "gu"):
        assert errs[k] <= C5_BACKWARD_TOL[k], (k, errs[k])


# ---------------------------------------------------------------- gravity
def gravity_case(n_side):
    cfg = synth.make_gravity(n_side=n_side)
    return cfg


def pair_term(cfg, r, poly=None, G=1.0):
    """|force per unit neighbour mass| of a pair at separation r (with the
    optional polynomial subtracted)."""
    f = 1.0 / (r ** 2 + cfg["eps"] ** 2) ** 1.5
    if poly is not None:
        f = f - np.polyval(np.asarray(poly)[::-1], r ** 2)
    return G * np.abs(f) * r


def borderline_bound(cfg, G=1.0, poly=None):
    """Per-particle sum of |pair term| over pairs with |r^2 - rc^2| <= 2^-20 rc^2."""
    from scipy.spatial import cKDTree

    P = np.stack([cfg["x"], cfg["y"], cfg["z"]], 1)
    tree = cKDTree(P, boxsize=1.0)
    rc = cfg["r_cut"]
    lo = rc * np.sqrt(1 - 2.0 ** -20)
    hi = rc * np.sqrt(1 + 2.0 ** -20)
    pairs = tree.query_pairs(hi, output_type="ndarray")
    d = P[pairs[:, 0]] - P[pairs[:, 1]]
    d -= np.floor(d + 0.5)
    r = np.sqrt((d * d).sum(1))
    sel = r >= lo
    b = np.zeros(len(P))
    f = pair_term(cfg, r[sel], poly, G)
    np.add.at(b, pairs[sel, 0], cfg["m"][pairs[sel, 1]] * f)
    np.add.at(b, pairs[sel, 1], cfg["m"][pairs[sel, 0]] * f)
    return b


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gravity_parity(crk, prec):
    cfg = gravity_case(24)
    print(f"case gravity n={cfg['n']} prec={prec}", flush=True)
    ref = oracle.gravity(cfg)
    dt = torch.float32 if prec == "f32" else torch.float64
    x, y, z = (torch.as_tensor(cfg[k]).cuda() for k in ("x", "y", "z"))
    m = torch.as_tensor(cfg["m"]).to(dt).cuda()
    L = crk.crk_build_leaf_pairs(x, y, z, None, r_fixed=cfg["r_cut"], leaf_max=512, leaf_min=16,
                                 split_extent=cfg["r_cut"], prec=prec)
    a = crk.sr_gravity(L, x, y, z, m, cfg["G"], cfg["eps"], cfg["r_cut"], prec=prec)
    a = a.double().cpu().numpy()
    bound = borderline_bound(cfg)
    err = np.abs(a - ref).max(1)
    scale = np.abs(ref).max()
    assert np.all(err <= TOL[prec] * scale + bound), (err.max() / scale)
    st = L.stats()
    assert st["pairs_force"] == oracle.count_pairs(cfg, 2, r_fixed=cfg["r_cut"])[0]


def borderline_bound_targets(cfg, targets, G=1.0):
    """borderline_bound restricted to the given target particles."""
    from scipy.spatial import cKDTree

    P = np.stack([cfg["x"], cfg["y"], cfg["z"]], 1)
    tree = cKDTree(P, boxsize=1.0)
    rc = cfg["r_cut"]
    lo, hi = rc * np.sqrt(1 - 2.0 ** -20), rc * np.sqrt(1 + 2.0 ** -20)
    b = np.zeros(len(targets))
    for k, (i, nb) in enumerate(zip(targets, tree.query_ball_point(P[targets], hi))):
        nb = np.asarray([j for j in nb if j != i], dtype=np.int64)
        if nb.size == 0:
            continue
        d = P[i] - P[nb]
        d -= np.floor(d + 0.5)
        r = np.sqrt((d * d).sum(1))
        sel = r >= lo
        b[k] = (cfg["m"][nb[sel]] * pair_term(cfg, r[sel], None, G)).sum()
    return b


def gravity_gpu(crk, cfg, prec, leaf_max=512, tuning=None, poly=None):
    dt = torch.float32 if prec == "f32" else torch.float64
    x, y, z = (torch.as_tensor(cfg[k]).cuda() for k in ("x", "y", "z"))
    m = torch.as_tensor(cfg["m"]).to(dt).cuda()
    L = crk.crk_build_leaf_pairs(x, y, z, None, r_fixed=cfg["r_cut"], leaf_max=leaf_max, leaf_min=16,
                                 split_extent=cfg["r_cut"], prec=prec)
    if tuning:
        L.set_tuning(**tuning)
    a = crk.sr_gravity(L, x, y, z, m, cfg["G"], cfg["eps"], cfg["r_cut"], poly=poly, prec=prec)
    return a.double().cpu().numpy(), L


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gravity_unsoftened(crk, prec):
    """eps = 0: the self pair and coincident pairs must be excluded explicitly."""
    cfg = dict(gravity_case(16), eps=0.0)
    print(f"case gravity eps=0 n={cfg['n']} prec={prec}", flush=True)
    ref = oracle.gravity(cfg)
    a, _ = gravity_gpu(crk, cfg, prec, leaf_max=128)
    err = np.abs(a - ref).max(1)
    assert np.all(err <= TOL[prec] * np.abs(ref).max() + borderline_bound(cfg)), err.max()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gravity_spread_tiles(crk, prec):
    """Tiles whose particles span more than a quarter of the box take the
    fixed-point separation path (no bounding-box cull)."""
    rng = np.random.default_rng(5)
    n = 300
    cfg = dict(x=synth.grid_round(rng.random(n)), y=synth.grid_round(rng.random(n)),
               z=synth.grid_round(rng.random(n)), m=synth.f32(rng.uniform(0.5, 1.5, n) / n),
               G=1.0, eps=float(synth.f32(0.01)), r_cut=float(synth.f32(0.2)))
    print(f"case gravity spread n={n} prec={prec}", flush=True)
    ref = oracle.gravity(cfg)
    for leaf_max in (64, 512):
        a, _ = gravity_gpu(crk, cfg, prec, leaf_max=leaf_max)
        err = np.abs(a - ref).max(1)
        assert np.all(err <= TOL[prec] * np.abs(ref).max() + borderline_bound(cfg)), (leaf_max, err.max())


_c3 = {}


def c3_reference():
    if not _c3:
        cfg = synth.make_config("C3")
        t = synth.sample_targets(cfg["n"], 256, seed=13)
        _c3.update(cfg=cfg, t=t, ref=oracle.gravity(cfg, t), bound=borderline_bound_targets(cfg, t))
    return _c3["cfg"], _c3["t"], _c3["ref"], _c3["bound"]


@pytest.mark.parametrize("prec,tuning", [("f32", None), ("f32", {"xcd_groups": 1, "tile_order": 1}),
                                         ("f32", {"persistent": 1, "waves_per_cu": 8}), ("f64", None)])
def test_gravity_full_size_sampled(crk, prec, tuning):
    """C3 at 2 x 128^3, leaf 512 (the benchmarked launch): 256 sampled particles
    against the brute-force oracle, FP32 (three launch forms) and FP64."""
    cfg, t, ref, bound = c3_reference()
    print(f"case C3 full n={cfg['n']} prec={prec} tuning={tuning}", flush=True)
    a, L = gravity_gpu(crk, cfg, prec, leaf_max=512, tuning=tuning)
    err = np.abs(a[t] - ref).max(1)
    assert np.all(err <= TOL[prec] * np.abs(a).max() + bound), err.max()
    L.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gravity_polynomial(crk, prec):
    cfg = gravity_case(16)
    poly = np.array([1.0, -2.0, 3.0, 0.5, -0.25, 0.125]) * 1e3
    ref = oracle.gravity(cfg, poly=poly)
    a, _ = gravity_gpu(crk, cfg, prec, leaf_max=64, poly=poly)
    err = np.abs(a - ref).max(1)
    assert np.all(err <= TOL[prec] * np.abs(ref).max() + borderline_bound(cfg, poly=poly)), err.max()


# ---------------------------------------------------------------- edges and errors
def test_empty_and_tiny_inputs(crk):
    for n in (0, 1, 5, 63, 65):
        rng = np.random.default_rng(n)
        cfg = dict(x=synth.grid_round(rng.random(n)), y=synth.grid_round(rng.random(n)),
                   z=synth.grid_round(rng.random(n)), h=synth.f32(np.full(n, 0.2)),
                   m=synth.f32(np.full(n, 1.0 / max(n, 1))), vx=np.zeros(n), vy=np.zeros(n),
                   vz=synth.f32(rng.normal(0, 0.1, n)), u=np.ones(n), gamma=5.0 / 3.0)
        got, L = run_gpu(crk, cfg, "f64", leaf_max=8)
        if n == 0:
            assert got["V"].size == 0
            continue
        V, rho = oracle.volume(cfg)
        assert normwise(got["V"], V) <= 1e-12
        if n >= 8:
            ref = oracle.hydro(cfg)
            assert normwise(got["a"], ref["a"]) <= 1e-12
            assert int(got["n_fallback"][0]) == ref["n_fallback"]


def short_list_case(lo, hi, seed):
    """209 random particles (three full tiles and a ragged one) with h for lo..hi
    neighbours: tiles whose longest list lies below, at and just past the gathered
    loop's unroll of eight (and lanes with no gather neighbour at lo = 0)."""
    rng = np.random.default_rng(seed)
    n = 3 * 64 + 17
    x, y, z = (synth.grid_round(rng.random(n)) for _ in range(3))
    H = synth.knn_support(x, y, z, rng.integers(lo, hi + 1, n))
    return dict(n=n, x=x, y=y, z=z, h=synth.f32(0.5 * H), m=synth.f32(rng.uniform(0.5, 1.5, n) / n),
                vx=synth.f32(rng.normal(0, 0.1, n)), vy=synth.f32(rng.normal(0, 0.1, n)),
                vz=synth.f32(rng.normal(0, 0.1, n)), u=synth.f32(np.exp(0.5 * rng.normal(size=n))),
                gamma=5.0 / 3.0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("lo,hi", [(0, 3), (5, 9), (14, 18)])
def test_short_lists_around_the_loop_unroll(crk, prec, lo, hi):
    """The gathered passes' outputs -- volumes and the raw moment sums (the
    latter for the GPU's own volumes) -- at the standard bars.  The solve that
    follows is left to the other tests: with five to nine neighbours the second
    moment is close to singular and its FP64 solution moves with the summation
    order alone."""
    cfg = short_list_case(lo, hi, seed=40 + lo)
    print(f"case short lists {lo}..{hi} prec={prec} n={cfg['n']}", flush=True)
    g = crk.gas_to_device(cfg, prec)
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec=prec)
    V, rho = crk.crk_volume(L, g, prec)
    *_, S = crk.crk_corrections(L, g, V, prec, store_sums=True)
    V_ref, rho_ref = oracle.volume(cfg)
    Vg = V.double().cpu().numpy()
    assert normwise(Vg, V_ref) <= TOL[prec]
    assert normwise(rho.double().cpu().numpy(), rho_ref) <= TOL[prec]
    M_ref, nnb_ref = oracle.moments(cfg, Vg)
    S = S.cpu().numpy()
    M = moments_from_stored_sums(S)
    for a, b in MOMENT_BLOCKS:
        assert normwise(M[:, a:b], M_ref[:, a:b]) <= TOL[prec], (a, b)
    if prec == "f64":
        assert np.array_equal(S[29].astype(np.int64), nnb_ref)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", [fallback_case, planar_case])
def test_singular_moment_fallback(crk, prec, case):
    """Few neighbours (fallback_case) and a singular second moment (planar_case)."""
    cfg = case()
    ref = oracle.hydro(cfg)
    assert ref["n_fallback"] > 0
    got, _ = run_gpu(crk, cfg, prec, leaf_max=32)
    assert int(got["n_fallback"][0]) == ref["n_fallback"]
    for k in KEYS:
        assert normwise(got[k], ref[k]) <= TOL[prec], k


def test_gravity_empty_and_tiny(crk):
    for n in (0, 1, 2, 63, 65):
        rng = np.random.default_rng(100 + n)
        cfg = dict(x=synth.grid_round(rng.random(n)), y=synth.grid_round(rng.random(n)),
                   z=synth.grid_round(rng.random(n)), m=synth.f32(rng.uniform(0.5, 1.5, n) / max(n, 1)),
                   G=1.0, eps=float(synth.f32(0.01)), r_cut=float(synth.f32(0.3)))
        a, _ = gravity_gpu(crk, cfg, "f64", leaf_max=16)
        assert a.shape == (n, 3)
        if n == 0:
            continue
        ref = oracle.gravity(cfg)
        bound = borderline_bound(cfg)
        assert np.all(np.abs(a - ref).max(1) <= 1e-12 * max(np.abs(ref).max(), 1e-300) + bound), n


def test_invalid_arguments(crk):
    x = torch.rand(100, dtype=torch.float64, device="cuda")
    h = torch.full((100,), 0.3, dtype=torch.float32, device="cuda")  # 2h >= 1/2
    with pytest.raises(crk.CrkError) as e:
        crk.crk_build_leaf_pairs(x, x, x, h, prec="f32")
    assert e.value.code == -1
    with pytest.raises(crk.CrkError):
        crk.crk_build_leaf_pairs(x, x, x, None, r_fixed=0.5, prec="f32")
    with pytest.raises(crk.CrkError):
        crk.crk_build_leaf_pairs(x, x, x, None, r_fixed=0.1, leaf_max=0, prec="f32")
    L = crk.crk_build_leaf_pairs(x, x, x, None, r_fixed=0.1, prec="f32")
    g = {"x": x, "y": x, "z": x, "h": h, "m": h}
    with pytest.raises(crk.CrkError) as e:
        crk.crk_volume(L, g, "f32")
    assert e.value.code == -4
    with pytest.raises(crk.CrkError):
        L.set_tuning(block_waves=3)
    with pytest.raises(crk.CrkError):
        L.set_tuning(kahan_chunk=3)  # not a power of two
    with pytest.raises(crk.CrkError):
        L.set_tuning(addr64=2)
    m = torch.ones(100, dtype=torch.float32, device="cuda")
    with pytest.raises(crk.CrkError):
        crk.sr_gravity(L, x, x, x, m, 1.0, 0.0, r_cut=0.2, prec="f32")  # r_cut > r_fixed


@pytest.mark.parametrize("tuning", [dict(persistent=0), dict(persistent=1, waves_per_cu=8),
                                    dict(persistent=1, waves_per_cu=32, xcd_groups=8, tile_order=0),
                                    dict(persistent=1, waves_per_cu=1, xcd_groups=16, block_waves=4),
                                    dict(persistent=0, xcd_groups=8, block_waves=4, tile_order=1)])
def test_work_queue_hands_out_every_tile_once(crk, tuning):
    """The persistent atomic queue (and the one-tile-per-wave form) hands every
    tile to exactly one wave, for grids smaller and larger than the work."""
    cfg, _ = oracle_full("C2", 21)
    g = crk.gas_to_device(cfg, "f32")
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec="f32")
    L.set_tuning(**tuning)
    v = L.queue_visits()
    torch.cuda.synchronize()
    assert v.numel() == L.stats()["tiles"] and bool((v == 1).all()), (tuning, v.min().item(), v.max().item())
    L.free()


# ---------------------------------------------------------------- caller-owned workspace
def test_workspace_protocol(crk):
    """crk_build_leaf_pairs through the C ABI with too small a workspace: it
    returns CRK_ENOSPC and sets ws_needed (first the part without the lists,
    then the exact total once the lists are counted), and the call with that
    much succeeds and gives the same results as a build through the wrapper."""
    import ctypes

    cfg, _ = oracle_full("C2", 21)
    g = crk.gas_to_device(cfg, "f32")
    lib = crk.load_library()
    n = cfg["n"]
    need = ctypes.c_size_t(0)
    out = ctypes.c_void_p()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(ws, nbytes, h=g["h"], r_fixed=0.0, needp=ctypes.byref(need)):
        return lib.crk_build_leaf_pairs(n, g["x"].data_ptr(), g["y"].data_ptr(), g["z"].data_ptr(),
                                        None if h is None else h.data_ptr(), r_fixed, 64, 1, 0.0, 0,
                                        None if ws is None else ws.data_ptr(), nbytes, needp,
                                        ctypes.byref(out), stream)

    assert call(None, 0, needp=None) == -1  # ws_needed is required
    assert call(None, 0) == crk.CRK_ENOSPC and not out.value
    part_a = need.value
    assert part_a > 0
    ws = torch.empty(part_a, dtype=torch.uint8, device="cuda")
    assert call(ws, part_a) == crk.CRK_ENOSPC and not out.value  # the lists come on top
    total = need.value
    assert total > part_a
    ws = torch.empty(total + 4096, dtype=torch.uint8, device="cuda")
    view = ws[256:]  # an aligned view works; an unaligned one is refused
    assert call(ws[1:], total) == -1
    assert call(view, total) == 0 and out.value
    assert need.value == total
    L = crk.Leaves(out, n, True, "f32", ws)
    got = crk.forward(L, g, cfg["gamma"], "f32")
    ref, _ = run_gpu(crk, cfg, "f32", leaf_max=64)
    torch.cuda.synchronize()
    for k in KEYS:
        assert np.array_equal(got[k].double().cpu().numpy(), ref[k]), k
    # one byte short: refused again with the same figure
    short = torch.empty(total - 1, dtype=torch.uint8, device="cuda")
    assert call(short, total - 1) == crk.CRK_ENOSPC and need.value == total
    # fixed-radius mode needs no lists: the first figure is exact
    assert call(None, 0, h=None, r_fixed=0.05) == crk.CRK_ENOSPC
    ws_g = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    assert call(ws_g, need.value, h=None, r_fixed=0.05) == 0
    lib.crk_leaves_free(out)
    L.free()
