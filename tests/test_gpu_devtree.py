"""Leaf build on the device (crk_build_leaf_pairs_device), through the C ABI
(GPU only).

A neighbour list holds every j != i whose separation passes the list test
(r^2 < max(H_i, H_j)^2 with a fixed relative margin), whatever tree found the
candidates, so the device build (Morton octree) and the host build (recursive
coordinate bisection) must give every particle the same list: the counts of
list entries and of pairs agree exactly, and the pass results agree to the
rounding of the summation order.  Against the oracle the bars are those of the
other pass tests: FP64 <= 1e-12, FP32 <= 1e-5 normwise.
"""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
# host and device build: the same pairs summed in another order
ORDER_TOL = {"f64": 1e-13, "f32": 2e-6}
KEYS = ("V", "rho", "A", "B", "dA", "dB", "a", "dudt")


@pytest.fixture(scope="module")
def crk():
    import paper_2310_16122_amd as crk

    crk.load_library()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return crk


def normwise(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    err = np.abs(y - ref).max()
    return float(err / scale) if scale > 0 else float(err)


def hydro_run(crk, cfg, prec, device, leaf_max=64, skin=0.0):
    g = crk.gas_to_device(cfg, prec)
    build = crk.crk_build_leaf_pairs_device if device else crk.crk_build_leaf_pairs
    L = build(g["x"], g["y"], g["z"], g["h"], leaf_max=leaf_max, prec=prec, skin=skin)
    out = crk.forward(L, g, cfg["gamma"], prec)
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in out.items()}, L


def gravity_run(crk, cfg, prec, device, leaf_max=256):
    dt = torch.float32 if prec == "f32" else torch.float64
    x, y, z = (torch.as_tensor(cfg[k]).cuda() for k in ("x", "y", "z"))
    m = torch.as_tensor(cfg["m"]).to(dt).cuda()
    if device:
        L = crk.crk_build_leaf_pairs_device(x, y, z, None, r_fixed=cfg["r_cut"], leaf_max=leaf_max, prec=prec)
    else:
        L = crk.crk_build_leaf_pairs(x, y, z, None, r_fixed=cfg["r_cut"], leaf_max=leaf_max, leaf_min=16,
                                     split_extent=cfg["r_cut"], prec=prec)
    a = crk.sr_gravity(L, x, y, z, m, cfg["G"], cfg["eps"], cfg["r_cut"], prec=prec)
    return a.double().cpu().numpy(), L


def borderline(cfg):
    """Per-particle sum of |pair term| over pairs within 2^-20 (relative, in r^2)
    of the cutoff, where FP32 and FP64 may decide differently."""
    from scipy.spatial import cKDTree

    P = np.stack([cfg["x"], cfg["y"], cfg["z"]], 1)
    rc = cfg["r_cut"]
    lo, hi = rc * np.sqrt(1 - 2.0 ** -20), rc * np.sqrt(1 + 2.0 ** -20)
    pairs = cKDTree(P, boxsize=1.0).query_pairs(hi, output_type="ndarray")
    b = np.zeros(len(P))
    if len(pairs) == 0:
        return b
    d = P[pairs[:, 0]] - P[pairs[:, 1]]
    d -= np.floor(d + 0.5)
    r = np.sqrt((d * d).sum(1))
    sel = r >= lo
    f = cfg["G"] * r[sel] / (r[sel] ** 2 + cfg["eps"] ** 2) ** 1.5
    np.add.at(b, pairs[sel, 0], cfg["m"][pairs[sel, 1]] * f)
    np.add.at(b, pairs[sel, 1], cfg["m"][pairs[sel, 0]] * f)
    return b


_ref = {}


def oracle_case(name, n_side):
    if (name, n_side) not in _ref:
        cfg = synth.make_config(name, n_side)
        _ref[(name, n_side)] = (cfg, oracle.hydro(cfg))
    return _ref[(name, n_side)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,n_side", [("C1", None), ("C2", 21), ("C5", 24)])
def test_device_build_forward_parity(crk, name, n_side, prec):
    cfg, ref = oracle_case(name, n_side)
    print(f"case {name} n_side={n_side} prec={prec} n={cfg['n']}", flush=True)
    got, L = hydro_run(crk, cfg, prec, device=True)
    errs = {k: normwise(got[k], ref[k]) for k in KEYS}
    print(errs, flush=True)
    for k in KEYS:
        assert errs[k] <= TOL[prec], (k, errs[k])
    assert int(got["n_fallback"][0]) == ref["n_fallback"]
    st = L.stats()
    assert st["pairs_gather"] == oracle.count_pairs(cfg, 0)[0]
    assert st["pairs_force"] == oracle.count_pairs(cfg, 1)[0]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("leaf_max,skin", [(16, 0.0), (64, 0.01), (1024, 0.0)])
def test_device_build_lists_match_host_build(crk, prec, leaf_max, skin):
    cfg, _ = oracle_case("C2", 21)
    print(f"case C2/21 prec={prec} leaf_max={leaf_max} skin={skin}", flush=True)
    dev, Ld = hydro_run(crk, cfg, prec, device=True, leaf_max=leaf_max, skin=skin)
    host, Lh = hydro_run(crk, cfg, prec, device=False, leaf_max=leaf_max, skin=skin)
    sd, sh = Ld.stats(), Lh.stats()
    print({k: (sd[k], sh[k]) for k in sd}, flush=True)
    for k in ("list_entries", "pairs_gather", "pairs_force", "tiles"):
        assert sd[k] == sh[k], k
    for k in KEYS:
        assert normwise(dev[k], host[k]) <= ORDER_TOL[prec], k


def test_device_build_is_deterministic(crk):
    cfg, _ = oracle_case("C2", 21)
    a, La = hydro_run(crk, cfg, "f32", device=True)
    b, Lb = hydro_run(crk, cfg, "f32", device=True)
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
    assert torch.equal(La.perm(), Lb.perm())


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_device_build_gravity(crk, prec):
    cfg = synth.make_gravity(n_side=24)
    print(f"case gravity n={cfg['n']} prec={prec}", flush=True)
    ref = oracle.gravity(cfg)
    a, L = gravity_run(crk, cfg, prec, device=True)
    err = np.abs(a - ref).max(1)
    scale = np.abs(ref).max()
    assert np.all(err <= TOL[prec] * scale + borderline(cfg)), err.max() / scale
    assert L.stats()["pairs_force"] == oracle.count_pairs(cfg, 2, r_fixed=cfg["r_cut"])[0]


def test_device_build_coincident_clump(crk):
    """More particles than leaf_max inside one finest octree cell (2^-21 of the
    box per side): the build cuts that cell into runs of leaf_max."""
    rng = np.random.default_rng(31)
    n_clump, n_bg = 700, 1300
    c = 0.4321
    x, y, z = (synth.grid_round(np.concatenate([c + 1e-8 * rng.random(n_clump), rng.random(n_bg)]))
               for _ in range(3))
    n = n_clump + n_bg
    cfg = dict(n=n, x=x, y=y, z=z, m=synth.f32(rng.uniform(0.5, 1.5, n) / n), G=1.0,
               eps=float(synth.f32(0.01)), r_cut=float(synth.f32(0.1)))
    ref = oracle.gravity(cfg)
    a, L = gravity_run(crk, cfg, "f64", device=True, leaf_max=64)
    assert L.stats()["leaves"] >= n_clump // 64
    err = np.abs(a - ref).max(1)
    assert np.all(err <= 1e-12 * np.abs(ref).max() + borderline(cfg)), err.max()
    assert L.stats()["pairs_force"] == oracle.count_pairs(cfg, 2, r_fixed=cfg["r_cut"])[0]


def test_device_build_tiny_inputs(crk):
    for n in (0, 1, 5, 63, 65):
        rng = np.random.default_rng(n)
        cfg = dict(n=n, x=synth.grid_round(rng.random(n)), y=synth.grid_round(rng.random(n)),
                   z=synth.grid_round(rng.random(n)), h=synth.f32(np.full(n, 0.2)),
                   m=synth.f32(np.full(n, 1.0 / max(n, 1))), vx=np.zeros(n), vy=np.zeros(n),
                   vz=synth.f32(rng.normal(0, 0.1, n)), u=np.ones(n), gamma=5.0 / 3.0)
        print(f"case tiny n={n}", flush=True)
        got, L = hydro_run(crk, cfg, "f64", device=True, leaf_max=8)
        if n == 0:
            assert got["V"].size == 0
            continue
        V, _ = oracle.volume(cfg)
        assert normwise(got["V"], V) <= 1e-12
        if n >= 8:
            ref = oracle.hydro(cfg)
            assert normwise(got["a"], ref["a"]) <= 1e-12


def test_device_build_invalid_inputs(crk):
    n = 200
    x = torch.rand(n, dtype=torch.float64, device="cuda")
    h = torch.full((n,), 0.01, dtype=torch.float32, device="cuda")
    bad_x = x.clone()
    bad_x[17] = float("nan")
    bad_h = h.clone()
    bad_h[3] = 0.0
    big_h = torch.full((n,), 0.3, dtype=torch.float32, device="cuda")  # 2h >= 1/2
    for args, kw in (((bad_x, x, x, h), {}), ((x, x, x, bad_h), {}), ((x, x, x, big_h), {}),
                     ((x, x, x, h), {"leaf_max": 1025}), ((x, x, x, h), {"leaf_max": 0}),
                     ((x, x, x, None), {"r_fixed": 0.5})):
        with pytest.raises(crk.CrkError) as e:
            crk.crk_build_leaf_pairs_device(*args, prec="f32", **kw)
        assert e.value.code == -1, kw
    # no error is left behind for the next call
    L = crk.crk_build_leaf_pairs_device(x, x, x, h, prec="f32")
    assert L.stats()["tiles"] == (n + 63) // 64


def test_device_build_workspace_protocol(crk):
    """Through the C ABI: CRK_ENOSPC with the size needed so far, until the
    workspace suffices; the result equals the wrapper's build bit for bit."""
    cfg, _ = oracle_case("C2", 21)
    g = crk.gas_to_device(cfg, "f32")
    lib = crk.load_library()
    n = cfg["n"]
    need = ctypes.c_size_t(0)
    out = ctypes.c_void_p()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(ws, nbytes):
        return lib.crk_build_leaf_pairs_device(n, g["x"].data_ptr(), g["y"].data_ptr(), g["z"].data_ptr(),
                                               g["h"].data_ptr(), 0.0, 64, 0,
                                               None if ws is None else ws.data_ptr(), nbytes,
                                               ctypes.byref(need), ctypes.byref(out), stream)

    assert call(None, 0) == crk.CRK_ENOSPC and not out.value
    sizes = [need.value]
    ws = None
    for _ in range(3):
        ws = torch.empty(sizes[-1], dtype=torch.uint8, device="cuda")
        code = call(ws, sizes[-1])
        if code == 0:
            break
        assert code == crk.CRK_ENOSPC and not out.value
        assert need.value > sizes[-1]
        sizes.append(need.value)
    assert code == 0 and out.value, sizes
    print("workspace sizes", sizes, flush=True)
    L = crk.Leaves(out, n, True, "f32", ws)
    a = crk.forward(L, g, cfg["gamma"], "f32")
    b = crk.forward(crk.crk_build_leaf_pairs_device(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec="f32"),
                    g, cfg["gamma"], "f32")
    for k in KEYS:
        assert torch.equal(a[k], b[k]), k


def test_device_build_full_size(crk):
    """C2 at 128^3 (FP32, leaf 128): the device build's lists match the host
    build's, and the passes agree; build times printed."""
    cfg = synth.make_config("C2")
    print(f"case C2 full n={cfg['n']}", flush=True)
    dev, Ld = hydro_run(crk, cfg, "f32", device=True, leaf_max=128)
    host, Lh = hydro_run(crk, cfg, "f32", device=False, leaf_max=128)
    sd, sh = Ld.stats(), Lh.stats()
    print("device build", sd, "\nhost build", sh, flush=True)
    for k in ("list_entries", "pairs_gather", "pairs_force"):
        assert sd[k] == sh[k], k
    for k in KEYS:
        assert normwise(dev[k], host[k]) <= ORDER_TOL["f32"], k
