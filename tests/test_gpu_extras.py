"""Extras pass (CRK density, gradients of v and u) and the force pass with the
artificial viscosity, through the C ABI, against the FP64 oracle (GPU only).

Bars as for the other passes: FP64 path <= 1e-12 and FP32 path <= 1e-5,
normwise per output array (max_i |y_i - y_ref_i| / max_i |y_ref_i|).
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
EXTRA_KEYS = ("rhoR", "dv", "du")


@pytest.fixture(scope="module")
def crk():
    import paper_2310_16122_amd as crk

    crk.load_library()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return crk


def normwise(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(y - ref).max() / np.abs(ref).max())


_ref = {}


def oracle_visc(name, n_side):
    key = (name, n_side)
    if key not in _ref:
        cfg = synth.make_config(name, n_side)
        _ref[key] = (cfg, oracle.hydro_visc(cfg))
    return _ref[key]


def gpu_visc(crk, cfg, prec, leaf_max=64):
    g = crk.gas_to_device(cfg, prec)
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=leaf_max, prec=prec)
    out = crk.forward_visc(L, g, cfg["gamma"], prec)
    torch.cuda.synchronize()
    host = {k: v.double().cpu().numpy() for k, v in out.items()}
    return host, L


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,n_side", [("C2", 21), ("C5", 24)])
def test_extras_and_viscous_forces_parity(crk, name, n_side, prec):
    cfg, ref = oracle_visc(name, n_side)
    print(f"case extras+visc {name} n={cfg['n']} prec={prec}", flush=True)
    got, L = gpu_visc(crk, cfg, prec)
    errs = {k: normwise(got[k], ref[k]) for k in EXTRA_KEYS + ("a", "dudt")}
    print(errs, flush=True)
    for k, e in errs.items():
        assert e <= TOL[prec], (k, e)
    T = got["totals"]
    lim = 1e-13 if prec == "f64" else 2e-6
    assert np.abs(T[:3]).max() <= lim * T[4]
    assert abs(T[3]) <= lim * T[5]
    # the viscosity changed the forces (this random velocity field is compressive somewhere)
    o0 = oracle.hydro(cfg)
    assert np.abs(ref["a"] - o0["a"]).max() > 1e-3 * np.abs(o0["a"]).max()
    L.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_extras_reproduce_linear_fields_gpu(crk, prec):
    """v = v0 + M x and u = u0 + g.x (a cluster away from the periodic seam):
    the GPU gradients are M and g at every particle."""
    from tests.test_oracle_pins import cluster_gas

    cfg = cluster_gas(n=3000, nbr=40)
    rng = np.random.default_rng(12)
    M = rng.normal(size=(3, 3))
    gu = rng.normal(size=3)
    X = np.stack([cfg["x"], cfg["y"], cfg["z"]], 1) - 0.5
    v = 0.3 + X @ M.T
    cfg.update(vx=synth.f32(v[:, 0]), vy=synth.f32(v[:, 1]), vz=synth.f32(v[:, 2]), u=synth.f32(2.0 + X @ gu))
    # the fields rounded to FP32 are no longer exactly linear: compare with the oracle on
    # the same inputs, and with M and g to the rounding of the inputs
    ref = oracle.hydro_visc(cfg)
    got, L = gpu_visc(crk, cfg, prec)
    for k in EXTRA_KEYS:
        assert normwise(got[k], ref[k]) <= TOL[prec], k
    assert np.abs(got["dv"] - M[None]).max() <= 1e-4 * np.abs(M).max()
    assert np.abs(got["du"] - gu[None]).max() <= 1e-4 * np.abs(gu).max()
    L.free()


def test_viscous_pass_bitwise_reproducible_and_schedule_independent(crk):
    cfg, _ = oracle_visc("C2", 21)
    g = crk.gas_to_device(cfg, "f32")
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec="f32")
    o1 = crk.forward_visc(L, g, cfg["gamma"], "f32")
    o2 = crk.forward_visc(L, g, cfg["gamma"], "f32")
    L.set_tuning(persistent=1, waves_per_cu=8, tile_order=1, block_waves=1)
    o3 = crk.forward_visc(L, g, cfg["gamma"], "f32")
    torch.cuda.synchronize()
    for k in ("rhoR", "dv", "du", "a", "dudt", "totals"):
        assert torch.equal(o1[k], o2[k]) and torch.equal(o1[k], o3[k]), k
    L.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_extras_and_viscosity_full_size_c2(crk, prec):
    """C2 at 128^3, leaf 128: every particle's extras and viscous forces against
    the oracle's chain over exact neighbour lists."""
    from tests.test_gpu_parity import oracle_listed

    cfg, ref = oracle_listed("C2")
    key = ("C2", "visc")
    if key not in _ref:
        off, idx = oracle.neighbour_lists(cfg)
        _ref[key] = oracle.visc_listed(cfg, off, idx, ref)
    rv = _ref[key]
    print(f"case extras+visc C2 full n={cfg['n']} prec={prec}", flush=True)
    got, L = gpu_visc(crk, cfg, prec, leaf_max=128)
    errs = {k: normwise(got[k], rv[k]) for k in EXTRA_KEYS + ("a", "dudt")}
    print(errs, flush=True)
    for k, e in errs.items():
        assert e <= TOL[prec], (k, e)
    L.free()


def test_invalid_viscosity_arguments(crk):
    cfg, _ = oracle_visc("C2", 21)
    g = crk.gas_to_device(cfg, "f64")
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec="f64")
    o = crk.forward(L, g, cfg["gamma"], "f64")
    corr = (o["A"], o["B"], o["dA"], o["dB"])
    _, dv, _ = crk.crk_extras(L, g, o["V"], corr, "f64")
    for bad in (dict(Cl=-1.0), dict(Cq=-0.5), dict(eps_q=0.0)):
        with pytest.raises(crk.CrkError):
            crk.crk_accel_energy_visc(L, g, o["V"], o["rho"], corr, dv, cfg["gamma"], "f64", **bad)
    with pytest.raises(crk.CrkError):
        crk.crk_accel_energy_visc(L, g, o["V"], o["rho"], corr, dv, 1.0, "f64")
    L.free()
