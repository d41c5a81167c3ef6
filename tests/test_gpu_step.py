"""Time step (device minimum) and kick-drift update through the C ABI, against
the oracle's plain definitions (GPU only)."""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crk():
    import paper_2310_16122_amd as crk

    crk.load_library()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return crk


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_timestep_and_kick_drift_against_oracle(crk, prec):
    cfg = synth.make_config("C2", n_side=21)
    print(f"case step C2 n={cfg['n']} prec={prec}", flush=True)
    ref = oracle.hydro(cfg)
    dt_ref = oracle.timestep(cfg, ref["a"], cfg["gamma"], 0.25, 0.25)
    g = crk.gas_to_device(cfg, prec)
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec=prec)
    out = crk.forward(L, g, cfg["gamma"], prec)
    dt = crk.crk_timestep(g, out["a"], cfg["gamma"], 0.25, 0.25, prec)
    dt_gpu = float(dt.item())
    tol = 1e-12 if prec == "f64" else 1e-5
    assert abs(dt_gpu - dt_ref) <= tol * dt_ref, (dt_gpu, dt_ref)
    # the kick-drift with the GPU's own step, against the oracle's update of the
    # GPU's inputs (the step and accelerations are inputs of this definition)
    host = {k: v.double().cpu().numpy() for k, v in g.items()}
    a = out["a"].double().cpu().numpy()
    du = out["dudt"].double().cpu().numpy()
    want = oracle.kick_drift(dict(cfg, **host), a, du, dt_gpu)
    crk.crk_kick_drift(g, out["a"], out["dudt"], dt, prec)
    torch.cuda.synchronize()
    for k in ("vx", "vy", "vz", "u"):
        got = g[k].double().cpu().numpy()
        assert np.abs(got - want[k]).max() <= (1e-15 if prec == "f64" else 1e-6) * np.abs(want[k]).max(), k
    for k in ("x", "y", "z"):
        got = g[k].cpu().numpy()
        d = got - want[k]
        d -= np.round(d)  # wrap-around of a value that lands on 1
        assert np.abs(d).max() <= 1e-15 if prec == "f64" else 1e-9, k
    L.free()


def test_timestep_is_deterministic_and_handles_empty(crk):
    cfg = synth.make_config("C2", n_side=16)
    g = crk.gas_to_device(cfg, "f32")
    a = torch.randn(cfg["n"], 3, generator=torch.Generator().manual_seed(1)).float().cuda()
    vals = {float(crk.crk_timestep(g, a, prec="f32").item()) for _ in range(5)}
    assert len(vals) == 1
    empty = {k: v[:0].contiguous() for k, v in g.items()}
    assert float(crk.crk_timestep(empty, a[:0].contiguous(), prec="f32").item()) == float("inf")


def test_simulation_steps_conserve_momentum_and_energy(crk):
    """A few kick-drift steps of the FP64 chain (lists rebuilt every step): total
    momentum is unchanged to roundoff, and each kick changes the total energy
    sum m (|v|^2/2 + u) by exactly dt sum m (v.a + du/dt) + dt^2/2 sum m |a|^2,
    whose first term the antisymmetric forces make vanish."""
    cfg = synth.make_config("C2", n_side=14)
    g = crk.gas_to_device(cfg, "f64")
    m = g["m"]
    p0 = None
    for step in range(3):
        L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec="f64")
        out = crk.forward(L, g, cfg["gamma"], "f64")
        T = out["totals"].cpu().numpy()
        assert np.abs(T[:3]).max() <= 1e-13 * T[4]
        assert abs(T[3]) <= 1e-13 * T[5]
        v = torch.stack([g["vx"], g["vy"], g["vz"]], 1)
        p = (m[:, None] * v).sum(0)
        if p0 is None:
            p0 = p
        assert (p - p0).abs().max().item() <= 1e-12 * float((m[:, None] * v.abs()).sum())
        e_before = float((m * (0.5 * (v * v).sum(1) + g["u"])).sum())
        dt = crk.crk_timestep(g, out["a"], cfg["gamma"], 0.1, 0.1, "f64")
        crk.crk_kick_drift(g, out["a"], out["dudt"], dt, "f64")
        v = torch.stack([g["vx"], g["vy"], g["vz"]], 1)
        e_after = float((m * (0.5 * (v * v).sum(1) + g["u"])).sum())
        d = float(dt.item())
        second = 0.5 * d * d * float((m * (out["a"] * out["a"]).sum(1)).sum())
        assert second > 0
        assert abs((e_after - e_before) - second) <= 1e-12 * e_before + 1e-6 * second
        L.free()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_lists_built_with_a_skin_serve_moved_particles(crk, prec, tol):
    """A handle built with a list skin and reused while the particles drift less
    than half the skin gives the passes of a fresh build on the moved positions
    (only the summation order differs), and so does it before they move."""
    cfg = synth.make_config("C2", n_side=16)
    print(f"case list reuse n={cfg['n']} prec={prec}", flush=True)
    g = crk.gas_to_device(cfg, prec)
    skin = 0.2 * 2.0 * float(np.mean(cfg["h"]))
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec=prec, skin=skin)
    keys = ("V", "rho", "A", "B", "dA", "dB", "a", "dudt")

    def compare(o1, o2):
        for k in keys:
            a = o1[k].double().cpu().numpy()
            b = o2[k].double().cpu().numpy()
            err = np.abs(a - b).max() / np.abs(b).max()
            assert err <= tol, (k, err)

    fresh0 = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec=prec)
    compare(crk.forward(L, g, cfg["gamma"], prec), crk.forward(fresh0, g, cfg["gamma"], prec))
    fresh0.free()
    disp = torch.zeros(2, dtype=torch.float64, device="cuda")
    steps = 0
    while True:
        out = crk.forward(L, g, cfg["gamma"], prec)
        dt = crk.crk_timestep(g, out["a"], cfg["gamma"], 0.05, 0.05, prec)
        before = disp.clone()
        crk.crk_kick_drift(g, out["a"], out["dudt"], dt, prec, disp=disp)
        steps += 1
        if float(disp[0]) >= 0.4 * skin or steps == 40:
            break
    assert steps >= 2 and float(disp[1]) == 0.0
    assert 0.0 < float(disp[0]) < 0.5 * skin, float(disp[0])
    # the largest drift of the last step is at least what the tracker added for it
    assert float(disp[0] - before[0]) > 0.0
    fresh = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec=prec)
    compare(crk.forward(L, g, cfg["gamma"], prec), crk.forward(fresh, g, cfg["gamma"], prec))
    st, sf = L.stats(), fresh.stats()
    assert st["pairs_gather"] == sf["pairs_gather"] and st["pairs_force"] == sf["pairs_force"]
    assert st["list_entries"] > sf["list_entries"]
    L.free()
    fresh.free()
