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
