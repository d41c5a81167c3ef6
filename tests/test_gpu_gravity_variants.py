"""The exchange variants of the short-range gravity kernels (LDS broadcast,
scalar-register broadcast, cross-lane permute) through the C ABI: each gives
the LDS form's results bit for bit, forward and adjoint, on compact tiles
(box cull) and on spread tiles (fixed-point separations) (GPU only)."""

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


def spread_case(n=300, seed=5):
    rng = np.random.default_rng(seed)
    return dict(n=n, x=synth.grid_round(rng.random(n)), y=synth.grid_round(rng.random(n)),
                z=synth.grid_round(rng.random(n)), m=synth.f32(rng.uniform(0.5, 1.5, n) / n),
                G=1.0, eps=float(synth.f32(0.01)), r_cut=float(synth.f32(0.2)))


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", ["clustered", "spread"])
def test_exchange_variants_are_bitwise_equal(crk, prec, case):
    cfg = synth.make_gravity(n_side=16) if case == "clustered" else spread_case()
    print(f"case gravity exchange {case} n={cfg['n']} prec={prec}", flush=True)
    dt = torch.float32 if prec == "f32" else torch.float64
    x, y, z = (torch.as_tensor(cfg[k]).cuda() for k in ("x", "y", "z"))
    m = torch.as_tensor(cfg["m"]).to(dt).cuda()
    ga = torch.randn(cfg["n"], 3, generator=torch.Generator().manual_seed(2)).to(dt).cuda()
    L = crk.crk_build_leaf_pairs(x, y, z, None, r_fixed=cfg["r_cut"], leaf_max=128, leaf_min=16,
                                 split_extent=cfg["r_cut"], prec=prec)
    poly = crk.sr_gravity_fit_poly(cfg["r_cut"] / 5, cfg["r_cut"])
    ref = oracle.gravity(cfg, poly=poly)
    out = {}
    for ex in (0, 1, 2):
        L.set_tuning(exchange=ex)
        for p in (None, poly):
            a = crk.sr_gravity(L, x, y, z, m, cfg["G"], cfg["eps"], cfg["r_cut"], poly=p, prec=prec)
            g = crk.sr_gravity_backward(L, x, y, z, m, ga, cfg["G"], cfg["eps"], cfg["r_cut"], poly=p, prec=prec)
            out[(ex, p is None)] = (a, g)
    torch.cuda.synchronize()
    for ex in (1, 2):
        for nop in (True, False):
            assert torch.equal(out[(ex, nop)][0], out[(0, nop)][0]), (ex, nop, "forward")
            assert torch.equal(out[(ex, nop)][1], out[(0, nop)][1]), (ex, nop, "adjoint")
    # and the shared result is the oracle's
    from tests.test_gpu_parity import borderline_bound

    a = out[(2, False)][0].double().cpu().numpy()
    tol = 1e-12 if prec == "f64" else 1e-5
    err = np.abs(a - ref).max(1)
    assert np.all(err <= tol * np.abs(ref).max() + borderline_bound(cfg, poly=poly)), err.max()
    L.free()
