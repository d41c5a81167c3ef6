"""Short-range gravity with the fitted particle-mesh polynomial, and its adjoint,
through the C ABI (GPU only).

The fitted coefficients come from the library's own fit (sr_gravity_fit_poly,
checked against the oracle's on the CPU); the forward pass with them is checked
against the brute-force oracle, and the adjoint sr_gravity_backward against the
oracle's forward-mode dual-number gradient of L = sum_i abar_i . a_i at sampled
coordinates, and in FP64 with torch.autograd.gradcheck.
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
GRAD_TOL = {"f64": 1e-10, "f32": 1e-5}


@pytest.fixture(scope="module")
def crk():
    import paper_2310_16122_amd as crk

    crk.load_library()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return crk


def device_case(crk, cfg, prec, leaf_max=128):
    dt = torch.float32 if prec == "f32" else torch.float64
    x, y, z = (torch.as_tensor(cfg[k]).cuda() for k in ("x", "y", "z"))
    m = torch.as_tensor(cfg["m"]).to(dt).cuda()
    L = crk.crk_build_leaf_pairs(x, y, z, None, r_fixed=cfg["r_cut"], leaf_max=leaf_max, leaf_min=16,
                                 split_extent=cfg["r_cut"], prec=prec)
    return x, y, z, m, L


def upstream(cfg, seed=5):
    return np.random.default_rng(seed).standard_normal((cfg["n"], 3))


def borderline_free(cfg, parts, margin=1e-6):
    """Coordinates whose particle has no pair within margin of the cutoff (the
    pair set is then the same for both precisions and for the oracle)."""
    P = np.stack([cfg["x"], cfg["y"], cfg["z"]], 1)
    keep = []
    for p in parts:
        d = P - P[p]
        d -= np.floor(d + 0.5)
        r = np.sqrt((d * d).sum(1))
        keep.append(not np.any(np.abs(r - cfg["r_cut"]) < margin))
    return np.array(keep)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("with_poly", [False, True])
def test_gravity_adjoint_against_oracle_dual(crk, prec, with_poly):
    cfg = synth.make_gravity(n_side=12)
    print(f"case gravity adjoint n={cfg['n']} prec={prec} poly={with_poly}", flush=True)
    poly = crk.sr_gravity_fit_poly(cfg["r_cut"] / 5, cfg["r_cut"]) if with_poly else None
    ab = upstream(cfg)
    rng = np.random.default_rng(7)
    parts = rng.choice(cfg["n"], 48, replace=False)
    kinds = rng.integers(0, 3, 48)
    sel = borderline_free(cfg, parts)
    parts, kinds = parts[sel], kinds[sel]
    gd, _ = oracle.gravity_grad(cfg, ab, parts, kinds, poly=poly)
    x, y, z, m, L = device_case(crk, cfg, prec)
    dt = m.dtype
    gx = crk.sr_gravity_backward(L, x, y, z, m, torch.as_tensor(ab).to(dt).cuda().contiguous(), cfg["G"],
                                 cfg["eps"], cfg["r_cut"], poly=poly, prec=prec)
    gx = gx.double().cpu().numpy()
    got = gx[parts, kinds]
    scale = np.abs(gx).max()
    err = np.abs(got - gd).max() / scale
    print("max err / max|gx|", err, flush=True)
    assert err <= GRAD_TOL[prec]
    L.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gravity_with_fitted_polynomial(crk, prec):
    cfg = synth.make_gravity(n_side=16)
    print(f"case gravity fitted poly n={cfg['n']} prec={prec}", flush=True)
    poly = crk.sr_gravity_fit_poly(cfg["r_cut"] / 5, cfg["r_cut"])
    ref = oracle.gravity(cfg, poly=poly)
    x, y, z, m, L = device_case(crk, cfg, prec)
    a = crk.sr_gravity(L, x, y, z, m, cfg["G"], cfg["eps"], cfg["r_cut"], poly=poly, prec=prec)
    a = a.double().cpu().numpy()
    # pairs on the cutoff may be taken or not: widen by their terms
    from tests.test_gpu_parity import borderline_bound

    bound = borderline_bound(cfg, poly=poly)
    err = np.abs(a - ref).max(1)
    assert np.all(err <= TOL[prec] * np.abs(ref).max() + bound), err.max()
    L.free()


def test_gravity_gradcheck_fp64(crk):
    cfg = synth.make_gravity(n_side=5)
    # a cutoff with no pair within 1e-5 of it, so that no perturbation moves a pair across
    P = np.stack([cfg["x"], cfg["y"], cfg["z"]], 1)
    d = P[:, None, :] - P[None, :, :]
    d -= np.floor(d + 0.5)
    r = np.sqrt((d * d).sum(2))
    rc = 0.3
    while np.any(np.abs(r - rc) < 1e-5):
        rc -= 1e-4
    cfg["r_cut"] = rc
    print(f"case gravity gradcheck n={cfg['n']} r_cut={rc}", flush=True)
    poly = crk.sr_gravity_fit_poly(cfg["r_cut"] / 5, cfg["r_cut"])
    x, y, z, m, L = device_case(crk, cfg, "f64", leaf_max=32)
    pos = torch.stack([x, y, z], 1).clone().requires_grad_(True)

    def f(p):
        return crk.SRGravity.apply(p, m, L, cfg["G"], cfg["eps"], cfg["r_cut"], poly, "f64")

    # the step 2^-20 keeps perturbed positions on the 2^-32 grid
    scale = float(f(pos).abs().max())
    assert torch.autograd.gradcheck(f, (pos,), eps=2.0 ** -20, atol=1e-6 * scale, rtol=1e-4)
    L.free()


def test_gravity_adjoint_bitwise_reproducible_and_schedule_independent(crk):
    cfg = synth.make_gravity(n_side=16)
    ab = torch.as_tensor(upstream(cfg)).float().cuda().contiguous()
    x, y, z, m, L = device_case(crk, cfg, "f32")
    args = (cfg["G"], cfg["eps"], cfg["r_cut"])
    g1 = crk.sr_gravity_backward(L, x, y, z, m, ab, *args, prec="f32")
    g2 = crk.sr_gravity_backward(L, x, y, z, m, ab, *args, prec="f32")
    L.set_tuning(persistent=1, waves_per_cu=8, tile_order=1)
    g3 = crk.sr_gravity_backward(L, x, y, z, m, ab, *args, prec="f32")
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(g1, g3)
    L.free()


def test_gravity_adjoint_full_size_c3(crk):
    """C3 at 2 x 128^3, leaf 512 (the benchmarked tree): the FP32 adjoint
    against the FP64 one over every particle, and the FP64 one against the
    oracle's dual-number gradient at 16 sampled coordinates."""
    cfg = synth.make_gravity()
    print(f"case gravity adjoint C3 n={cfg['n']}", flush=True)
    ab = upstream(cfg)
    res = {}
    for prec in ("f64", "f32"):
        x, y, z, m, L = device_case(crk, cfg, prec, leaf_max=512)
        g = crk.sr_gravity_backward(L, x, y, z, m, torch.as_tensor(ab).to(m.dtype).cuda().contiguous(),
                                    cfg["G"], cfg["eps"], cfg["r_cut"], prec=prec)
        res[prec] = g.double().cpu().numpy()
        L.free()
        del x, y, z, m, g
        torch.cuda.empty_cache()
    scale = np.abs(res["f64"]).max()
    # per particle: pairs on the cutoff may differ between the precisions
    rng = np.random.default_rng(23)
    parts = rng.choice(cfg["n"], 16, replace=False)
    kinds = rng.integers(0, 3, 16)
    sel = borderline_free(cfg, parts)
    gd, _ = oracle.gravity_grad(cfg, ab, parts[sel], kinds[sel])
    err64 = np.abs(res["f64"][parts[sel], kinds[sel]] - gd).max() / scale
    print("C3 adjoint FP64 vs dual", err64, flush=True)
    assert err64 <= GRAD_TOL["f64"]
    err32 = np.abs(res["f32"] - res["f64"]).max() / scale
    print("C3 adjoint FP32 vs FP64 normwise", err32, flush=True)
    assert err32 <= 1e-4
