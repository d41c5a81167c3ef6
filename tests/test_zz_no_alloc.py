"""The allocation-free force pass against the one on the handle's workspace,
through the C ABI (GPU only).

crk_accel_energy_noalloc takes its scratch (neighbour records and the FP64
totals partials) from a fixed device array instead of the handle's workspace
and runs the same kernels, so its outputs must equal crk_accel_energy's bit
for bit.  Two calls in a row, the second on fewer particles, check that what
the first call left in the shared array does not leak into the second; a
particle count beyond the array is refused with an error before any launch.
"""

import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def crk():
    import paper_2310_16122_amd as crk

    crk.load_library()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return crk


def chain(crk, cfg, prec):
    g = crk.gas_to_device(cfg, prec)
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec=prec)
    V, rho = crk.crk_volume(L, g, prec)
    corr = crk.crk_corrections(L, g, V, prec)
    return g, L, V, rho, corr


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_force_pass_equals_workspace_form(crk, prec):
    # larger input first, then a smaller one: the second call reuses the array
    for n_side in (24, 14):
        cfg = synth.make_config("C4", n_side=n_side)
        print(f"case noalloc C4 n={cfg['n']} prec={prec}", flush=True)
        g, L, V, rho, corr = chain(crk, cfg, prec)
        ref = crk.crk_accel_energy(L, g, V, rho, corr, cfg["gamma"], prec)
        got = crk.crk_accel_energy_noalloc(L, g, V, rho, corr, cfg["gamma"], prec)
        torch.cuda.synchronize()
        for name, r, y in zip(("a", "dudt", "totals"), ref, got):
            assert torch.equal(r, y), (n_side, prec, name)
        assert float(ref[2][4]) > 0.0  # a real force field, not an empty one
        L.free()


def test_noalloc_refuses_inputs_beyond_the_static_scratch(crk):
    # FP64 records are 256 bytes per particle: 72^3 particles need more than
    # the 80 MiB array, and the call must fail before launching anything
    cfg = synth.make_config("C4", n_side=72)
    print(f"case noalloc refusal n={cfg['n']}", flush=True)
    g, L, V, rho, corr = chain(crk, cfg, "f64")
    with pytest.raises(crk.CrkError) as e:
        crk.crk_accel_energy_noalloc(L, g, V, rho, corr, cfg["gamma"], "f64")
    assert e.value.code == -1 and "static" in str(e.value)
    # the workspace form still runs on the same handle
    a, du, tot = crk.crk_accel_energy(L, g, V, rho, corr, cfg["gamma"], "f64")
    torch.cuda.synchronize()
    assert np.isfinite(a.cpu().numpy()).all()
    L.free()
