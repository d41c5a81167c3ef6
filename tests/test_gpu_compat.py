"""Force pass with the compatible energy partition
(crk_accel_energy_compatible), through the C ABI, against the FP64 oracle
(GPU only).

Each pair's work W_ij = (v_j - v_i) . F_ij goes f_ij W_ij to i and
(1 - f_ij) W_ij to j, f_ij = 1/2 [1 + sgn(W_ij) (u_j - u_i) / (|u_j - u_i| +
eps_u (u_i + u_j))].  Bars as for the other passes: FP64 <= 1e-12 and FP32 <=
1e-5 normwise; the accelerations are those of the symmetric pass bit for bit.
"""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
EPS_U = 0.1


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


def oracle_case(name, n_side, visc):
    key = (name, n_side, visc)
    if key not in _ref:
        cfg = synth.make_config(name, n_side)
        o = oracle.hydro_visc(cfg) if visc else oracle.hydro(cfg)
        corr = (o["A"], o["B"], o["dA"], o["dB"])
        a, du = oracle.accel_compat(cfg, o["V"], o["rho"], corr, eps_u=EPS_U, dv=o["dv"] if visc else None)
        _ref[key] = (cfg, a, du)
    return _ref[key]


def gpu_chain(crk, cfg, prec, visc):
    g = crk.gas_to_device(cfg, prec)
    L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=64, prec=prec)
    V, rho = crk.crk_volume(L, g, prec)
    corr = crk.crk_corrections(L, g, V, prec)
    dv = crk.crk_extras(L, g, V, corr, prec)[1] if visc else None
    return g, L, V, rho, corr, dv


@pytest.mark.parametrize("visc", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,n_side", [("C1", None), ("C2", 21)])
def test_compatible_partition_parity(crk, name, n_side, prec, visc):
    cfg, a_ref, du_ref = oracle_case(name, n_side, visc)
    print(f"case {name} n_side={n_side} prec={prec} visc={visc} n={cfg['n']}", flush=True)
    g, L, V, rho, corr, dv = gpu_chain(crk, cfg, prec, visc)
    a, du, T = crk.crk_accel_energy_compatible(L, g, V, rho, corr, eps_u=EPS_U, dv=dv, prec=prec,
                                               visc=crk.VISC_DEFAULT if visc else None)
    ea = normwise(a.double().cpu().numpy(), a_ref)
    ed = normwise(du.double().cpu().numpy(), du_ref)
    print({"a": ea, "dudt": ed}, flush=True)
    assert ea <= TOL[prec] and ed <= TOL[prec]
    # the forces are those of the symmetric pass, bit for bit
    if visc:
        a_s, du_s, _ = crk.crk_accel_energy_visc(L, g, V, rho, corr, dv, prec=prec)
    else:
        a_s, du_s, _ = crk.crk_accel_energy(L, g, V, rho, corr, prec=prec)
    assert torch.equal(a, a_s)
    # total energy conserved (FP64 totals of the pass)
    T = T.cpu().numpy()
    lim = 1e-13 if prec == "f64" else 2e-6
    assert abs(T[3]) <= lim * T[5]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_equal_energies_give_the_symmetric_split_bitwise(crk, prec):
    cfg = dict(synth.make_config("C2", 21))
    cfg["u"] = np.full(cfg["n"], 1.25)
    g, L, V, rho, corr, _ = gpu_chain(crk, cfg, prec, False)
    a, du, _ = crk.crk_accel_energy_compatible(L, g, V, rho, corr, eps_u=EPS_U, prec=prec)
    a_s, du_s, _ = crk.crk_accel_energy(L, g, V, rho, corr, prec=prec)
    assert torch.equal(a, a_s) and torch.equal(du, du_s)


def test_compatible_partition_arguments(crk):
    cfg = synth.make_config("C1")
    g, L, V, rho, corr, dv = gpu_chain(crk, cfg, "f32", True)
    for kw in (dict(eps_u=-1.0), dict(eps_u=float("inf")), dict(eps_u=0.1, dv=dv),
               dict(eps_u=0.1, visc=crk.VISC_DEFAULT)):
        with pytest.raises(crk.CrkError) as e:
            crk.crk_accel_energy_compatible(L, g, V, rho, corr, prec="f32", **kw)
        assert e.value.code == -1, kw
    # eps_u = 0: the whole share to one side wherever the energies differ; still conservative
    a, du, T = crk.crk_accel_energy_compatible(L, g, V, rho, corr, eps_u=0.0, prec="f32")
    T = T.cpu().numpy()
    assert abs(T[3]) <= 2e-6 * T[5]


_full = {}


def test_compatible_partition_full_size_every_particle(crk):
    """C2 at 128^3 (leaf 128, the benchmark's build): every particle's a and
    du/dt against the oracle's chain over exact neighbour lists, FP64 and FP32."""
    if "C2" not in _full:
        cfg = synth.make_config("C2")
        off, idx = oracle.neighbour_lists(cfg)
        ref = oracle.hydro_listed(cfg, off, idx)
        _full["C2"] = (cfg, oracle.compat_listed(cfg, off, idx, ref, eps_u=EPS_U))
    cfg, (a_ref, du_ref) = _full["C2"]
    for prec in ("f64", "f32"):
        print(f"case C2 full n={cfg['n']} prec={prec}", flush=True)
        g = crk.gas_to_device(cfg, prec)
        L = crk.crk_build_leaf_pairs(g["x"], g["y"], g["z"], g["h"], leaf_max=128, prec=prec)
        V, rho = crk.crk_volume(L, g, prec)
        corr = crk.crk_corrections(L, g, V, prec)
        a, du, T = crk.crk_accel_energy_compatible(L, g, V, rho, corr, eps_u=EPS_U, prec=prec)
        ea = normwise(a.double().cpu().numpy(), a_ref)
        ed = normwise(du.double().cpu().numpy(), du_ref)
        print({"a": ea, "dudt": ed}, flush=True)
        assert ea <= TOL[prec] and ed <= TOL[prec], (prec, ea, ed)
        L.free()
        del g, L, V, rho, corr, a, du
        torch.cuda.empty_cache()
