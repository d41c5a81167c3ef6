"""FP64 CPU oracle for the CRK-SPH pair passes and short-range gravity.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library (``paper_2310_16122_amd``)
and never importing it.  The arithmetic lives in ``crk_oracle.cpp`` (plain C++,
FP64, brute-force neighbour search); this module compiles it with g++ and
wraps it with ctypes and numpy.

Reading of the paper (which names the passes and cites the method without
printing its equations): linear conservative reproducing-kernel SPH with a
Wendland C4 kernel of support 2h, a volume-based density, an ideal-gas
pressure and antisymmetrised corrected-kernel gradients; short-range gravity is
Plummer-softened Newtonian attraction cut at r_c.  The header of
``crk_oracle.cpp`` writes every formula out.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crk_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MOMENT_NAMES = (["m0"] + [f"m1_{a}" for a in "xyz"] +
                [f"m2_{p}" for p in ("xx", "xy", "xz", "yy", "yz", "zz")] +
                [f"g0_{c}" for c in "xyz"] +
                [f"g1_{a}{c}" for a in "xyz" for c in "xyz"] +
                [f"g2_{p}{c}" for p in ("xx", "xy", "xz", "yy", "yz", "zz") for c in "xyz"])


def build(force=False):
    """Compile the oracle (g++ -O3 -march=x86-64-v3 -fopenmp; portable to any AVX2 host).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-std=c++17", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_volume.argtypes = [I64, P, P, P, P, P, I64, P, P, P]
        lib.oracle_moments.argtypes = [I64, P, P, P, P, P, I64, P, P, P]
        lib.oracle_corrections.argtypes = [I64, P, P, P, P, P, I64, P, P, P, P, P]
        lib.oracle_corrections.restype = I64
        lib.oracle_accel.argtypes = [I64] + [P] * 15 + [D, I64, P, P, P, P, P]
        lib.oracle_totals.argtypes = [I64] + [P] * 9
        lib.oracle_hydro_targets.argtypes = [I64] + [P] * 9 + [D, I64, P] + [P] * 10
        lib.oracle_hydro_targets.restype = I64
        lib.oracle_gravity.argtypes = [I64, P, P, P, P, D, D, D, P, I64, P, P, P, P]
        lib.oracle_count_pairs.argtypes = [I64, P, P, P, P, ctypes.c_int, D, I64, P, P]
        lib.oracle_count_pairs.restype = I64
        lib.oracle_kernel.argtypes = [I64, P, D, P, P]
        lib.oracle_grad.argtypes = [I64] + [P] * 9 + [D, P, P, I64, P, P, D, P, P, P]
        lib.oracle_flops.argtypes = [P]
        lib.oracle_flops_selftest.argtypes = [P]
        lib.oracle_passes_listed.argtypes = [I64] + [P] * 9 + [D] + [P] * 6 + [I64, P, P, P,
                                                                               ctypes.c_int] + [P] * 4
        lib.oracle_passes_listed.restype = I64
        lib.oracle_hydro_listed.argtypes = [I64] + [P] * 9 + [D] + [P] * 12
        lib.oracle_hydro_listed.restype = I64
        lib.oracle_gravity_listed.argtypes = [I64, P, P, P, P, D, D, D, P, I64, P, P, P, ctypes.c_int,
                                              P, P, P]
        lib.oracle_long_range_force.argtypes = [I64, P, D, P]
        lib.oracle_extras.argtypes = [I64] + [P] * 14 + [I64, P, P, P, P]
        lib.oracle_visc_listed.argtypes = [I64] + [P] * 9 + [D, D, D, D] + [P] * 15
        lib.oracle_accel_visc.argtypes = [I64] + [P] * 16 + [D, D, D, D, I64, P, P, P, P, P]
        lib.oracle_compat_listed.argtypes = [I64] + [P] * 9 + [D, D] + [P] * 12
        lib.oracle_grad_visc.argtypes = [I64] + [P] * 9 + [D, D, D, D, P, P, I64, P, P, D, P, P]
        lib.oracle_accel_compat.argtypes = [I64] + [P] * 16 + [D, D, D, D, D, I64, P, P, P, P, P]
        lib.oracle_gravity_grad.argtypes = [I64, P, P, P, P, D, D, D, P, P, I64, P, P, D, P, P]
        _lib = lib
    return _lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def threads():
    return _load().oracle_threads()


def kernel(r, h):
    """Wendland C4 W(r, h) and F(r, h) with grad_i W = F x_ij."""
    r = _c(r)
    W = np.empty_like(r)
    F = np.empty_like(r)
    _load().oracle_kernel(r.size, _p(r), float(h), _p(W), _p(F))
    return W, F


def _targets(targets, n):
    if targets is None:
        return None, n
    t = _c(targets, np.int64)
    return t, t.size


def volume(g, targets=None):
    """V_i = 1/S_i and rho_i = m_i S_i (brute force)."""
    x, y, z, h, m = (_c(g[k]) for k in ("x", "y", "z", "h", "m"))
    t, nt = _targets(targets, x.size)
    V = np.empty(nt)
    rho = np.empty(nt)
    _load().oracle_volume(x.size, _p(x), _p(y), _p(z), _p(h), _p(m), nt, _p(t), _p(V), _p(rho))
    return V, rho


def moments(g, V, targets=None):
    """The 40 raw moment sums per particle and the neighbour count."""
    x, y, z, h = (_c(g[k]) for k in ("x", "y", "z", "h"))
    V = _c(V)
    t, nt = _targets(targets, x.size)
    M = np.empty((nt, 40))
    nnb = np.empty(nt, dtype=np.int32)
    _load().oracle_moments(x.size, _p(x), _p(y), _p(z), _p(h), _p(V), nt, _p(t), _p(M), _p(nnb))
    return M, nnb


def corrections(g, V, targets=None):
    """(A, B[n,3], dA[n,3], dB[n,3,3], n_fallback); dB[i,a,c] = d_c B^a."""
    x, y, z, h = (_c(g[k]) for k in ("x", "y", "z", "h"))
    V = _c(V)
    t, nt = _targets(targets, x.size)
    A = np.empty(nt)
    B = np.empty((nt, 3))
    dA = np.empty((nt, 3))
    dB = np.empty((nt, 3, 3))
    nf = _load().oracle_corrections(x.size, _p(x), _p(y), _p(z), _p(h), _p(V), nt, _p(t),
                                    _p(A), _p(B), _p(dA), _p(dB))
    return A, B, dA, dB, int(nf)


def accel(g, V, rho, corr, targets=None):
    """Accelerations a[n,3] and du/dt[n] given V, rho and corrections of all particles."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    V, rho = _c(V), _c(rho)
    A, B, dA, dB = (_c(c) for c in corr[:4])
    t, nt = _targets(targets, arr[0].size)
    a = np.empty((3, nt))
    du = np.empty(nt)
    _load().oracle_accel(arr[0].size, *[_p(v) for v in arr], _p(V), _p(rho), _p(A), _p(B),
                         _p(dA), _p(dB), float(g["gamma"]), nt, _p(t), _p(a[0]), _p(a[1]),
                         _p(a[2]), _p(du))
    return a.T.copy(), du


VISC_DEFAULT = dict(Cl=1.0, Cq=2.0, eps_q=0.01)


def extras(g, V, corr, targets=None):
    """CRK density rhoR[n], velocity gradients dv[n,3,3] (dv[i,a,c] = d_c v^a) and
    energy gradients du[n,3] over the gather support (crk_oracle.cpp)."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    A, B, dA, dB = (_c(c) for c in corr[:4])
    t, nt = _targets(targets, arr[0].size)
    rhoR = np.empty(nt)
    dv = np.empty((nt, 3, 3))
    du = np.empty((nt, 3))
    _load().oracle_extras(arr[0].size, *[_p(v) for v in arr], _p(_c(V)), _p(A), _p(B), _p(dA), _p(dB),
                          nt, _p(t), _p(rhoR), _p(dv), _p(du))
    return dict(rhoR=rhoR, dv=dv, du=du)


def accel_visc(g, V, rho, corr, dv, targets=None, Cl=1.0, Cq=2.0, eps_q=0.01):
    """Accelerations and du/dt with the artificial viscosity fed by the
    velocity gradients dv [n,3,3] (all particles)."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    A, B, dA, dB = (_c(c) for c in corr[:4])
    t, nt = _targets(targets, arr[0].size)
    a = np.empty((3, nt))
    du = np.empty(nt)
    _load().oracle_accel_visc(arr[0].size, *[_p(v) for v in arr], _p(_c(V)), _p(_c(rho)), _p(A), _p(B),
                              _p(dA), _p(dB), _p(_c(dv)), float(Cl), float(Cq), float(eps_q),
                              float(g["gamma"]), nt, _p(t), _p(a[0]), _p(a[1]), _p(a[2]), _p(du))
    return a.T.copy(), du


def accel_compat(g, V, rho, corr, eps_u=0.1, dv=None, targets=None, Cl=1.0, Cq=2.0, eps_q=0.01):
    """Accelerations and du/dt with the compatible energy partition (weights
    f_ij of the pair work, see crk_oracle.cpp), with the artificial viscosity
    when the velocity gradients dv [n,3,3] are given."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    A, B, dA, dB = (_c(c) for c in corr[:4])
    t, nt = _targets(targets, arr[0].size)
    a = np.empty((3, nt))
    du = np.empty(nt)
    _load().oracle_accel_compat(arr[0].size, *[_p(v) for v in arr], _p(_c(V)), _p(_c(rho)), _p(A), _p(B),
                                _p(dA), _p(dB), None if dv is None else _p(_c(dv)), float(Cl), float(Cq),
                                float(eps_q), float(eps_u), float(g["gamma"]), nt, _p(t), _p(a[0]), _p(a[1]),
                                _p(a[2]), _p(du))
    return a.T.copy(), du


def hydro_visc(g, **visc):
    """Full brute-force chain with the extras pass and the viscous forces."""
    V, rho = volume(g)
    A, B, dA, dB, nf = corrections(g, V)
    ex = extras(g, V, (A, B, dA, dB))
    a, du = accel_visc(g, V, rho, (A, B, dA, dB), ex["dv"], **{**VISC_DEFAULT, **visc})
    return dict(V=V, rho=rho, A=A, B=B, dA=dA, dB=dB, a=a, dudt=du, n_fallback=nf,
                totals=totals(g, a, du), **ex)


def timestep(g, a, gamma, c_cfl, c_acc):
    """Global time step: the minimum over particles of
    min(c_cfl 2h_i / (c_i + |v_i|), c_acc sqrt(2h_i / |a_i|)), c_i = sqrt(gamma (gamma-1) u_i)
    (the acceleration limit only where |a_i| > 0); a plain loop in FP64."""
    best = np.inf
    for i in range(len(g["h"])):
        H = 2.0 * float(g["h"][i])
        cs = np.sqrt(gamma * (gamma - 1.0) * float(g["u"][i]))
        v = np.sqrt(float(g["vx"][i]) ** 2 + float(g["vy"][i]) ** 2 + float(g["vz"][i]) ** 2)
        t = c_cfl * H / (cs + v)
        am = np.sqrt(float(a[i, 0]) ** 2 + float(a[i, 1]) ** 2 + float(a[i, 2]) ** 2)
        if am > 0.0:
            t = min(t, c_acc * np.sqrt(H / am))
        best = min(best, t)
    return best


def kick_drift(g, a, dudt, dt):
    """v + a dt, u + du/dt dt, then x + v_new dt wrapped into [0, 1): returns a new dict."""
    out = dict(g)
    for c, k in enumerate(("vx", "vy", "vz")):
        out[k] = np.asarray(g[k], dtype=np.float64) + np.asarray(a)[:, c] * dt
    out["u"] = np.asarray(g["u"], dtype=np.float64) + np.asarray(dudt) * dt
    for k, kv in zip(("x", "y", "z"), ("vx", "vy", "vz")):
        q = np.asarray(g[k], dtype=np.float64) + out[kv] * dt
        out[k] = q - np.floor(q)
    return out


def totals(g, a, dudt):
    """[sum m a (3), sum m (v.a + du/dt), sum m |a|, sum m (|v.a| + |du/dt|),
    sum m du/dt, sum m v.a] over all particles."""
    m, vx, vy, vz = (_c(g[k]) for k in ("m", "vx", "vy", "vz"))
    a = _c(a)
    ax, ay, az = (_c(a[:, c]) for c in range(3))
    du = _c(dudt)
    out = np.empty(8)
    _load().oracle_totals(m.size, _p(m), _p(vx), _p(vy), _p(vz), _p(ax), _p(ay), _p(az),
                          _p(du), _p(out))
    return out


def hydro(g):
    """Full brute-force forward chain over all particles."""
    V, rho = volume(g)
    A, B, dA, dB, nf = corrections(g, V)
    a, du = accel(g, V, rho, (A, B, dA, dB))
    return dict(V=V, rho=rho, A=A, B=B, dA=dA, dB=dB, a=a, dudt=du, n_fallback=nf,
                totals=totals(g, a, du))


def hydro_targets(g, targets):
    """Forward chain for sampled targets, each evaluated inside its 3-hop pool."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    t = _c(targets, np.int64)
    nt = t.size
    V = np.empty(nt)
    rho = np.empty(nt)
    A = np.empty(nt)
    B = np.empty((nt, 3))
    dA = np.empty((nt, 3))
    dB = np.empty((nt, 3, 3))
    a = np.empty((3, nt))
    du = np.empty(nt)
    nf = _load().oracle_hydro_targets(arr[0].size, *[_p(v) for v in arr], float(g["gamma"]), nt,
                                      _p(t), _p(V), _p(rho), _p(A), _p(B), _p(dA), _p(dB),
                                      _p(a[0]), _p(a[1]), _p(a[2]), _p(du))
    return dict(V=V, rho=rho, A=A, B=B, dA=dA, dB=dB, a=a.T.copy(), dudt=du, n_fallback=int(nf))


def gravity(g, targets=None, poly=None):
    """Short-range Plummer-softened gravity with a hard cutoff (brute force)."""
    x, y, z, m = (_c(g[k]) for k in ("x", "y", "z", "m"))
    t, nt = _targets(targets, x.size)
    pc = None if poly is None else _c(poly)
    a = np.empty((3, nt))
    _load().oracle_gravity(x.size, _p(x), _p(y), _p(z), _p(m), float(g["G"]), float(g["eps"]),
                           float(g["r_cut"]), _p(pc), nt, _p(t), _p(a[0]), _p(a[1]), _p(a[2]))
    return a.T.copy()


def long_range_force(r, r_s):
    """Long-range (particle-mesh) force per unit mass at separations r > 0 for
    a mesh potential filtered by exp(-k^2 r_s^2): [erf(x) - 2x exp(-x^2)/sqrt(pi)] / r^2,
    x = r / (2 r_s) (crk_oracle.cpp)."""
    r = _c(np.atleast_1d(r))
    f = np.empty_like(r)
    _load().oracle_long_range_force(r.size, _p(r), float(r_s), _p(f))
    return f


FIT_SAMPLES = 256


def fit_poly(r_s, r_cut, samples=FIT_SAMPLES, target=None):
    """The six coefficients p_0..p_5 of P(s) = sum_k p_k s^k, s = r^2, that the
    short-range gravity subtracts (its pair kernel is
    x [(r^2 + eps^2)^(-3/2) - P(r^2)]): the weighted least-squares fit of the
    long-range force over r, g(s) = f_L(r)/r, at s_k = r_cut^2 (k + 1/2) / samples,
    minimising sum_k [r_k^3 (g(s_k) - P(s_k))]^2 -- the error of the pair force
    relative to the Newtonian force at each separation.  Solved in the scaled
    variable t = s / r_cut^2 with numpy's least squares.  target(r), when
    given, replaces f_L(r)/r (to check the fit on known functions)."""
    t = (np.arange(samples) + 0.5) / samples
    r = r_cut * np.sqrt(t)
    y = long_range_force(r, r_s) / r if target is None else target(r)
    w = r ** 3
    A = np.vander(t, 6, increasing=True)
    c = np.linalg.lstsq(A * w[:, None], y * w, rcond=None)[0]
    return c / (r_cut * r_cut) ** np.arange(6)


def gravity_grad(g, abar, parts, kinds, poly=None, fd_step=1e-7):
    """dL/dx of L = sum_i abar_i . a_i (short-range gravity, masses fixed) at
    coordinates (parts[k], kinds[k] in 0..2).  Returns (forward-mode dual-number
    gradient, central differences)."""
    x, y, z, m = (_c(g[k]) for k in ("x", "y", "z", "m"))
    ab = _c(abar).reshape(-1)
    pt = _c(parts, np.int64)
    kd = _c(kinds, np.int32)
    pc = None if poly is None else _c(poly)
    gd = np.empty(pt.size)
    gf = np.empty(pt.size)
    _load().oracle_gravity_grad(x.size, _p(x), _p(y), _p(z), _p(m), float(g["G"]), float(g["eps"]),
                                float(g["r_cut"]), _p(pc), _p(ab), pt.size, _p(pt), _p(kd),
                                float(fd_step), _p(gd), _p(gf))
    return gd, gf


def count_pairs(g, mode, targets=None, r_fixed=0.0):
    """Ordered pairs j != i inside the pass radius: mode 0 = 2h_i, 1 = 2max(h_i,h_j), 2 = r_fixed."""
    x, y, z = (_c(g[k]) for k in ("x", "y", "z"))
    h = _c(g["h"]) if "h" in g else np.zeros_like(x)
    t, nt = _targets(targets, x.size)
    per = np.empty(nt, dtype=np.int32)
    tot = _load().oracle_count_pairs(x.size, _p(x), _p(y), _p(z), _p(h), int(mode), float(r_fixed),
                                     nt, _p(t), _p(per))
    return int(tot), per


COORD_KINDS = ("x", "y", "z", "vx", "vy", "vz", "u")


def grad(g, parts, kinds, fd_step=1e-6):
    """dL/dtheta of L = sum w |a|^2 + sum c du/dt for coordinates (parts[k], kinds[k]).

    kinds index COORD_KINDS.  Returns (forward-mode dual-number gradient,
    central-difference gradient, cone sizes [k, (|D1|, |D2|, |D3|)]).  Both are
    evaluated over each coordinate's dependency cone with baseline values
    elsewhere (see crk_oracle.cpp).
    """
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    w, cw = _c(g["w"]), _c(g["c"])
    pt = _c(parts, np.int64)
    kd = _c(kinds, np.int32)
    nc = pt.size
    gd = np.empty(nc)
    gf = np.empty(nc)
    cs = np.empty((nc, 3), dtype=np.int64)
    _load().oracle_grad(arr[0].size, *[_p(v) for v in arr], float(g["gamma"]), _p(w), _p(cw), nc,
                        _p(pt), _p(kd), float(fd_step), _p(gd), _p(gf), _p(cs))
    return gd, gf, cs


def grad_visc(g, parts, kinds, fd_step=1e-6, Cl=1.0, Cq=2.0, eps_q=0.01):
    """dL/dtheta of L = sum w |a|^2 + sum c du/dt through the chain with the
    extras pass and the viscous forces, at coordinates (parts[k], kinds[k]).
    Returns (dual-number gradient, central-difference gradient); every
    particle's chain is evaluated, so keep n small."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    w, cw = _c(g["w"]), _c(g["c"])
    pt = _c(parts, np.int64)
    kd = _c(kinds, np.int32)
    nc = pt.size
    gd = np.empty(nc)
    gf = np.empty(nc)
    _load().oracle_grad_visc(arr[0].size, *[_p(v) for v in arr], float(g["gamma"]), float(Cl), float(Cq),
                             float(eps_q), _p(w), _p(cw), nc, _p(pt), _p(kd), float(fd_step), _p(gd), _p(gf))
    return gd, gf


def grad_coordinates(n, n_pos=32, n_vel=16, n_u=16, seed=19):
    """The seeded sample of coordinates the gradient checks use: (parts, kinds)."""
    rng = np.random.default_rng(seed)
    parts = rng.choice(n, size=n_pos + n_vel + n_u, replace=False).astype(np.int64)
    kinds = np.concatenate([rng.integers(0, 3, n_pos), rng.integers(3, 6, n_vel),
                            np.full(n_u, 6)]).astype(np.int32)
    return parts, kinds


FLOP_KINDS = ("volume", "moments", "accel", "gravity", "gravity_poly", "volume_adj", "moments_adj",
              "accel_adj", "extras", "accel_visc", "gravity_adj", "gravity_adj_poly", "accel_compat",
              "accel_visc_adj", "extras_adj")


def flops():
    """FLOP per ordered pair inside each pass's radius, counted on the oracle's
    own per-pair code with its operation-recording scalar (per-particle work
    hoisted, common subexpressions once, FMA = 2, sqrt and division 1; the
    adjoints as the reverse-mode derivative of the pair term with respect to
    the lane particle's inputs).  Returns {kind: count}."""
    out = np.zeros(len(FLOP_KINDS))
    _load().oracle_flops(_p(out))
    return {k: int(v) for k, v in zip(FLOP_KINDS, out)}


def flops_selftest():
    """Counts of eight small expressions that pin the counting rules
    (see oracle_flops_selftest in crk_oracle.cpp)."""
    out = np.zeros(8)
    _load().oracle_flops_selftest(_p(out))
    return [int(v) for v in out]


def passes_listed(g, targets, off, idx, V, rho, corr, threads=0):
    """Volume, corrections and accel/energy of the targets over precomputed
    candidate lists (CSR off/idx, one row per target).  V, rho and corr are the
    values of all particles the passes read.  Returns (2 x gather pairs,
    V of the targets, A of the targets, a_x of the targets, du/dt of the targets)."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    V, rho = _c(V), _c(rho)
    A, B, dA, dB = (_c(c) for c in corr[:4])
    t = _c(targets, np.int64)
    off, idx = _c(off, np.int64), _c(idx, np.int64)
    nt = t.size
    Vo, Ao, ax, du = (np.empty(nt) for _ in range(4))
    pairs = _load().oracle_passes_listed(arr[0].size, *[_p(v) for v in arr], float(g["gamma"]),
                                         _p(V), _p(rho), _p(A), _p(B), _p(dA), _p(dB), nt, _p(t),
                                         _p(off), _p(idx), int(threads), _p(Vo), _p(Ao), _p(ax),
                                         _p(du))
    return int(pairs), Vo, Ao, ax, du


def gravity_listed(g, targets, off, idx, threads=0, poly=None):
    """Short-range gravity of the targets over precomputed candidate lists (CSR off/idx)."""
    x, y, z, m = (_c(g[k]) for k in ("x", "y", "z", "m"))
    t = _c(targets, np.int64)
    off, idx = _c(off, np.int64), _c(idx, np.int64)
    pc = None if poly is None else _c(poly)
    a = np.empty((3, t.size))
    _load().oracle_gravity_listed(x.size, _p(x), _p(y), _p(z), _p(m), float(g["G"]), float(g["eps"]),
                                  float(g["r_cut"]), _p(pc), t.size, _p(t), _p(off), _p(idx),
                                  int(threads), _p(a[0]), _p(a[1]), _p(a[2]))
    return a.T.copy()


def hydro_listed(g, off, idx):
    """Full forward chain of all particles with candidates from precomputed
    lists (CSR off/idx over all particles).  With exact lists in increasing
    index order (``neighbour_lists``) it equals ``hydro`` bit for bit."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    n = arr[0].size
    off, idx = _c(off, np.int64), _c(idx, np.int64)
    V, rho, A, du = (np.empty(n) for _ in range(4))
    B, dA = np.empty((n, 3)), np.empty((n, 3))
    dB = np.empty((n, 3, 3))
    a = np.empty((3, n))
    nf = _load().oracle_hydro_listed(n, *[_p(v) for v in arr], float(g["gamma"]), _p(off), _p(idx),
                                     _p(V), _p(rho), _p(A), _p(B), _p(dA), _p(dB), _p(a[0]), _p(a[1]),
                                     _p(a[2]), _p(du))
    a = a.T.copy()
    return dict(V=V, rho=rho, A=A, B=B, dA=dA, dB=dB, a=a, dudt=du, n_fallback=int(nf),
                totals=totals(g, a, du))


def visc_listed(g, off, idx, ref, Cl=1.0, Cq=2.0, eps_q=0.01):
    """Extras of all particles and their viscous forces over precomputed lists,
    from the oracle's own V, rho and corrections ``ref`` (a hydro_listed or
    hydro result).  With exact lists it equals extras + accel_visc bit for bit."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    n = arr[0].size
    off, idx = _c(off, np.int64), _c(idx, np.int64)
    rhoR, du = np.empty(n), np.empty(n)
    dv, de = np.empty((n, 3, 3)), np.empty((n, 3))
    a = np.empty((3, n))
    _load().oracle_visc_listed(n, *[_p(v) for v in arr], float(g["gamma"]), float(Cl), float(Cq), float(eps_q),
                               _p(off), _p(idx), _p(_c(ref["V"])), _p(_c(ref["rho"])), _p(_c(ref["A"])),
                               _p(_c(ref["B"])), _p(_c(ref["dA"])), _p(_c(ref["dB"])), _p(rhoR), _p(dv),
                               _p(de), _p(a[0]), _p(a[1]), _p(a[2]), _p(du))
    a = a.T.copy()
    return dict(rhoR=rhoR, dv=dv, du=de, a=a, dudt=du, totals=totals(g, a, du))


def compat_listed(g, off, idx, ref, eps_u=0.1):
    """Forces with the compatible energy partition of all particles over
    precomputed lists, from the oracle's own V, rho and corrections ``ref``.
    With exact lists it equals accel_compat bit for bit."""
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")
    arr = [_c(g[k]) for k in keys]
    n = arr[0].size
    off, idx = _c(off, np.int64), _c(idx, np.int64)
    a = np.empty((3, n))
    du = np.empty(n)
    _load().oracle_compat_listed(n, *[_p(v) for v in arr], float(g["gamma"]), float(eps_u), _p(off), _p(idx),
                                 _p(_c(ref["V"])), _p(_c(ref["rho"])), _p(_c(ref["A"])), _p(_c(ref["B"])),
                                 _p(_c(ref["dA"])), _p(_c(ref["dB"])), _p(a[0]), _p(a[1]), _p(a[2]), _p(du))
    return a.T.copy(), du


def neighbour_lists(g, margin=1e-9):
    """Candidate lists for the listed oracle entries: CSR (off, idx) holding,
    for every particle i, every j != i with |x_ij| < max(2h_i, 2h_j) (and a
    few more within a relative margin, which the passes reject themselves) in
    increasing index order.  Built from the nearest neighbours of a periodic
    k-d tree (scipy; input preparation, no method arithmetic): the gather
    pairs r < 2h_i of every particle, united with their transposes."""
    from scipy.spatial import cKDTree

    P = np.stack([np.asarray(g[k], dtype=np.float64) for k in ("x", "y", "z")], 1)
    H = 2.0 * np.asarray(g["h"], dtype=np.float64) * (1.0 + margin)
    n = len(H)
    tree = cKDTree(P, boxsize=1.0)
    gi, gj = [], []
    todo = np.arange(n, dtype=np.int64)
    k = 64
    while todo.size:
        k = min(k, n)
        d, j = tree.query(P[todo], k=k, workers=-1)
        d = d.reshape(len(todo), k)
        j = j.reshape(len(todo), k)
        done = np.ones(len(todo), bool) if k == n else d[:, -1] >= H[todo]
        ii = np.repeat(todo[done], k)
        jj = j[done].ravel().astype(np.int64)
        keep = (d[done].ravel() < np.repeat(H[todo[done]], k)) & (jj != ii)
        gi.append(ii[keep])
        gj.append(jj[keep])
        todo = todo[~done]
        k *= 2
    gi, gj = np.concatenate(gi), np.concatenate(gj)
    key = np.unique(np.concatenate([gi * n + gj, gj * n + gi]))
    i, j = key // n, key % n
    off = np.searchsorted(i, np.arange(n + 1, dtype=np.int64))
    return off.astype(np.int64), j.astype(np.int64)
