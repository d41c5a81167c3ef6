"""Python binding of ``libcrk.so``: the CRK-SPH pair passes and short-range
gravity for MI355X (gfx950).

Argument marshalling only.  Every step runs in the HIP library; PyTorch
supplies device memory and the current stream.  The functions have the names
of the C entry points declared in ``include/crk.h`` and follow its
conventions (caller particle order; FP64 positions; other fields and outputs
in the precision of the call, ``"f32"`` or ``"f64"``).

There is no CPU fallback: if the library is missing or no GPU is present the
calls raise.
"""

from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrk.so")

CRK_F32, CRK_F64 = 0, 1
_PREC = {"f32": CRK_F32, "f64": CRK_F64}
_DTYPE = {"f32": torch.float32, "f64": torch.float64}
CRK_ENOSPC = -5
_STATUS = {0: "CRK_OK", -1: "CRK_EINVAL", -3: "CRK_EHIP", -4: "CRK_ESTATE", -5: "CRK_ENOSPC"}

# the C symbols declared in include/crk.h
EXPORTS = ("crk_build_leaf_pairs", "crk_build_leaf_pairs_device", "crk_volume", "crk_corrections",
           "crk_accel_energy", "crk_accel_energy_noalloc", "crk_extras", "crk_accel_energy_visc",
           "crk_accel_energy_compatible", "sr_gravity",
           "sr_gravity_backward", "sr_gravity_fit_poly", "crk_timestep", "crk_kick_drift",
           "crk_queue_visits", "crk_accel_energy_backward", "crk_accel_energy_visc_backward",
           "crk_leaves_stats", "crk_leaves_perm",
           "crk_get_tuning", "crk_set_tuning",
           "crk_timing", "crk_kernel_times", "crk_leaves_free", "crk_last_error")
KERNEL_KINDS = ("cull", "volume", "moments", "accel", "gravity", "pack", "accel_adj",
                "moments_adj", "volume_adj", "solve_adj", "gravity_adj", "extras", "accel_visc", "extras_adj")


class CrkError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed with {_STATUS.get(code, code)}: {msg}")
        self.code = code


class _Gas(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in
                                          ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m")]


class _Corr(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("A", "B", "dA", "dB", "M")]


def _corr(corr):
    """(A, B, dA, dB[, M]) -> crk_corr; M (the stored moment sums) is optional."""
    ptrs = [t.data_ptr() for t in corr[:4]]
    M = corr[4] if len(corr) > 4 else None
    if M is not None:
        _dev(M, torch.float64)
    return _Corr(*ptrs, None if M is None else M.data_ptr())


class Visc(ctypes.Structure):
    _fields_ = [("Cl", ctypes.c_double), ("Cq", ctypes.c_double), ("eps_q", ctypes.c_double)]


VISC_DEFAULT = dict(Cl=1.0, Cq=2.0, eps_q=0.01)


class Tuning(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int), ("waves_per_cu", ctypes.c_int),
                ("kahan_chunk", ctypes.c_int), ("block_waves", ctypes.c_int),
                ("xcd_groups", ctypes.c_int), ("tile_order", ctypes.c_int), ("addr64", ctypes.c_int),
                ("exchange", ctypes.c_int), ("stage16", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path=None):
    """Load libcrk.so (built by ``paper_2310_16122_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P, I64, D, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.crk_build_leaf_pairs.argtypes = [I64, P, P, P, P, D, I, I, D, I, P, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(P), P]
    lib.crk_build_leaf_pairs_device.argtypes = [I64, P, P, P, P, D, I, I, P, ctypes.c_size_t,
                                                ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(P), P]
    lib.crk_volume.argtypes = [P, ctypes.POINTER(_Gas), I, P, P, P]
    lib.crk_corrections.argtypes = [P, ctypes.POINTER(_Gas), P, I, ctypes.POINTER(_Corr), P, P]
    lib.crk_accel_energy.argtypes = [P, ctypes.POINTER(_Gas), P, P, ctypes.POINTER(_Corr), D, I,
                                     P, P, P, P]
    lib.crk_accel_energy_noalloc.argtypes = lib.crk_accel_energy.argtypes
    lib.sr_gravity.argtypes = [P, I64, P, P, P, P, D, D, D, P, I, P, P]
    lib.sr_gravity_backward.argtypes = [P, I64, P, P, P, P, D, D, D, P, P, I, P, P]
    lib.sr_gravity_fit_poly.argtypes = [D, D, I, P]
    lib.crk_timestep.argtypes = [I64, P, P, P, P, P, P, D, D, D, I, P, P]
    lib.crk_kick_drift.argtypes = [I64, P, P, P, P, P, P, P, P, P, P, P, I, P]
    lib.crk_extras.argtypes = [P, ctypes.POINTER(_Gas), P, ctypes.POINTER(_Corr), I, P, P, P, P]
    lib.crk_accel_energy_visc.argtypes = [P, ctypes.POINTER(_Gas), P, P, ctypes.POINTER(_Corr), P,
                                          ctypes.POINTER(Visc), D, I, P, P, P, P]
    lib.crk_accel_energy_compatible.argtypes = [P, ctypes.POINTER(_Gas), P, P, ctypes.POINTER(_Corr), P,
                                                ctypes.POINTER(Visc), D, D, I, P, P, P, P]
    lib.crk_accel_energy_backward.argtypes = [P, ctypes.POINTER(_Gas), P, P, ctypes.POINTER(_Corr), D,
                                              P, P, I, P, P, P, P]
    lib.crk_accel_energy_visc_backward.argtypes = [P, ctypes.POINTER(_Gas), P, P, ctypes.POINTER(_Corr), P,
                                                   ctypes.POINTER(Visc), D, P, P, I, P, P, P, P]
    lib.crk_leaves_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.crk_leaves_perm.argtypes = [P, P, P]
    lib.crk_queue_visits.argtypes = [P, P, P]
    lib.crk_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.crk_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.crk_timing.argtypes = [P, I]
    lib.crk_kernel_times.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.crk_leaves_free.argtypes = [P]
    lib.crk_leaves_free.restype = None
    lib.crk_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("crk_leaves_free", "crk_last_error"):
            getattr(lib, name).restype = I
    _lib = lib
    return lib


def _check(fn, code):
    if code != 0:
        raise CrkError(fn, code, load_library().crk_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t


def _gas(gas, prec, keys):
    dt = _DTYPE[prec]
    g = _Gas()
    g.n = int(gas["x"].numel())
    for k in ("x", "y", "z"):
        setattr(g, k, _dev(gas[k], torch.float64).data_ptr())
    for k in keys:
        setattr(g, k, _dev(gas[k], dt).data_ptr())
    return g


class Leaves:
    """Owner of a ``crk_leaves`` handle and of the device workspace it points
    into (tree order, interaction lists, scratch: a uint8 torch tensor)."""

    def __init__(self, handle, n, hydro, prec, ws):
        # a copy of the pointer: the caller's ctypes object may be reused
        self._h = ctypes.c_void_p(handle.value if isinstance(handle, ctypes.c_void_p) else handle)
        self.n = n
        self.hydro = hydro
        self.prec = prec
        self.ws = ws

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("handle already freed")
        return self._h

    def stats(self):
        out = (ctypes.c_int64 * 8)()
        _check("crk_leaves_stats", load_library().crk_leaves_stats(self.handle, out))
        keys = ("leaves", "tiles", "candidate_pairs", "list_entries", "pairs_gather",
                "pairs_force", "padded_slots", "build_us")
        return dict(zip(keys, list(out)))

    def perm(self, device="cuda"):
        """Tree order: perm[s] = caller index of the s-th particle in tree order."""
        out = torch.empty(self.n, dtype=torch.int32, device=device)
        _check("crk_leaves_perm", load_library().crk_leaves_perm(self.handle, _ptr(out), _stream()))
        return out

    def queue_visits(self, device="cuda"):
        """How often the work distribution hands out each tile (int32 per tile; all 1)."""
        out = torch.zeros(self.stats()["tiles"], dtype=torch.int32, device=device)
        _check("crk_queue_visits", load_library().crk_queue_visits(self.handle, _ptr(out), _stream()))
        return out

    def get_tuning(self):
        t = Tuning()
        _check("crk_get_tuning", load_library().crk_get_tuning(self.handle, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning(**{**self.get_tuning(), **kw})
        _check("crk_set_tuning", load_library().crk_set_tuning(self.handle, ctypes.byref(t)))

    def timing(self, enable=True):
        """Start (and reset) or stop per-kernel event timing on this handle."""
        _check("crk_timing", load_library().crk_timing(self.handle, int(bool(enable))))

    def kernel_times(self):
        """{kind: (total ms, launches)} of the kernels timed since timing was enabled."""
        ms = (ctypes.c_double * len(KERNEL_KINDS))()
        nl = (ctypes.c_int64 * len(KERNEL_KINDS))()
        _check("crk_kernel_times", load_library().crk_kernel_times(self.handle, ms, nl))
        return {k: (ms[i], nl[i]) for i, k in enumerate(KERNEL_KINDS)}

    def free(self):
        if self._h is not None:
            load_library().crk_leaves_free(self._h)
            self._h = None
        self.ws = None  # back to torch's allocator, ordered on the stream the passes ran on

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _ws_guess(n, hydro):
    """First workspace size tried: per particle the tree order, positions,
    counts and the scratch of an FP64 backward pass, plus (hydro) about 128
    neighbour-list slots of 9 bytes.  The library reports the exact need when
    it is larger."""
    return (1 << 20) + n * ((830 + 9 * 128) if hydro else 96)


def _build(fn, call, x, y, z, h, prec, ws):
    """The workspace protocol of both builds: ``ws`` (a uint8 CUDA tensor) when
    given and large enough, else one allocated here; on CRK_ENOSPC the
    workspace is reallocated at the size the library reports and the call
    repeated."""
    for t in (x, y, z):
        _dev(t, torch.float64)
    if h is not None:
        _dev(h, _DTYPE[prec])
    n = int(x.numel())
    need = ctypes.c_size_t(0)
    size = _ws_guess(n, h is not None) if ws is None else int(ws.numel())
    for _ in range(4):
        if ws is None or int(ws.numel()) < size:
            ws = torch.empty(size, dtype=torch.uint8, device=x.device)
        out = ctypes.c_void_p()
        code = call(n, ws, need, out)
        if code != CRK_ENOSPC:
            _check(fn, code)
            return Leaves(out, n, h is not None, prec, ws)
        size = int(need.value)
        ws = None
    _check(fn, code)


def crk_build_leaf_pairs(x, y, z, h=None, r_fixed=0.0, leaf_max=128, leaf_min=1,
                         split_extent=0.0, prec="f32", ws=None, skin=0.0):
    """Tree + interaction lists (hydro mode when h is given, else radius r_fixed).

    In hydro mode ``skin`` widens every support for the lists, so that the
    handle can be reused while no particle has moved by skin / 2 (the C call
    takes it in place of r_fixed).  The library resumes a call that stopped
    for want of workspace from the host tree it built."""
    lib = load_library()

    def call(n, ws, need, out):
        return lib.crk_build_leaf_pairs(n, _ptr(x), _ptr(y), _ptr(z), _ptr(h),
                                        float(skin if h is not None else r_fixed),
                                        int(leaf_max), int(leaf_min), float(split_extent), _PREC[prec],
                                        _ptr(ws), int(ws.numel()), ctypes.byref(need), ctypes.byref(out),
                                        _stream())
    return _build("crk_build_leaf_pairs", call, x, y, z, h, prec, ws)


def crk_build_leaf_pairs_device(x, y, z, h=None, r_fixed=0.0, leaf_max=128, prec="f32", ws=None,
                                skin=0.0):
    """The same handle built on the GPU (Morton octree leaves of at most
    leaf_max <= 1024 particles); every particle's list holds the same
    neighbours as with crk_build_leaf_pairs."""
    lib = load_library()

    def call(n, ws, need, out):
        return lib.crk_build_leaf_pairs_device(n, _ptr(x), _ptr(y), _ptr(z), _ptr(h),
                                               float(skin if h is not None else r_fixed),
                                               int(leaf_max), _PREC[prec], _ptr(ws), int(ws.numel()),
                                               ctypes.byref(need), ctypes.byref(out), _stream())
    return _build("crk_build_leaf_pairs_device", call, x, y, z, h, prec, ws)


def crk_volume(leaves, gas, prec="f32"):
    g = _gas(gas, prec, ("h", "m"))
    V = torch.empty(g.n, dtype=_DTYPE[prec], device=gas["x"].device)
    rho = torch.empty_like(V)
    _check("crk_volume", load_library().crk_volume(leaves.handle, ctypes.byref(g), _PREC[prec],
                                                   _ptr(V), _ptr(rho), _stream()))
    return V, rho


def crk_corrections(leaves, gas, V, prec="f32", n_fallback=None, store_sums=False):
    """(A, B, dA, dB), plus M [30, n] FP64 (the moment sums the backward can reuse)
    when store_sums is true."""
    g = _gas(gas, prec, ("h",))
    dt, dev = _DTYPE[prec], gas["x"].device
    _dev(V, dt)
    A = torch.empty(g.n, dtype=dt, device=dev)
    B = torch.empty(g.n, 3, dtype=dt, device=dev)
    dA = torch.empty(g.n, 3, dtype=dt, device=dev)
    dB = torch.empty(g.n, 3, 3, dtype=dt, device=dev)
    M = torch.empty(30, g.n, dtype=torch.float64, device=dev) if store_sums else None
    c = _corr((A, B, dA, dB, M))
    if n_fallback is not None:
        _dev(n_fallback, torch.int64)
    _check("crk_corrections",
           load_library().crk_corrections(leaves.handle, ctypes.byref(g), _ptr(V), _PREC[prec],
                                          ctypes.byref(c), _ptr(n_fallback), _stream()))
    return (A, B, dA, dB, M) if store_sums else (A, B, dA, dB)


def crk_accel_energy(leaves, gas, V, rho, corr, gamma=5.0 / 3.0, prec="f32", totals=True,
                     noalloc=False):
    """(a [n,3], du/dt [n], totals [8] FP64 or None).  noalloc: the variant whose
    scratch is the library's fixed device array (crk_accel_energy_noalloc)."""
    g = _gas(gas, prec, ("vx", "vy", "vz", "u", "h", "m"))
    dt, dev = _DTYPE[prec], gas["x"].device
    for t in (V, rho, *corr[:4]):
        _dev(t, dt)
    c = _corr(corr)
    a = torch.empty(g.n, 3, dtype=dt, device=dev)
    du = torch.empty(g.n, dtype=dt, device=dev)
    tot = torch.empty(8, dtype=torch.float64, device=dev) if totals else None
    name = "crk_accel_energy_noalloc" if noalloc else "crk_accel_energy"
    _check(name, getattr(load_library(), name)(leaves.handle, ctypes.byref(g), _ptr(V), _ptr(rho),
                                               ctypes.byref(c), float(gamma), _PREC[prec], _ptr(a),
                                               _ptr(du), _ptr(tot), _stream()))
    return a, du, tot


def crk_accel_energy_noalloc(leaves, gas, V, rho, corr, gamma=5.0 / 3.0, prec="f32", totals=True):
    return crk_accel_energy(leaves, gas, V, rho, corr, gamma, prec, totals, noalloc=True)


def crk_accel_energy_backward(leaves, gas, V, rho, corr, ga, gdudt, gamma=5.0 / 3.0, prec="f32"):
    """dL/dx [n,3], dL/dv [n,3], dL/du [n] from ga = dL/da [n,3] and gdudt = dL/d(du/dt) [n].

    corr = (A, B, dA, dB) recomputes the moments; (A, B, dA, dB, M) with the
    forward's stored sums M reuses them."""
    g = _gas(gas, prec, ("vx", "vy", "vz", "u", "h", "m"))
    dt, dev = _DTYPE[prec], gas["x"].device
    for t in (V, rho, *corr[:4], ga, gdudt):
        _dev(t, dt)
    c = _corr(corr)
    gx = torch.empty(g.n, 3, dtype=dt, device=dev)
    gv = torch.empty(g.n, 3, dtype=dt, device=dev)
    gu = torch.empty(g.n, dtype=dt, device=dev)
    _check("crk_accel_energy_backward",
           load_library().crk_accel_energy_backward(leaves.handle, ctypes.byref(g), _ptr(V), _ptr(rho),
                                                    ctypes.byref(c), float(gamma), _ptr(ga),
                                                    _ptr(gdudt), _PREC[prec], _ptr(gx), _ptr(gv),
                                                    _ptr(gu), _stream()))
    return gx, gv, gu


class CRKAccelEnergy(torch.autograd.Function):
    """(pos [n,3] f64, v [n,3], u [n]) -> (a [n,3], du/dt [n]) through the full chain
    volume -> corrections -> accel/energy over the handle's interaction lists.

    h and m are constants.  Backward calls crk_accel_energy_backward (the
    hand-written adjoint); the position gradient is returned in FP64.
    """

    @staticmethod
    def forward(ctx, pos, v, u, leaves, h, m, gamma=5.0 / 3.0, prec="f32"):
        gas = {"x": pos[:, 0].contiguous(), "y": pos[:, 1].contiguous(), "z": pos[:, 2].contiguous(),
               "vx": v[:, 0].contiguous(), "vy": v[:, 1].contiguous(), "vz": v[:, 2].contiguous(),
               "u": u.contiguous(), "h": h, "m": m}
        out = forward(leaves, gas, gamma, prec, store_sums=True)
        ctx.leaves, ctx.gamma, ctx.prec = leaves, gamma, prec
        ctx.gas = gas
        ctx.save_for_backward(out["V"], out["rho"], out["A"], out["B"], out["dA"], out["dB"], out["M"])
        return out["a"], out["dudt"]

    @staticmethod
    def backward(ctx, ga, gdu):
        V, rho, A, B, dA, dB, M = ctx.saved_tensors
        dt = _DTYPE[ctx.prec]
        ga = torch.zeros_like(A.new_empty(A.shape[0], 3)) if ga is None else ga.to(dt).contiguous()
        gdu = torch.zeros_like(A) if gdu is None else gdu.to(dt).contiguous()
        gx, gv, gu = crk_accel_energy_backward(ctx.leaves, ctx.gas, V, rho, (A, B, dA, dB, M), ga, gdu,
                                               ctx.gamma, ctx.prec)
        return gx.double(), gv, gu, None, None, None, None, None


def crk_extras(leaves, gas, V, corr, prec="f32"):
    """(rhoR [n], dv [n,3,3] with dv[i,a,c] = d_c v^a, du [n,3])."""
    g = _gas(gas, prec, ("vx", "vy", "vz", "u", "h", "m"))
    dt, dev = _DTYPE[prec], gas["x"].device
    for t in (V, *corr[:4]):
        _dev(t, dt)
    c = _corr(corr)
    rhoR = torch.empty(g.n, dtype=dt, device=dev)
    dv = torch.empty(g.n, 3, 3, dtype=dt, device=dev)
    du = torch.empty(g.n, 3, dtype=dt, device=dev)
    _check("crk_extras", load_library().crk_extras(leaves.handle, ctypes.byref(g), _ptr(V), ctypes.byref(c),
                                                   _PREC[prec], _ptr(rhoR), _ptr(dv), _ptr(du), _stream()))
    return rhoR, dv, du


def crk_accel_energy_visc(leaves, gas, V, rho, corr, dv, gamma=5.0 / 3.0, prec="f32", totals=True, **visc):
    """Force pass with the artificial viscosity (constants Cl, Cq, eps_q; defaults VISC_DEFAULT)."""
    g = _gas(gas, prec, ("vx", "vy", "vz", "u", "h", "m"))
    dt, dev = _DTYPE[prec], gas["x"].device
    for t in (V, rho, *corr[:4], dv):
        _dev(t, dt)
    c = _corr(corr)
    q = Visc(**{**VISC_DEFAULT, **visc})
    a = torch.empty(g.n, 3, dtype=dt, device=dev)
    du = torch.empty(g.n, dtype=dt, device=dev)
    tot = torch.empty(8, dtype=torch.float64, device=dev) if totals else None
    _check("crk_accel_energy_visc",
           load_library().crk_accel_energy_visc(leaves.handle, ctypes.byref(g), _ptr(V), _ptr(rho),
                                                ctypes.byref(c), _ptr(dv), ctypes.byref(q), float(gamma),
                                                _PREC[prec], _ptr(a), _ptr(du), _ptr(tot), _stream()))
    return a, du, tot


def crk_accel_energy_compatible(leaves, gas, V, rho, corr, eps_u=0.1, dv=None, visc=None, gamma=5.0 / 3.0,
                                prec="f32", totals=True):
    """Force pass with the compatible energy partition (pair work split by
    f_ij, see include/crk.h); with the viscosity when dv and visc (a dict of
    Cl, Cq, eps_q) are given."""
    g = _gas(gas, prec, ("vx", "vy", "vz", "u", "h", "m"))
    dt, dev = _DTYPE[prec], gas["x"].device
    for t in (V, rho, *corr[:4]):
        _dev(t, dt)
    if dv is not None:
        _dev(dv, dt)
    c = _corr(corr)
    q = None if visc is None else Visc(**{**VISC_DEFAULT, **visc})
    a = torch.empty(g.n, 3, dtype=dt, device=dev)
    du = torch.empty(g.n, dtype=dt, device=dev)
    tot = torch.empty(8, dtype=torch.float64, device=dev) if totals else None
    _check("crk_accel_energy_compatible",
           load_library().crk_accel_energy_compatible(leaves.handle, ctypes.byref(g), _ptr(V), _ptr(rho),
                                                      ctypes.byref(c), _ptr(dv),
                                                      None if q is None else ctypes.byref(q), float(eps_u),
                                                      float(gamma), _PREC[prec], _ptr(a), _ptr(du), _ptr(tot),
                                                      _stream()))
    return a, du, tot


def crk_accel_energy_visc_backward(leaves, gas, V, rho, corr, dv, ga, gdudt, gamma=5.0 / 3.0, prec="f32",
                                   **visc):
    """dL/dx [n,3], dL/dv [n,3], dL/du [n] through the viscous chain (volume,
    corrections, Extras' velocity gradients dv, viscous forces) from
    ga = dL/da and gdudt = dL/d(du/dt); corr as for crk_accel_energy_backward."""
    g = _gas(gas, prec, ("vx", "vy", "vz", "u", "h", "m"))
    dt, dev = _DTYPE[prec], gas["x"].device
    for t in (V, rho, *corr[:4], dv, ga, gdudt):
        _dev(t, dt)
    c = _corr(corr)
    q = Visc(**{**VISC_DEFAULT, **visc})
    gx = torch.empty(g.n, 3, dtype=dt, device=dev)
    gv = torch.empty(g.n, 3, dtype=dt, device=dev)
    gu = torch.empty(g.n, dtype=dt, device=dev)
    _check("crk_accel_energy_visc_backward",
           load_library().crk_accel_energy_visc_backward(leaves.handle, ctypes.byref(g), _ptr(V), _ptr(rho),
                                                         ctypes.byref(c), _ptr(dv), ctypes.byref(q), float(gamma),
                                                         _ptr(ga), _ptr(gdudt), _PREC[prec], _ptr(gx), _ptr(gv),
                                                         _ptr(gu), _stream()))
    return gx, gv, gu


def forward_visc(leaves, gas, gamma=5.0 / 3.0, prec="f32", **visc):
    """volume -> corrections -> extras -> accel/energy with the viscosity."""
    V, rho = crk_volume(leaves, gas, prec)
    nf = torch.zeros(1, dtype=torch.int64, device=gas["x"].device)
    corr = crk_corrections(leaves, gas, V, prec, n_fallback=nf)
    rhoR, dv, du_grad = crk_extras(leaves, gas, V, corr, prec)
    a, du, tot = crk_accel_energy_visc(leaves, gas, V, rho, corr, dv, gamma, prec, **visc)
    return dict(V=V, rho=rho, A=corr[0], B=corr[1], dA=corr[2], dB=corr[3], rhoR=rhoR, dv=dv,
                du=du_grad, a=a, dudt=du, totals=tot, n_fallback=nf)


def sr_gravity_fit_poly(r_s, r_cut, samples=256):
    """The six coefficients of the particle-mesh force polynomial (host fit in the library)."""
    out = (ctypes.c_double * 6)()
    _check("sr_gravity_fit_poly", load_library().sr_gravity_fit_poly(float(r_s), float(r_cut), int(samples), out))
    return [out[k] for k in range(6)]


def sr_gravity_backward(leaves, x, y, z, m, ga, G=1.0, eps=0.0, r_cut=None, poly=None, prec="f32"):
    """dL/dx [n,3] of the short-range gravity given ga = dL/da [n,3]."""
    dt = _DTYPE[prec]
    for t in (x, y, z):
        _dev(t, torch.float64)
    _dev(m, dt)
    _dev(ga, dt)
    n = int(x.numel())
    gx = torch.empty(n, 3, dtype=dt, device=x.device)
    pc = None if poly is None else (ctypes.c_double * 6)(*[float(p) for p in poly])
    _check("sr_gravity_backward",
           load_library().sr_gravity_backward(leaves.handle, n, _ptr(x), _ptr(y), _ptr(z), _ptr(m), float(G),
                                              float(eps), float(r_cut), pc, _ptr(ga), _PREC[prec], _ptr(gx),
                                              _stream()))
    return gx


class SRGravity(torch.autograd.Function):
    """pos [n,3] f64 -> a [n,3]: short-range gravity over the handle's candidate
    leaves; backward calls sr_gravity_backward (masses are constants)."""

    @staticmethod
    def forward(ctx, pos, m, leaves, G=1.0, eps=0.0, r_cut=None, poly=None, prec="f32"):
        x, y, z = (pos[:, k].contiguous() for k in range(3))
        ctx.args = (leaves, m, G, eps, r_cut, poly, prec)
        ctx.save_for_backward(x, y, z)
        return sr_gravity(leaves, x, y, z, m, G, eps, r_cut, poly, prec)

    @staticmethod
    def backward(ctx, ga):
        x, y, z = ctx.saved_tensors
        leaves, m, G, eps, r_cut, poly, prec = ctx.args
        gx = sr_gravity_backward(leaves, x, y, z, m, ga.to(_DTYPE[prec]).contiguous(), G, eps, r_cut, poly, prec)
        return gx.double(), None, None, None, None, None, None, None


def sr_gravity(leaves, x, y, z, m, G=1.0, eps=0.0, r_cut=None, poly=None, prec="f32"):
    dt = _DTYPE[prec]
    for t in (x, y, z):
        _dev(t, torch.float64)
    _dev(m, dt)
    n = int(x.numel())
    a = torch.empty(n, 3, dtype=dt, device=x.device)
    pc = None
    if poly is not None:
        pc = (ctypes.c_double * 6)(*[float(p) for p in poly])
    _check("sr_gravity",
           load_library().sr_gravity(leaves.handle, n, _ptr(x), _ptr(y), _ptr(z), _ptr(m),
                                     float(G), float(eps), float(r_cut), pc, _PREC[prec], _ptr(a),
                                     _stream()))
    return a


def crk_timestep(gas, a, gamma=5.0 / 3.0, c_cfl=0.25, c_acc=0.25, prec="f32"):
    """The global time step as a one-element device tensor (no host synchronisation)."""
    dt_ = _DTYPE[prec]
    n = int(gas["h"].numel())
    for k in ("h", "u", "vx", "vy", "vz"):
        _dev(gas[k], dt_)
    _dev(a, dt_)
    dt = torch.empty(1, dtype=dt_, device=gas["h"].device)
    _check("crk_timestep",
           load_library().crk_timestep(n, _ptr(gas["h"]), _ptr(gas["u"]), _ptr(gas["vx"]), _ptr(gas["vy"]),
                                       _ptr(gas["vz"]), _ptr(a), float(gamma), float(c_cfl), float(c_acc),
                                       _PREC[prec], _ptr(dt), _stream()))
    return dt


def crk_kick_drift(gas, a, dudt, dt, prec="f32", disp=None):
    """Updates gas x, y, z, vx, vy, vz and u in place with the device time step dt.
    disp (float64 CUDA tensor of 2, optional): disp[0] accumulates the largest
    drift of each step (zero it after a build)."""
    dt_ = _DTYPE[prec]
    for k in ("x", "y", "z"):
        _dev(gas[k], torch.float64)
    for k in ("vx", "vy", "vz", "u"):
        _dev(gas[k], dt_)
    for t in (a, dudt, dt):
        _dev(t, dt_)
    if disp is not None:
        _dev(disp, torch.float64)
        if disp.numel() < 2:
            raise ValueError("disp needs two elements")
    n = int(gas["x"].numel())
    _check("crk_kick_drift",
           load_library().crk_kick_drift(n, _ptr(gas["x"]), _ptr(gas["y"]), _ptr(gas["z"]), _ptr(gas["vx"]),
                                         _ptr(gas["vy"]), _ptr(gas["vz"]), _ptr(gas["u"]), _ptr(a), _ptr(dudt),
                                         _ptr(dt), _ptr(disp), _PREC[prec], _stream()))


def forward(leaves, gas, gamma=5.0 / 3.0, prec="f32", store_sums=False):
    """volume -> corrections -> accel/energy; returns a dict of device tensors
    (with M, the moment sums for the backward, when store_sums is true)."""
    V, rho = crk_volume(leaves, gas, prec)
    nf = torch.zeros(1, dtype=torch.int64, device=gas["x"].device)
    corr = crk_corrections(leaves, gas, V, prec, n_fallback=nf, store_sums=store_sums)
    a, du, tot = crk_accel_energy(leaves, gas, V, rho, corr, gamma, prec)
    out = dict(V=V, rho=rho, A=corr[0], B=corr[1], dA=corr[2], dB=corr[3], a=a, dudt=du,
               totals=tot, n_fallback=nf)
    if store_sums:
        out["M"] = corr[4]
    return out


def gas_to_device(cfg, prec="f32", device="cuda"):
    """Copy a synthetic configuration's arrays to the device in the call's precision."""
    dt = _DTYPE[prec]
    g = {}
    for k in ("x", "y", "z"):
        g[k] = torch.as_tensor(cfg[k], dtype=torch.float64).to(device)
    for k in ("vx", "vy", "vz", "u", "h", "m"):
        if k in cfg:
            g[k] = torch.as_tensor(cfg[k]).to(dt).to(device)
    return g
