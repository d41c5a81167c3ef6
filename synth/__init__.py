"""Seeded synthetic particle sets for the CRK-SPH and short-range gravity passes.

This module only *makes inputs*: positions, smoothing lengths, masses,
velocities, internal energies and loss weights.  It holds none of the method's
arithmetic (no smoothing kernel, no moments, no forces) and is shared by the
CPU oracle's tests and by the GPU path's tests and benchmark; neither of those
is imported here.

Stand-in for the paper's workload.  The paper runs CRK-HACC in adiabatic mode
on 2x512^3 particles (dark matter + gas) split over 8 ranks, i.e. 2x256^3 per
GPU (Sec. 3.4, "Problem Size"), from HACC initial conditions that are not
available here.  These generators produce seeded, clustered particle sets of
the same per-GPU sizes instead:

* periodic unit box; positions on the 2^-32 grid (so that every separation is
  exact in FP64 and a signed 32-bit difference in fixed point);
* every other field rounded to FP32, stored as float64, so one FP64 oracle run
  serves both the FP32 and the FP64 GPU paths;
* clustering: Gaussian random field with P(k) ~ k^-2 on an n_g^3 grid,
  lognormal density exp(sigma g - sigma^2/2) with sigma = 1, particles placed
  multinomially over cells and uniformly inside a cell;
* smoothing length h_i chosen so that particle i has a prescribed number of
  neighbours j != i with |x_ij| < 2 h_i (k-nearest-neighbour distances from a
  periodic k-d tree, midway between the n-th and (n+1)-th neighbour).

Named configurations (sizes as the benchmark uses them):

  C1  16^3 jittered lattice, uniform h = 1.3 spacing, u = 1    (FP64 parity)
  C2  128^3 clustered gas, h for 64 +- 8 neighbours            (throughput)
  C3  128^3 gas + 128^3 dark matter, Plummer-softened gravity  (gravity)
  C4  64^3 clustered gas with loss weights w, c ~ U(0,1)       (backward)
  C5  256^3 clustered gas, 32..256 neighbours over a 16x density contrast

Every configuration can be shrunk with ``n_side`` for tests (same recipe).
"""

from __future__ import annotations

import sys

import numpy as np

GRID = 2.0 ** 32
SEED_BASE = {"C1": 1001, "C2": 1002, "C3": 1003, "C4": 1004, "C5": 1005}
GAMMA = 5.0 / 3.0


def grid_round(x):
    """Round positions to the 2^-32 grid of the unit periodic box, in [0, 1)."""
    q = np.floor(np.asarray(x, dtype=np.float64) * GRID + 0.5)
    q = np.mod(q, GRID)
    return q / GRID


def to_u32(x):
    """Fixed-point image of grid positions (exact for grid values)."""
    return (np.asarray(x, dtype=np.float64) * GRID).astype(np.uint64).astype(np.uint32)


def f32(a):
    """Round to the nearest FP32 value, returned as float64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _streams(name, k=8):
    ss = np.random.SeedSequence(SEED_BASE[name])
    return [np.random.default_rng(s) for s in ss.spawn(k)]


def gaussian_field(n_g, rng):
    """Unit-variance Gaussian random field with power spectrum P(k) ~ k^-2 (k=0 removed)."""
    white = rng.standard_normal((n_g, n_g, n_g))
    fk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(n_g) * n_g
    kz = np.fft.rfftfreq(n_g) * n_g
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = 1.0 / np.sqrt(k2[nz])  # sqrt(P), P ~ k^-2
    g = np.fft.irfftn(fk * amp, s=(n_g, n_g, n_g), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def lognormal_density(n_g, rng, sigma=1.0):
    g = gaussian_field(n_g, rng)
    return np.exp(sigma * g - 0.5 * sigma * sigma)


def place_particles(rho_cell, n, rng):
    """Multinomial placement over cells (p ~ rho), uniform inside each cell."""
    n_g = rho_cell.shape[0]
    p = rho_cell.ravel() / rho_cell.sum()
    counts = rng.multinomial(n, p)
    cell = np.repeat(np.arange(p.size, dtype=np.int64), counts)
    rng.shuffle(cell)
    ix = cell // (n_g * n_g)
    iy = (cell // n_g) % n_g
    iz = cell % n_g
    u = rng.random((n, 3))
    x = (ix + u[:, 0]) / n_g
    y = (iy + u[:, 1]) / n_g
    z = (iz + u[:, 2]) / n_g
    return grid_round(x), grid_round(y), grid_round(z), cell


def knn_support(x, y, z, n_target, chunk=1 << 18, workers=-1):
    """Support radius H_i = 2 h_i with exactly n_target[i] neighbours j != i inside H_i.

    H_i is placed midway between the n-th and (n+1)-th nearest non-self
    neighbour distances (periodic unit box).  Pure input construction.
    """
    from scipy.spatial import cKDTree

    pts = np.stack([x, y, z], axis=1)
    tree = cKDTree(pts, boxsize=1.0)
    n_target = np.asarray(n_target, dtype=np.int64)
    H = np.empty(len(x))
    # particles with similar targets are queried together with k = group max + 2
    kq = (n_target + 2 + 15) // 16 * 16
    verbose = len(x) >= (1 << 22)
    for k in np.unique(kq):
        if verbose:
            print(f"[synth] neighbour search k={int(k)} for {int((kq == k).sum())} particles",
                  file=sys.stderr, flush=True)
        sel = np.nonzero(kq == k)[0]
        for s in range(0, len(sel), max(1, chunk * 64 // int(k))):
            idx = sel[s:s + max(1, chunk * 64 // int(k))]
            d, _ = tree.query(pts[idx], k=int(k), workers=workers)
            nt = n_target[idx]
            rows = np.arange(len(idx))
            # d[:, 0] is the particle itself; d[:, n] is the n-th neighbour
            H[idx] = 0.5 * (d[rows, nt] + d[rows, nt + 1])
    return H


def _gas_fields(n, rng_v, rng_u, v_sigma, u_lognormal):
    vx, vy, vz = (f32(rng_v.normal(0.0, v_sigma, n)) for _ in range(3))
    if u_lognormal:
        u = f32(np.exp(0.5 * rng_u.standard_normal(n)))
    else:
        u = f32(np.ones(n))
    return vx, vy, vz, u


def make_lattice(n_side=16, jitter=0.1, h_factor=1.3, seed_name="C1"):
    """C1: n_side^3 lattice at (k+1/2)/n_side with Gaussian jitter (fraction of spacing)."""
    r_pos, r_v, r_u = _streams(seed_name, 3)
    s = 1.0 / n_side
    k = (np.arange(n_side) + 0.5) * s
    X, Y, Z = np.meshgrid(k, k, k, indexing="ij")
    n = n_side ** 3
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if jitter > 0:
        pos = pos + r_pos.normal(0.0, jitter * s, (n, 3))
    x, y, z = (grid_round(pos[:, a]) for a in range(3))
    h = f32(np.full(n, h_factor * s))
    m = f32(np.full(n, 1.0 / n))
    vx, vy, vz = (f32(r_v.normal(0.0, 0.01, n)) for _ in range(3))
    u = f32(np.ones(n))
    return dict(name="C1", n=n, x=x, y=y, z=z, h=h, m=m, vx=vx, vy=vy, vz=vz, u=u,
                gamma=GAMMA)


def make_clustered_gas(name, n_side, nbr_lo=56, nbr_hi=72, contrast=None):
    """C2 / C4 / C5 recipe at n_side^3 gas particles."""
    r_field, r_pos, r_v, r_u, r_n, r_w, r_c = _streams(name, 7)
    n = n_side ** 3
    rho = lognormal_density(n_side, r_field)
    x, y, z, cell = place_particles(rho, n, r_pos)
    if contrast is None:
        n_target = r_n.integers(nbr_lo, nbr_hi + 1, n)
    else:
        # neighbour target follows the cell density of the lognormal field over
        # a `contrast`-fold range: n = nbr_lo * (rho/rho_lo)^(3/4), rho clipped
        # to [rho_lo, contrast * rho_lo], rho_lo its 5th percentile
        rho_hat = rho.ravel()[cell]
        rho_lo = np.percentile(rho_hat, 5)
        rho_hat = np.clip(rho_hat, rho_lo, contrast * rho_lo)
        n_target = np.rint(nbr_lo * (rho_hat / rho_lo) ** 0.75).astype(np.int64)
        n_target = np.clip(n_target, nbr_lo, nbr_hi)
    H = knn_support(x, y, z, n_target)
    h = f32(0.5 * H)
    m = f32(np.full(n, 1.0 / n))
    vx, vy, vz, u = _gas_fields(n, r_v, r_u, 0.05, True)
    w = f32(r_w.random(n))
    c = f32(r_c.random(n))
    return dict(name=name, n=n, x=x, y=y, z=z, h=h, m=m, vx=vx, vy=vy, vz=vz, u=u,
                gamma=GAMMA, w=w, c=c, n_target=n_target)


def make_gravity(n_side=128, name="C3"):
    """C3: gas + dark matter from one clustered field, m_dm = 5 m_gas, total mass 1."""
    r_field, r_gas, r_dm = _streams(name, 3)
    n = n_side ** 3
    rho = lognormal_density(n_side, r_field)
    xg, yg, zg, _ = place_particles(rho, n, r_gas)
    xd, yd, zd, _ = place_particles(rho, n, r_dm)
    m_gas = 1.0 / (6.0 * n)
    m = f32(np.concatenate([np.full(n, m_gas), np.full(n, 5.0 * m_gas)]))
    spacing = 1.0 / n_side
    return dict(name=name, n=2 * n, n_gas=n,
                x=np.concatenate([xg, xd]), y=np.concatenate([yg, yd]),
                z=np.concatenate([zg, zd]), m=m,
                G=1.0, eps=float(f32(0.02 * spacing)), r_cut=float(f32(3.0 * spacing)))


def make_config(name, n_side=None):
    """Build one named configuration (optionally shrunk to n_side^3 per species)."""
    if name == "C1":
        return make_lattice(n_side or 16)
    if name == "C2":
        return make_clustered_gas("C2", n_side or 128)
    if name == "C3":
        return make_gravity(n_side or 128)
    if name == "C4":
        return make_clustered_gas("C4", n_side or 64)
    if name == "C5":
        return make_clustered_gas("C5", n_side or 256, nbr_lo=32, nbr_hi=256, contrast=16.0)
    raise ValueError(f"unknown configuration {name!r}")


def check_support(cfg):
    """The periodic minimum image needs 2 max(h) < 1/2 (unit box)."""
    H = 2.0 * float(np.max(cfg["h"]))
    if not H < 0.5:
        raise ValueError(f"support 2h_max = {H} is not below half the box")
    return H


def sample_targets(n, k, seed=7):
    """A seeded sample of k distinct particle indices (for sampled parity checks)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int64)
