"""Small hand-made particle sets shared by the GPU tests."""

import numpy as np

import synth


def fallback_case():
    """240 random particles, a tenth of them with h for only 2 neighbours: the
    singular-moment fallback (fewer than 4 neighbours) triggers for those."""
    rng = np.random.default_rng(21)
    n = 240
    x, y, z = (synth.grid_round(rng.random(n)) for _ in range(3))
    target = np.where(rng.random(n) < 0.1, 2, 18)
    H = synth.knn_support(x, y, z, target)
    return dict(n=n, x=x, y=y, z=z, h=synth.f32(0.5 * H), m=synth.f32(np.full(n, 1.0 / n)),
                vx=synth.f32(rng.normal(0, 0.1, n)), vy=synth.f32(rng.normal(0, 0.1, n)),
                vz=synth.f32(rng.normal(0, 0.1, n)), u=synth.f32(np.exp(0.5 * rng.normal(size=n))),
                gamma=5.0 / 3.0, w=rng.random(n), c=rng.random(n))


def planar_case():
    """A jittered 12 x 12 sheet of particles in the plane z = 1/2: many
    neighbours, but the second moment m2 has no z extent, so every particle
    takes the determinant branch of the fallback."""
    rng = np.random.default_rng(8)
    k = 12
    gx, gy = np.meshgrid((np.arange(k) + 0.5) / k, (np.arange(k) + 0.5) / k, indexing="ij")
    n = k * k
    x = synth.grid_round(gx.ravel() + rng.normal(0, 0.05 / k, n))
    y = synth.grid_round(gy.ravel() + rng.normal(0, 0.05 / k, n))
    z = synth.grid_round(np.full(n, 0.5))
    return dict(n=n, x=x, y=y, z=z, h=synth.f32(np.full(n, 1.3 / k)), m=synth.f32(np.full(n, 1.0 / n)),
                vx=synth.f32(rng.normal(0, 0.1, n)), vy=synth.f32(rng.normal(0, 0.1, n)),
                vz=np.zeros(n), u=np.ones(n), gamma=5.0 / 3.0)


def dense_case():
    """6000 random particles with h for about 600 neighbours: the neighbours of
    a tile's 64 particles number more than the list schedule's table holds, so
    its tiles keep their fill order with one-per-lane staging sets."""
    rng = np.random.default_rng(17)
    n = 6000
    x, y, z = (synth.grid_round(rng.random(n)) for _ in range(3))
    H = synth.knn_support(x, y, z, np.full(n, 600))
    return dict(n=n, x=x, y=y, z=z, h=synth.f32(0.5 * H), m=synth.f32(np.full(n, 1.0 / n)),
                vx=synth.f32(rng.normal(0, 0.1, n)), vy=synth.f32(rng.normal(0, 0.1, n)),
                vz=synth.f32(rng.normal(0, 0.1, n)), u=synth.f32(np.exp(0.5 * rng.normal(size=n))),
                gamma=5.0 / 3.0)
