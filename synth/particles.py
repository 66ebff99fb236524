"""Seeded particle sets for the simulation-step workloads.

The paper seeds eight particles per background cell (Sec. 6).  Here each cell
gets a 2 x 2 x 2 lattice of particles, each jittered by up to a quarter of
its sub-cell; the smoke density and temperature are 1 inside a spherical
emitter and 0 elsewhere; velocities come from the seeded Fourier field.
This module only generates inputs.
"""
import numpy as np

from .fields import fourier_field


def seeded_particles(N, seed=0, emitter=((0.5, 0.5, 0.15), 0.1), velocity_seed=0):
    """Positions [8 N^3, 3], velocities [8 N^3, 3], density and temperature [8 N^3]."""
    rng = np.random.default_rng(seed)
    h = 1.0 / N
    i = np.arange(N)
    cx, cy, cz = np.meshgrid(i, i, i, indexing="ij")
    base = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.float64)
    sub = np.array([[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)], dtype=np.float64)
    pos = (base[:, None, :] + (sub[None, :, :] + 0.5) / 2.0).reshape(-1, 3)
    pos += rng.uniform(-0.25, 0.25, size=pos.shape) / 2.0
    x = pos * h
    vel = fourier_field(x, velocity_seed).reshape(-1, 3)
    c, r = np.asarray(emitter[0]), emitter[1]
    inside = ((x - c) ** 2).sum(axis=1) <= r * r
    rho = inside.astype(np.float64)
    temp = inside.astype(np.float64)
    return x, vel, rho, temp
