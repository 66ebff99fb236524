"""Seeded velocity fields sampled at vertex positions.

Both generators are functions of position, so any two producers of the same
vertex set (in any order) obtain the same velocity degrees of freedom.
"""
import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x):
    """SplitMix64 finaliser (Steele, Lea & Flood 2014), on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def normal_field(coords, seed, quantum=2.0 ** -26):
    """i.i.d. N(0,1) per (vertex, component), keyed by the quantised position.

    A counter-based generator: SplitMix64 over (seed, quantised x, y, z,
    component, draw), two 53-bit uniforms per value, Box-Muller transform.
    Returns float64 [n, 3].
    """
    X = np.asarray(coords, dtype=np.float64)
    q = np.rint(X / quantum).astype(np.int64).view(np.uint64)
    with np.errstate(over="ignore"):
        base = _splitmix64(np.uint64(seed) * np.uint64(0xD1342543DE82EF95) & _M64)
        h = base
        h = _splitmix64(h ^ q[:, 0])
        h = _splitmix64(h ^ q[:, 1])
        h = _splitmix64(h ^ q[:, 2])
        out = np.empty((len(X), 3))
        for c in range(3):
            h1 = _splitmix64(h ^ np.uint64(2 * c + 1))
            h2 = _splitmix64(h ^ np.uint64(2 * c + 2))
            u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
            u2 = ((h2 >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
            out[:, c] = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return out


def fourier_modes(seed, n_modes=32, kmax=8):
    """Draw (k_m, a_m, phi_m) in the order k, g, phi per mode."""
    rng = np.random.default_rng(seed)
    ks, amps, phis = [], [], []
    for _ in range(n_modes):
        while True:
            k = rng.integers(-kmax, kmax + 1, size=3)
            nk = float(np.linalg.norm(k))
            if 1.0 <= nk <= kmax:
                break
        g = rng.standard_normal(3)
        a = g / np.linalg.norm(g)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        ks.append(k)
        amps.append(a)
        phis.append(phi)
    return np.array(ks, dtype=np.float64), np.array(amps), np.array(phis)


def fourier_field(coords, seed, n_modes=32, kmax=8):
    """u(x) = sum_m |k_m|^-1 a_m cos(2 pi k_m . x + phi_m), float64 [n, 3]."""
    X = np.asarray(coords, dtype=np.float64)
    k, a, phi = fourier_modes(seed, n_modes, kmax)
    nk = np.linalg.norm(k, axis=1)
    arg = 2.0 * np.pi * (X @ k.T) + phi[None, :]
    return np.cos(arg) @ (a / nk[:, None])
