"""Seeded superpositions of vacuum plane-wave eigenmodes.

A mode is (m, e, amp, phase, sign): integer mode numbers m (k = 2 pi m /
(N d) per axis), a unit polarisation e perpendicular to m, an amplitude, a
phase and a propagation sign s = +-1.  At t = 0 its fields on the grid are
E = amp e cos(k.x + phase) and B = s amp (k/|k| x e) cos(k.x + phase).
"""
import numpy as np


def draw(seed, nmodes=16, mmax=31, amp=(0.5, 1.0)):
    rng = np.random.default_rng(seed)
    modes = []
    while len(modes) < nmodes:
        m = rng.integers(-mmax, mmax + 1, size=3)
        if not m.any():
            continue
        v = rng.normal(size=3)
        mh = m / np.linalg.norm(m)
        e = v - mh * (mh @ v)
        e /= np.linalg.norm(e)
        modes.append(dict(m=m.astype(np.int64), e=e,
                          amp=float(rng.uniform(*amp)),
                          phase=float(rng.uniform(0.0, 2.0 * np.pi)),
                          sign=int(rng.choice([-1, 1]))))
    return modes


def node_coords(grid):
    x = grid["x_min"] + np.arange(grid["nx"]) * grid["dx"]
    y = grid["y_min"] + np.arange(grid["ny"]) * grid["dy"]
    z = grid["z_min"] + np.arange(grid["nz"]) * grid["dz"]
    return x, y, z


def kvec(mode, grid):
    n = (grid["nx"], grid["ny"], grid["nz"])
    d = (grid["dx"], grid["dy"], grid["dz"])
    return np.array([2.0 * np.pi * mode["m"][a] / (n[a] * d[a]) for a in range(3)])


def fields(modes, grid, dtype=np.float64):
    """E, B at t = 0, each of shape (3, nz, ny, nx)."""
    x, y, z = node_coords(grid)
    shape = (grid["nz"], grid["ny"], grid["nx"])
    E = np.zeros((3,) + shape)
    B = np.zeros((3,) + shape)
    for md in modes:
        k = kvec(md, grid)
        ph = (k[0] * x[None, None, :] + k[1] * y[None, :, None]
              + k[2] * z[:, None, None] + md["phase"])
        c = md["amp"] * np.cos(ph)
        kh = k / np.linalg.norm(k)
        b = md["sign"] * np.cross(kh, md["e"])
        for a in range(3):
            E[a] += md["e"][a] * c
            B[a] += b[a] * c
    return E.astype(dtype), B.astype(dtype)


def random_fields(seed, shape, dtype=np.float64):
    """Unstructured seeded fields (not transverse), shape (3, nz, ny, nx) x2."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((3,) + tuple(shape)).astype(dtype),
            rng.standard_normal((3,) + tuple(shape)).astype(dtype))
