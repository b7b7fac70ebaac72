"""Cut-out of the primary pulse from the periodic layer (oracle O4).

Test infrastructure only (see ``oracle/__init__``).

Sec. II.C, Eqs. (13)-(16): a point R of the original space takes the field
of the layer point T(R) = (x_min + D {(x - x_min)/D}, y, z), multiplied by
the indicator I_S(t)(R), with l(t) = -R_max + c t and r(t) = -R_min + c t:

  r < 0:          0 if R >= -l or R < -r or x > 0
  l <= 0 <= r:    0 if x < 0 and R > L
                  0 if x >= 0 and R > r       (printed with l: read as r)
  l > 0:          0 if R <= l or R > r or x < 0
  otherwise 1.

Readings: {a} = a - floor(a); t is the time since the start of the run,
so the geometric focus is reached at t = R0/c.  The focal window is
node-aligned: its centre snaps to node floor((c - min)/d + 1/2), node i of
the window is centre + i - w//2 (unwrapped), x wraps modulo nx (this is T
on nodes) and y, z must stay inside the grid, unless the grid replicates
the pulse transversely (replicate_yz), where they wrap alike.  I_S is
discontinuous on its spheres (R = L, R = r(t), ...), which nodes can lie on:
when the origin is a node, a node's coordinate is its integer offset from
the origin times the spacing, so every grid with that spacing decides those
nodes alike (x_min + i dx rounds differently from grid to grid).
"""
import math

import numpy as np

C_LIGHT = 1.0


def indicator(x, y, z, t, R_min, R_max):
    """I_S(t)(R) of Eq. (15), its third case read as x >= 0 and R > r."""
    x, y, z = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (x, y, z)))
    R = np.sqrt(x * x + y * y + z * z)
    L = R_max - R_min
    l = -R_max + C_LIGHT * t
    r = -R_min + C_LIGHT * t
    if r < 0.0:
        zero = (R >= -l) | (R < -r) | (x > 0.0)
    elif l <= 0.0:
        zero = ((x < 0.0) & (R > L)) | ((x >= 0.0) & (R > r))
    else:
        zero = (R <= l) | (R > r) | (x < 0.0)
    return np.where(zero, 0.0, 1.0)


def window_nodes(grid, win):
    """Unwrapped node indices (I, J, K) of the window along x, y, z."""
    idx = []
    for ax, (w, c) in zip("xyz", ((win["wx"], win["cx"]), (win["wy"], win["cy"]),
                                  (win["wz"], win["cz"]))):
        d, lo = grid["d" + ax], grid[ax + "_min"]
        ic = math.floor((c - lo) / d + 0.5)
        idx.append(ic + np.arange(w) - w // 2)
    I, J, K = idx
    if not grid.get("replicate_yz") and (J.min() < 0 or J.max() >= grid["ny"] or K.min() < 0
                                         or K.max() >= grid["nz"]):
        raise ValueError("window leaves the transverse extent of the grid")
    return I, J, K


def node_coords(I, lo, d):
    """Coordinates of nodes I along an axis starting at lo with spacing d:
    integer offsets from the origin node times d when the origin is a node."""
    o = lo / d
    r = round(o)
    if abs(o - r) <= 1e-6:
        return (np.asarray(I, dtype=np.int64) + r).astype(np.float64) * d
    return lo + np.asarray(I) * d


def readout(fields6, grid, win, t, R_min, R_max):
    """Focal window (6, wz, wy, wx) cut out of layer fields (6, nz, ny, nx)."""
    I, J, K = window_nodes(grid, win)
    ix = np.mod(I, grid["nx"])                                   # T on nodes
    x = node_coords(I, grid["x_min"], grid["dx"])
    y = node_coords(J, grid["y_min"], grid["dy"])
    z = node_coords(K, grid["z_min"], grid["dz"])
    mask = indicator(x[None, None, :], y[None, :, None], z[:, None, None],
                     t, R_min, R_max)
    jy, kz = (np.mod(J, grid["ny"]), np.mod(K, grid["nz"])) if grid.get("replicate_yz") else (J, K)
    sub = fields6[:, kz][:, :, jy][:, :, :, ix]
    return sub * mask[None]
