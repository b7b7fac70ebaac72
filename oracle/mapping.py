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
on nodes) and y, z must stay inside the grid (no transverse wrap).
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
    if J.min() < 0 or J.max() >= grid["ny"] or K.min() < 0 or K.max() >= grid["nz"]:
        raise ValueError("window leaves the transverse extent of the grid")
    return I, J, K


def readout(fields6, grid, win, t, R_min, R_max):
    """Focal window (6, wz, wy, wx) cut out of layer fields (6, nz, ny, nx)."""
    I, J, K = window_nodes(grid, win)
    ix = np.mod(I, grid["nx"])                                   # T on nodes
    x = grid["x_min"] + I * grid["dx"]
    y = grid["y_min"] + J * grid["dy"]
    z = grid["z_min"] + K * grid["dz"]
    mask = indicator(x[None, None, :], y[None, :, None], z[:, None, None],
                     t, R_min, R_max)
    sub = fields6[:, K][:, :, J][:, :, :, ix]
    return sub * mask[None]
