"""Direct discrete Fourier transform (oracle O1).

Test infrastructure only (see ``oracle/__init__``).

The spectral solver of Sec. II.A needs a forward and an inverse transform
between the grid and plane-wave eigenmodes.  Here both are the plain DFT
definition applied axis by axis with explicit float64 matrices:

    F[m] = sum_j f[j] exp(-2 pi i m j / N)          (forward, sign -1)
    f[j] = (1/N) sum_m F[m] exp(+2 pi i m j / N)     (inverse, sign +1)

The phase of every matrix entry is built from the exact integer
r = (m * j) mod N, so no large argument ever reaches ``exp``.  Cost is
O(N^4) per 3-D component, so this is for grids up to about 64 per axis.
"""
import numpy as np


def dft_matrix(n, sign):
    """n x n DFT matrix exp(sign * 2 pi i (m j mod n) / n)."""
    idx = np.arange(n, dtype=np.int64)
    r = np.outer(idx, idx) % n
    return np.exp(sign * 2j * np.pi * r.astype(np.float64) / n)


def _apply_axis(a, mat, axis):
    a = np.moveaxis(a, axis, -1)
    out = a @ mat.T
    return np.moveaxis(out, -1, axis)


def dftn(f, axes=(-3, -2, -1)):
    """Full complex forward DFT over ``axes`` (no Hermitian halving)."""
    out = np.asarray(f, dtype=np.complex128)
    for ax in axes:
        out = _apply_axis(out, dft_matrix(out.shape[ax], -1), ax)
    return out


def idftn(F, axes=(-3, -2, -1)):
    """Full complex inverse DFT over ``axes``, including the 1/N factors."""
    out = np.asarray(F, dtype=np.complex128)
    for ax in axes:
        n = out.shape[ax]
        out = _apply_axis(out, dft_matrix(n, +1), ax) / n
    return out
