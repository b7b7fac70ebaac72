"""Vacuum PSATD step (oracles O1 and O2).

Test infrastructure only (see ``oracle/__init__``).

What is computed (Sec. II.A, Eqs. (3)-(4), notation of Eqs. (1)-(2)):
for every plane-wave mode k of the periodic grid, with kappa = |k|,
k_hat = k / kappa, C = cos(c kappa dt), S = sin(c kappa dt),

    E' = C (E - k_hat (k_hat . E)) + i S k_hat x B
    B' = C B - i S k_hat x E

applied to the Fourier coefficients of E and B, followed by the inverse
transform.  The longitudinal part of E is removed at every step, as the
paper does (Sec. II.A, text before Eq. (3)).

Readings where the paper is silent:

* the forward transform uses exp(-i k.x) (so grad -> +ik);
* k_hat := 0 at k = 0, so the DC mode is left unchanged;
* on an even axis the Nyquist index contributes 0 to k (to |k| and to
  k_hat), which keeps M(-k) = conj M(k) and so keeps fields real;
* ``project_b=True`` also removes the longitudinal part of B (used once
  at initialisation; Eq. (4) alone would make it oscillate as C).

Field arrays have shape (3, nz, ny, nx): component, z, y, x with x fastest,
matching the library's [component][z][y][x] layout.

With a current density j (``update_with_current``, ``step_fft_current``)
the step is Eqs. (1)-(2) as printed, with j the coefficients of the current
held over the step (j^{n+1/2}):

    E' = C E + i S k_hat x B - (4 pi S / (kappa c)) j + (1 - C) k_hat (k_hat . E)
         + 4 pi k_hat (k_hat . j) (S / (kappa c) - dt)
    B' = C B - i S k_hat x E + 4 pi i ((1 - C) / (kappa c)) k_hat x j

(CGS units).  The longitudinal part of E is kept and changes by
-4 pi dt (k_hat . j), as Gauss's law with charge continuity requires.
Reading: at kappa = 0 (k = 0, and modes whose only nonzero index is a
Nyquist index) S / (kappa c) is taken at its limit dt and (1 - C) / (kappa c)
at its limit 0, so a uniform current gives E' = E - 4 pi dt j, B' = B.
"""
import numpy as np
import scipy.fft

from . import dft

C_LIGHT = 1.0


def signed_index(n):
    """Signed mode number of each DFT index on an axis of length n (Nyquist -> 0)."""
    m = np.arange(n)
    s = np.where(m <= (n - 1) // 2, m, m - n).astype(np.float64)
    if n % 2 == 0:
        s[n // 2] = 0.0
    return s


def half_index(n):
    """Signed mode numbers of the rfft half axis 0..n/2 (Nyquist -> 0)."""
    s = np.arange(n // 2 + 1, dtype=np.float64)
    if n % 2 == 0:
        s[n // 2] = 0.0
    return s


def wavevector(shape, spacing, half_x):
    """k-space grid (kx, ky, kz), each broadcastable to the spectral shape.

    shape = (nz, ny, nx); spacing = (dz, dy, dx).  With ``half_x`` the x
    axis is the rfft half axis.
    """
    nz, ny, nx = shape
    dz, dy, dx = spacing
    sx = half_index(nx) if half_x else signed_index(nx)
    kx = (2.0 * np.pi / (nx * dx)) * sx
    ky = (2.0 * np.pi / (ny * dy)) * signed_index(ny)
    kz = (2.0 * np.pi / (nz * dz)) * signed_index(nz)
    return (kx[None, None, :], ky[None, :, None], kz[:, None, None])


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1],
            a[2] * b[0] - a[0] * b[2],
            a[0] * b[1] - a[1] * b[0])


def update(Eh, Bh, k, dt, project_b=False, c=C_LIGHT):
    """Eqs. (3)-(4) applied to every mode.  Eh, Bh: sequences of 3 complex
    arrays; k: (kx, ky, kz) broadcastable real arrays.  Returns (E', B')."""
    kx, ky, kz = k
    kappa = np.sqrt(kx * kx + ky * ky + kz * kz)
    nz = kappa > 0
    inv = np.where(nz, 1.0 / np.where(nz, kappa, 1.0), 0.0)
    kh = (kx * inv, ky * inv, kz * inv)                        # k_hat = 0 at k = 0
    C = np.cos(c * kappa * dt)
    S = np.sin(c * kappa * dt)
    kE = kh[0] * Eh[0] + kh[1] * Eh[1] + kh[2] * Eh[2]
    ET = [Eh[a] - kh[a] * kE for a in range(3)]
    if project_b:
        kB = kh[0] * Bh[0] + kh[1] * Bh[1] + kh[2] * Bh[2]
        Bh = [Bh[a] - kh[a] * kB for a in range(3)]
    kxB = _cross(kh, Bh)
    kxE = _cross(kh, Eh)
    En = [C * ET[a] + 1j * S * kxB[a] for a in range(3)]
    Bn = [C * Bh[a] - 1j * S * kxE[a] for a in range(3)]
    return En, Bn


def update_with_current(Eh, Bh, Jh, k, dt, project_b=False, c=C_LIGHT):
    """Eqs. (1)-(2) applied to every mode: Eh, Bh, Jh sequences of 3 complex
    arrays (Jh the current held over the step); k as in ``update``;
    ``project_b`` first removes the longitudinal part of B (as ``update``).
    Returns (E', B')."""
    kx, ky, kz = k
    kappa = np.sqrt(kx * kx + ky * ky + kz * kz)
    nz = kappa > 0
    safe = np.where(nz, kappa, 1.0)
    inv = np.where(nz, 1.0 / safe, 0.0)
    kh = (kx * inv, ky * inv, kz * inv)
    C = np.cos(c * kappa * dt)
    S = np.sin(c * kappa * dt)
    s_over = np.where(nz, S / (safe * c), dt)                 # S / (kappa c) -> dt at kappa = 0
    c_over = np.where(nz, (1.0 - C) / (safe * c), 0.0)        # (1 - C) / (kappa c) -> 0
    if project_b:
        kB = kh[0] * Bh[0] + kh[1] * Bh[1] + kh[2] * Bh[2]
        Bh = [Bh[a] - kh[a] * kB for a in range(3)]
    kE = kh[0] * Eh[0] + kh[1] * Eh[1] + kh[2] * Eh[2]
    kJ = kh[0] * Jh[0] + kh[1] * Jh[1] + kh[2] * Jh[2]
    kxB = _cross(kh, Bh)
    kxE = _cross(kh, Eh)
    kxJ = _cross(kh, Jh)
    En = [C * Eh[a] + 1j * S * kxB[a] - 4.0 * np.pi * s_over * Jh[a] + (1.0 - C) * kh[a] * kE
          + 4.0 * np.pi * kh[a] * kJ * (s_over - dt) for a in range(3)]
    Bn = [C * Bh[a] - 1j * S * kxE[a] + 4.0j * np.pi * c_over * kxJ[a] for a in range(3)]
    return En, Bn


def step_fft_current(E, B, J, spacing, dt, project_b=False, workers=None):
    """One step of Eqs. (1)-(2) with the real current density J (shape
    (3, nz, ny, nx)) held over the step: rfftn -> update_with_current ->
    irfftn, in float64."""
    workers = workers or _workers()
    shape = E.shape[1:]
    k = wavevector(shape, spacing, half_x=True)
    Eh = [scipy.fft.rfftn(np.asarray(E[a], np.float64), workers=workers) for a in range(3)]
    Bh = [scipy.fft.rfftn(np.asarray(B[a], np.float64), workers=workers) for a in range(3)]
    Jh = [scipy.fft.rfftn(np.asarray(J[a], np.float64), workers=workers) for a in range(3)]
    En, Bn = update_with_current(Eh, Bh, Jh, k, dt, project_b)
    E = np.stack([scipy.fft.irfftn(x, s=shape, workers=workers) for x in En])
    B = np.stack([scipy.fft.irfftn(x, s=shape, workers=workers) for x in Bn])
    return E, B


def step_direct(E, B, spacing, dt, project_b=False):
    """One step with the full complex direct DFT (oracle O1).

    Returns real float64 arrays; asserts that the imaginary residue of the
    inverse is at rounding level (pins the Nyquist reading)."""
    shape = E.shape[1:]
    k = wavevector(shape, spacing, half_x=False)
    Eh = [dft.dftn(E[a]) for a in range(3)]
    Bh = [dft.dftn(B[a]) for a in range(3)]
    En, Bn = update(Eh, Bh, k, dt, project_b)
    out = []
    for arrs in (En, Bn):
        comp = [dft.idftn(x) for x in arrs]
        re = np.stack([x.real for x in comp])
        im = np.stack([x.imag for x in comp])
        scale = max(np.abs(re).max(), 1e-300)
        assert np.abs(im).max() <= 1e-11 * scale, "non-real inverse (Nyquist reading)"
        out.append(re)
    return out[0], out[1]


def _workers():
    return max(1, len(__import__("os").sched_getaffinity(0)))


def step_fft(E, B, spacing, dt, nsteps=1, project_b_first=False,
             workers=None):
    """``nsteps`` steps of dt with scipy's real FFT (oracle O2).

    Every step is forward rfftn -> Eqs. (3)-(4) -> inverse irfftn, as the
    method's iteration.  ``project_b_first`` removes longitudinal B in the first step.
    """
    workers = workers or _workers()
    shape = E.shape[1:]
    k = wavevector(shape, spacing, half_x=True)
    E = np.array(E, dtype=np.float64, copy=True)
    B = np.array(B, dtype=np.float64, copy=True)
    for s in range(nsteps):
        Eh = [scipy.fft.rfftn(E[a], workers=workers) for a in range(3)]
        Bh = [scipy.fft.rfftn(B[a], workers=workers) for a in range(3)]
        En, Bn = update(Eh, Bh, k, dt, project_b=(project_b_first and s == 0))
        E = np.stack([scipy.fft.irfftn(x, s=shape, workers=workers) for x in En])
        B = np.stack([scipy.fft.irfftn(x, s=shape, workers=workers) for x in Bn])
    return E, B


def jump(E, B, spacing, T, project_b=False, workers=None):
    """Advance by T in a single step (exact for any interval, Sec. II.A)."""
    return step_fft(E, B, spacing, T, 1, project_b, workers)


def energy(E, B):
    """Sum over cells of E^2 + B^2 (a conserved quantity of the step)."""
    return float(np.sum(E * E) + np.sum(B * B))


def max_divergence(E, B, spacing, workers=None):
    """max |k_hat . E_hat| and max |k_hat . B_hat| over all modes, divided by
    max |E_hat| resp. max |B_hat| (0 for a purely transverse field)."""
    workers = workers or _workers()
    shape = E.shape[1:]
    kx, ky, kz = wavevector(shape, spacing, half_x=True)
    kappa = np.sqrt(kx * kx + ky * ky + kz * kz)
    inv = np.where(kappa > 0, 1.0 / np.where(kappa > 0, kappa, 1.0), 0.0)
    res = []
    for F in (E, B):
        Fh = [scipy.fft.rfftn(F[a], workers=workers) for a in range(3)]
        kd = (kx * Fh[0] + ky * Fh[1] + kz * Fh[2]) * inv
        top = max(max(np.abs(x).max() for x in Fh), 1e-300)
        res.append(float(np.abs(kd).max() / top))
    return tuple(res)
