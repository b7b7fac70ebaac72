"""Fourier neural operator: forward and manual backward in float64 (oracle O5).

Test infrastructure only (see ``oracle/__init__``).  Parity unpinned by the
paper, which only motivates learned models trained on many focusing runs
(Sec. I, last paragraph; Sec. III.B.3): this module is pinned by finite
differences, by the spectral convolution reproducing band-limited fields
exactly, and by translation equivariance.

Definition (one sample; x runs over the N^3 window nodes):
  a(x)    = [p (8 pulse parameters in [0, 1]), c(x) (3 coordinates in [-1, 1))]
  v0      = a W0 + b0                                   (lift, width C)
  layer l = 0..L-1:
    Xh    = rfftn(v_l)[modes]                           (per channel)
    Yh[k] = Xh[k] R_l[k]                                 (complex C x C per mode)
    u     = irfftn(Yh on the kept modes, 0 elsewhere)
    z_l   = u + v_l W_l + b_l
    v_l+1 = GELU(z_l) for l < L-1, z_L-1 for the last layer
  h       = GELU(v_L P1 + c1)                           (hidden H)
  o       = h P2 + c2                                   (6 K channels)
  out     = sum_k w[k] o[6k : 6k + 6]                   (6 field components)
With K = 1 and w = 1 (the plain head) out = o.  With K = 4 (the phasor head)
the channels are the real and imaginary parts of two complex basis fields and
w holds, per sample, the exact weights of the pulse's carrier phase and
polarisation (oracle.pulse.phasor_weights).
Kept modes: kx in [0, M) on the rfft axis, ky and kz in [0, M) U [N-M, N)
(the usual truncation; the set is not closed under negation, so in the
kx = 0 plane the index N-M has no kept partner).
Padded spectral transform (period P > N, ``HP.period``): v is extended by
zeros to a P^3 block, rfftn and irfftn run with period P (kept modes
[0, M) U [P-M, P) along y and z, [0, M) along x), and the inverse is cut
back to the N^3 window: u = crop(irfftn_P(Yh)).  A window whose fields do
not match across opposite faces is then not forced into an N-periodic
band-limited form (the usual padding of Fourier neural operators on
non-periodic domains).  P = N is the plain transform.
Mode order q = (kz_i * 2M + ky_i) * M + kx, ky_i / kz_i indexing the kept
list ascending.  GELU(x) = x (1 + erf(x / sqrt 2)) / 2.
Loss of a batch: mean over samples of ||out - y|| / ||y||.

Training update (``adam_step``): Adam with bias correction (Kingma and Ba,
"Adam: a method for stochastic optimization", ICLR 2015, Algorithm 1), in
float64 on flat parameter vectors: with g the gradient of step t = 1, 2, ...
  m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,
  p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
Pinned by closed forms: the first step moves every parameter by
lr g / (|g| + eps); a constant gradient keeps that step at every t (the bias
corrections undo the zero start exactly); alternating g, -g gives the
second step lr (1 - b1) / (1 + b1) g / (|g| + eps) backwards.
"""
import math

import numpy as np
import scipy.fft
import scipy.special


class HP:
    def __init__(self, n=64, width=32, modes=12, nparam=8, hidden=128, nout=6, layers=3, nbasis=1, period=None):
        self.n, self.width, self.modes = n, width, modes
        self.nparam, self.hidden, self.nout, self.layers = nparam, hidden, nout, layers
        self.nbasis = nbasis
        self.period = n if period is None else int(period)
        assert self.period >= n

    @property
    def nmodes(self):
        return 4 * self.modes ** 3


def kept_index(hp):
    """Arrays (kz, ky, kx) of the kept modes in the canonical order."""
    M, P = hp.modes, hp.period
    side = np.concatenate([np.arange(M), np.arange(P - M, P)])
    kz, ky, kx = np.meshgrid(side, side, np.arange(M), indexing="ij")
    return kz.ravel(), ky.ravel(), kx.ravel()


def coords(hp):
    g = (np.arange(hp.n) - hp.n // 2) / (hp.n // 2)
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([cx, cy, cz])                       # x, y, z coordinate channels


def init_params(seed, hp):
    rng = np.random.default_rng(seed)
    C, H = hp.width, hp.hidden
    nin = hp.nparam + 3
    P = {"W0": rng.normal(0, 1 / math.sqrt(nin), (nin, C)), "b0": np.zeros(C),
         "P1": rng.normal(0, 1 / math.sqrt(C), (C, H)), "c1": np.zeros(H),
         "P2": rng.normal(0, 1 / math.sqrt(H), (H, hp.nout * hp.nbasis)), "c2": np.zeros(hp.nout * hp.nbasis)}
    scale = 1.0 / (C * C)
    for l in range(hp.layers):
        P[f"W{l + 1}"] = rng.normal(0, 1 / math.sqrt(C), (C, C))
        P[f"b{l + 1}"] = np.zeros(C)
        P[f"R{l + 1}"] = scale * (rng.uniform(size=(hp.nmodes, C, C)) + 1j * rng.uniform(size=(hp.nmodes, C, C)))
    return P


def gelu(x):
    return 0.5 * x * (1.0 + scipy.special.erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + scipy.special.erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def spectral_forward(v, hp):
    """v: (B, C, N, N, N) real -> kept rfftn coefficients (B, C, nmodes) of
    v extended by zeros to the period P."""
    P = hp.period
    kz, ky, kx = kept_index(hp)
    Xf = scipy.fft.rfftn(v, s=(P, P, P), axes=(2, 3, 4))
    return Xf[:, :, kz, ky, kx]


def spectral_inverse(Yh, hp):
    """Kept coefficients (B, C, nmodes) -> irfftn of period P with zeros
    elsewhere, cut to the N^3 window."""
    N, P = hp.n, hp.period
    kz, ky, kx = kept_index(hp)
    full = np.zeros(Yh.shape[:2] + (P, P, P // 2 + 1), dtype=np.complex128)
    full[:, :, kz, ky, kx] = Yh
    return scipy.fft.irfftn(full, s=(P, P, P), axes=(2, 3, 4))[:, :, :N, :N, :N]


def _mult(hp):
    """Hermitian multiplicity of each kept mode under irfftn (1 at kx = 0)."""
    _, _, kx = kept_index(hp)
    return np.where(kx == 0, 1.0, 2.0)


def inputs(pb, hp):
    """(B, 11, N, N, N) lift inputs: broadcast parameters + coordinates."""
    B = pb.shape[0]
    N = hp.n
    a = np.empty((B, hp.nparam + 3, N, N, N))
    a[:, :hp.nparam] = pb[:, :, None, None, None]
    a[:, hp.nparam:] = coords(hp)[None]
    return a


def _pw(x, W, b):
    """Pointwise linear over channels: (B, Cin, ...) x (Cin, Cout) + b."""
    return np.einsum("bi...,io->bo...", x, W) + b[None, :, None, None, None]


def _outer(x, g):
    """sum over samples and nodes of x_i g_o: (B, Ci, ...), (B, Co, ...) -> (Ci, Co)."""
    B = x.shape[0]
    return np.einsum("bis,bos->io", x.reshape(B, x.shape[1], -1), g.reshape(B, g.shape[1], -1))


def _weights(w, B, hp):
    if w is None:
        assert hp.nbasis == 1
        return np.ones((B, 1))
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (B, hp.nbasis)
    return w


def forward(P, pb, hp, keep=False, w=None):
    cache = {}
    a = inputs(pb, hp)
    v = _pw(a, P["W0"], P["b0"])
    cache["a"] = a
    for l in range(hp.layers):
        cache[f"v{l}"] = v
        Xh = spectral_forward(v, hp)
        cache[f"X{l}"] = Xh
        Yh = np.einsum("bcq,qco->boq", Xh, P[f"R{l + 1}"])
        z = spectral_inverse(Yh, hp) + _pw(v, P[f"W{l + 1}"], P[f"b{l + 1}"])
        cache[f"z{l}"] = z
        v = gelu(z) if l < hp.layers - 1 else z
    cache["vL"] = v
    hpre = _pw(v, P["P1"], P["c1"])
    cache["hpre"] = hpre
    h = gelu(hpre)
    cache["h"] = h
    o = _pw(h, P["P2"], P["c2"])
    w = _weights(w, o.shape[0], hp)
    out = np.einsum("bk,bkc...->bc...", w, o.reshape((o.shape[0], hp.nbasis, hp.nout) + o.shape[2:]))
    cache["w"] = w
    return (out, cache) if keep else out


def loss(out, y):
    B = out.shape[0]
    d = (out - y).reshape(B, -1)
    return float(np.mean(np.linalg.norm(d, axis=1) / np.linalg.norm(y.reshape(B, -1), axis=1)))


def loss_and_grad(P, pb, y, hp, w=None):
    out, c = forward(P, pb, hp, keep=True, w=w)
    B = out.shape[0]
    d = (out - y).reshape(B, -1)
    nd = np.linalg.norm(d, axis=1)
    ny = np.linalg.norm(y.reshape(B, -1), axis=1)
    L = float(np.mean(nd / ny))
    g_out = (d / (B * nd[:, None] * ny[:, None])).reshape(out.shape)
    # the head's weights spread dL/dout over the K basis channel groups
    g_out = np.einsum("bk,bc...->bkc...", c["w"], g_out).reshape((B, hp.nbasis * hp.nout) + out.shape[2:])
    G = {}
    G["P2"] = _outer(c["h"], g_out)
    G["c2"] = g_out.sum(axis=(0, 2, 3, 4))
    g_h = np.einsum("bo...,io->bi...", g_out, P["P2"])
    g_hpre = g_h * gelu_grad(c["hpre"])
    G["P1"] = _outer(c["vL"], g_hpre)
    G["c1"] = g_hpre.sum(axis=(0, 2, 3, 4))
    g_v = np.einsum("bo...,io->bi...", g_hpre, P["P1"])
    N3 = float(hp.period) ** 3
    m = _mult(hp)
    for l in reversed(range(hp.layers)):
        z = c[f"z{l}"]
        g_z = g_v * gelu_grad(z) if l < hp.layers - 1 else g_v
        v = c[f"v{l}"]
        G[f"W{l + 1}"] = _outer(v, g_z)
        G[f"b{l + 1}"] = g_z.sum(axis=(0, 2, 3, 4))
        g_v = np.einsum("bo...,io->bi...", g_z, P[f"W{l + 1}"])
        # u = irfftn(Yh): dL/dYh = (m / P^3) rfftn(g_u) on the kept modes
        g_Y = spectral_forward(g_z, hp) * (m / N3)
        Xh = c[f"X{l}"]
        G[f"R{l + 1}"] = np.einsum("bcq,boq->qco", np.conj(Xh), g_Y)
        g_X = np.einsum("boq,qco->bcq", g_Y, np.conj(P[f"R{l + 1}"]))
        # Xh = rfftn(v)[modes]: dL/dv = Re sum g_X e^{+ik.x} = P^3 irfftn(g_X / m)
        g_v = g_v + spectral_inverse(g_X / m, hp) * N3
    G["W0"] = _outer(c["a"], g_v)
    G["b0"] = g_v.sum(axis=(0, 2, 3, 4))
    return L, G


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Algorithm 1 of Kingma and Ba) on flat
    float64 arrays; t counts steps from 1.  Returns (p, m, v) as new arrays."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
