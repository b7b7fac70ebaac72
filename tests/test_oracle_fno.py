"""Pins of the float64 FNO oracle (parity unpinned by the paper): central
finite differences of every parameter group, exact reproduction of
band-limited fields by the spectral convolution, and translation
equivariance of the spectral branch."""
import numpy as np
import pytest

from oracle import fno


def tiny(nbasis=1):
    return fno.HP(n=8, width=4, modes=2, nparam=8, hidden=6, nout=6, layers=3, nbasis=nbasis)


@pytest.mark.parametrize("nbasis", [1, 4])
def test_gradients_match_central_differences(nbasis):
    hp = tiny(nbasis)
    P = fno.init_params(1, hp)
    for k in list(P):
        if k.startswith("b") or k.startswith("c"):
            P[k] = np.random.default_rng(len(k)).normal(0, 0.1, P[k].shape)
    rng = np.random.default_rng(2)
    pb = rng.uniform(size=(2, 8))
    y = rng.normal(size=(2, 6, 8, 8, 8))
    w = rng.normal(size=(2, nbasis)) if nbasis > 1 else None
    L, G = fno.loss_and_grad(P, pb, y, hp, w=w)
    h = 1e-6
    for k, v in P.items():
        flat = v.reshape(-1)
        g = G[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            for part in ((1.0,) if not np.iscomplexobj(v) else (1.0, 1j)):
                orig = flat[idx]
                flat[idx] = orig + h * part
                Lp = fno.loss(fno.forward(P, pb, hp, w=w), y)
                flat[idx] = orig - h * part
                Lm = fno.loss(fno.forward(P, pb, hp, w=w), y)
                flat[idx] = orig
                fd = (Lp - Lm) / (2 * h)
                an = g[idx].real if part == 1.0 else g[idx].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, part, fd, an)


def test_spectral_branch_reproduces_band_limited_fields():
    hp = fno.HP(n=16, width=2, modes=4)
    rng = np.random.default_rng(3)
    kz, ky, kx = fno.kept_index(hp)
    coef = rng.normal(size=(1, 2, hp.nmodes)) + 1j * rng.normal(size=(1, 2, hp.nmodes))
    # band-limited real field on modes whose Hermitian partners are kept too
    edge = hp.n - hp.modes
    coef[:, :, (kx == 0) | (ky == edge) | (kz == edge)] = 0.0
    v = fno.spectral_inverse(coef, hp)
    Xh = fno.spectral_forward(v, hp)
    u = fno.spectral_inverse(Xh, hp)                           # identity mixing
    assert np.abs(u - v).max() < 1e-12 * np.abs(v).max()
    x = np.arange(16)
    hi = np.cos(2 * np.pi * 7 * x / 16)[None, None, None, None, :] * np.ones((1, 1, 16, 16, 16))
    assert np.abs(fno.spectral_inverse(fno.spectral_forward(hi, hp), hp)).max() < 1e-12


def test_spectral_branch_is_translation_equivariant():
    hp = fno.HP(n=16, width=3, modes=3)
    P = fno.init_params(4, hp)
    v = np.random.default_rng(5).normal(size=(1, 3, 16, 16, 16))
    f = lambda w: fno.spectral_inverse(np.einsum("bcq,qco->boq", fno.spectral_forward(w, hp), P["R1"]), hp)
    sh = lambda w: np.roll(w, (2, -3, 5), axis=(2, 3, 4))
    assert np.abs(f(sh(v)) - sh(f(v))).max() < 1e-12


def test_phasor_head_is_the_plain_head_when_the_weights_select_one_group():
    hp4 = tiny(4)
    P = fno.init_params(6, hp4)
    pb = np.random.default_rng(7).uniform(size=(1, 8))
    o = fno.forward(P, pb, hp4, w=np.array([[0.0, 0.0, 1.0, 0.0]]))
    P1 = dict(P, P2=P["P2"][:, 12:18], c2=P["c2"][12:18])
    assert np.array_equal(o, fno.forward(P1, pb, tiny(1)))
