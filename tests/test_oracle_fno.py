"""Pins of the float64 FNO oracle (parity unpinned by the paper): central
finite differences of every parameter group, exact reproduction of
band-limited fields by the spectral convolution, and translation
equivariance of the spectral branch."""
import numpy as np
import pytest

from oracle import fno


def tiny(nbasis=1, period=None):
    return fno.HP(n=8, width=4, modes=2, nparam=8, hidden=6, nout=6, layers=3, nbasis=nbasis, period=period)


@pytest.mark.parametrize("nbasis, period", [(1, None), (4, None), (4, 11)])
def test_gradients_match_central_differences(nbasis, period):
    hp = tiny(nbasis, period)
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


def test_padded_transform_is_translation_equivariant_inside_the_window():
    """Period P > N: the spectral branch is a convolution on the P-periodic
    torus of the zero-extended input, cut to the window, so moving an input
    supported away from the window's far faces by s nodes moves the output
    by s at every window node that stays inside (x - s >= 0).  It is also
    the plain branch on a P^3 grid (pinned by the band-limited reproduction
    above) applied to the input extended by zeros at the far faces and cut
    back to the window's corner, which a wrong period, padding or cut would
    break."""
    hp = fno.HP(n=16, width=3, modes=3, period=22)
    P = fno.init_params(4, hp)
    v = np.zeros((1, 3, 16, 16, 16))
    v[:, :, :11, :12, :10] = np.random.default_rng(5).normal(size=(1, 3, 11, 12, 10))
    f = lambda w: fno.spectral_inverse(np.einsum("bcq,qco->boq", fno.spectral_forward(w, hp), P["R1"]), hp)
    s = (2, 3, 5)
    vs = np.zeros_like(v)
    vs[:, :, s[0]:, s[1]:, s[2]:] = v[:, :, :16 - s[0], :16 - s[1], :16 - s[2]]
    a, b = f(vs), f(v)
    assert np.abs(a[:, :, s[0]:, s[1]:, s[2]:] - b[:, :, :16 - s[0], :16 - s[1], :16 - s[2]]).max() < 1e-12 * np.abs(b).max()
    big = fno.HP(n=22, width=3, modes=3)
    ext = np.zeros((1, 3, 22, 22, 22))
    ext[:, :, :16, :16, :16] = v
    g = fno.spectral_inverse(np.einsum("bcq,qco->boq", fno.spectral_forward(ext, big), P["R1"]), big)
    assert np.abs(g[:, :, :16, :16, :16] - b).max() < 1e-12 * np.abs(b).max()


def test_padded_transform_of_period_n_is_the_plain_one():
    hp, hq = fno.HP(n=8, width=2, modes=2), fno.HP(n=8, width=2, modes=2, period=8)
    v = np.random.default_rng(6).normal(size=(1, 2, 8, 8, 8))
    assert np.array_equal(fno.spectral_forward(v, hp), fno.spectral_forward(v, hq))


def test_phasor_head_is_the_plain_head_when_the_weights_select_one_group():
    hp4 = tiny(4)
    P = fno.init_params(6, hp4)
    pb = np.random.default_rng(7).uniform(size=(1, 8))
    o = fno.forward(P, pb, hp4, w=np.array([[0.0, 0.0, 1.0, 0.0]]))
    P1 = dict(P, P2=P["P2"][:, 12:18], c2=P["c2"][12:18])
    assert np.array_equal(o, fno.forward(P1, pb, tiny(1)))


# ---- Adam (Kingma and Ba, Algorithm 1), pinned by hand-derived closed forms

def _grads(seed, n=257):
    g = np.random.default_rng(seed).normal(size=n) * np.logspace(-6, 3, n)
    g[::17] = 0.0
    return g


def test_adam_first_step_is_lr_times_sign_like_ratio():
    """t = 1: m_hat = g and v_hat = g^2 exactly, so p moves by lr g / (|g| + eps)."""
    g = _grads(1)
    p0 = np.random.default_rng(2).normal(size=g.size)
    lr = 3e-3
    p1, m, v = fno.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    assert np.allclose(p1 - p0, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    assert np.allclose(m, 0.1 * g, rtol=1e-15) and np.allclose(v, 0.001 * g * g, rtol=1e-12)
    assert np.array_equal(p1[g == 0.0], p0[g == 0.0])


def test_adam_constant_gradient_moves_by_the_same_step_every_time():
    """The bias corrections undo the zero start: with a constant gradient
    m_hat = g and v_hat = g^2 at every t (a wrong exponent or a missing
    correction breaks this from t = 2 on)."""
    g = _grads(3)
    p = np.zeros_like(g)
    m, v = np.zeros_like(g), np.zeros_like(g)
    lr = 1e-2
    step = -lr * g / (np.abs(g) + 1e-8)
    for t in range(1, 8):
        q, m, v = fno.adam_step(p, g, m, v, t, lr)
        assert np.allclose(q - p, step, rtol=1e-9, atol=1e-20), t
        p = q


def test_adam_alternating_gradient_second_step():
    """g then -g: m_2 = -(1 - b1)^2 g, so m_hat_2 = -(1 - b1) g / (1 + b1);
    v_2 = (1 - b2)(1 + b2) g^2, so v_hat_2 = g^2.  The second step moves p by
    +lr (1 - b1) / (1 + b1) g / (|g| + eps) (b1 and b2 swapped would give
    (1 - b2) / (1 + b2) instead)."""
    g = _grads(4)
    p0 = np.zeros_like(g)
    lr = 2e-3
    p1, m, v = fno.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    p2, m, v = fno.adam_step(p1, -g, m, v, 2, lr)
    expect = lr * (0.1 / 1.9) * g / (np.abs(g) + 1e-8)
    assert np.allclose(p2 - p1, expect, rtol=1e-9, atol=1e-20)
    assert np.allclose(m, -(0.1 ** 2) * g, rtol=1e-12, atol=1e-300)


def test_adam_is_invariant_to_gradient_scale_without_eps():
    """With eps = 0 the update depends on g only through m / sqrt(v), which
    scaling every gradient by c > 0 leaves unchanged."""
    rng = np.random.default_rng(5)
    gs = [rng.normal(size=64) for _ in range(5)]
    runs = []
    for c in (1.0, 1e3):
        p, m, v = np.zeros(64), np.zeros(64), np.zeros(64)
        for t, g in enumerate(gs, 1):
            p, m, v = fno.adam_step(p, c * g, m, v, t, 1e-2, eps=0.0)
        runs.append(p)
    assert np.allclose(runs[0], runs[1], rtol=1e-12, atol=1e-15)
