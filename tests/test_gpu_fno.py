"""GPU parity of the surrogate (Fourier neural operator) against the float64
oracle, through the C ABI.

The oracle runs with the same weights, rounded to bf16 where the GPU feeds
them to MFMA (W_l, R_l, P1, P2), so the remaining differences are the GPU's
bf16 rounding of the activations that enter those contractions and fp32
accumulation.  The truncated transforms alone use split-bf16 products and
must match to about fp32 accuracy."""
import math

import numpy as np
import pytest
import torch

from oracle import fno
from paper_2010_00409_amd import tfocus as tf

pytestmark = pytest.mark.gpu

HP = fno.HP()
SPECTRAL_TOL = 2e-5       # split-bf16 products (about 16 mantissa bits) with fp32 accumulation
# bf16 operands carry a relative rounding error of at most 2^-9; about ten
# rounded operand sets lie on the path from the parameters to the output
# (mixing input, pointwise input and weights per layer, projection input,
# hidden layer and the two projection weights), mostly averaging out in the
# contractions: the forward output stays within 5e-3 in relative L2.
FORWARD_TOL = 5e-3
# Gradients: the backward pass's own rounding (weight-gradient GEMMs in split
# bf16, about float32; one bf16 copy of the stored hidden layer and of the
# data-gradient operands) stays within 1e-2 (relative L2) for residuals with
# a structured part and for white residuals four times the output.  The loss
# gradient is J^T applied to the residual out - y (J the network's Jacobian),
# and the GPU's residual also carries the forward's bf16 error (gated above):
# that error lies in the range of J, white noise mostly does not, so when a
# white residual dominates, J^T amplifies the forward error's share.  At white
# residuals of 0.5 (output about 1e-2 of that) the four-basis head measures
# 1.2e-2; that case is held to 1.5e-2.
GRAD_TOL = 1e-2
GRAD_TOL_WHITE = 1.5e-2
GRAD_COS = 0.999


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def bf16_round(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def make_params(seed, r_scale=16.0, hp=HP):
    """Oracle initialisation with the spectral weights scaled up so the
    Fourier branch carries a sizeable part of every layer, and non-zero
    biases; MFMA weights rounded to bf16."""
    P = fno.init_params(seed, hp)
    rng = np.random.default_rng(seed + 1)
    for l in range(1, HP.layers + 1):
        P[f"R{l}"] = P[f"R{l}"] * r_scale
        P[f"b{l}"] = rng.normal(0, 0.1, HP.width)
    P["b0"] = rng.normal(0, 0.1, HP.width)
    P["c1"] = rng.normal(0, 0.1, HP.hidden)
    P["c2"] = rng.normal(0, 0.1, hp.nout * hp.nbasis)
    for k in list(P):
        if k.startswith(("W", "P")) and k != "W0":
            P[k] = bf16_round(P[k])
        elif k.startswith("R"):
            P[k] = bf16_round(P[k].real) + 1j * bf16_round(P[k].imag)
        else:
            P[k] = np.asarray(P[k], dtype=np.float32).astype(np.float64)
    return P


def modes_to_oracle(m):
    """[B][kz][s][ky][kx][c] float -> (B, C, nmodes) complex, q = (kz*24 + ky)*12 + kx."""
    z = m[:, :, 0] + 1j * m[:, :, 1]                  # (B, kz, ky, kx, c)
    return z.reshape(m.shape[0], -1, HP.width).transpose(0, 2, 1)


def modes_from_oracle(Xh):
    B = Xh.shape[0]
    z = Xh.transpose(0, 2, 1).reshape(B, 24, 24, 12, HP.width)
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=2), dtype=np.float32)


@pytest.mark.parametrize("period", [64, 80, 96])
def test_truncated_transforms_match_oracle(period):
    """The truncated DFTs of the spectral branch, plain (period 64) and on
    the window extended by zeros to a longer period, against the oracle's
    rfftn / irfftn."""
    hp = fno.HP(period=period)
    rng = np.random.default_rng(11)
    B = 2
    v = rng.standard_normal((B, 64, 64, 64, HP.width)).astype(np.float32)
    with tf.Surrogate(B, period=period) as s:
        assert s.period == period
        vd = torch.from_numpy(v).cuda()
        md = torch.zeros((B, 24, 2, 24, 12, HP.width), dtype=torch.float32, device="cuda")
        s.spectral_forward(vd, md)
        got = modes_to_oracle(md.cpu().numpy().astype(np.float64))
        ref = fno.spectral_forward(v.astype(np.float64).transpose(0, 4, 1, 2, 3), hp)
        assert rel(got, ref) <= SPECTRAL_TOL
        Xh = (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)) * 100.0
        mi = torch.from_numpy(modes_from_oracle(Xh)).cuda()
        ud = torch.zeros((B, 64, 64, 64, HP.width), dtype=torch.float32, device="cuda")
        s.spectral_inverse(mi, ud)
        got_u = ud.cpu().numpy().astype(np.float64).transpose(0, 4, 1, 2, 3)
        ref_u = fno.spectral_inverse(modes_to_oracle(mi.cpu().numpy().astype(np.float64)), hp)
        assert rel(got_u, ref_u) <= SPECTRAL_TOL


def run_forward(P, pb, w=None, period=64):
    B = pb.shape[0]
    nb = 1 if w is None else w.shape[1]
    with tf.Surrogate(B, nbasis=nb, period=period) as s:
        s.set_params(P)
        pd = torch.from_numpy(pb.astype(np.float32)).cuda()
        wd = None if w is None else torch.from_numpy(w.astype(np.float32)).cuda()
        out = torch.zeros((B, 6, 64, 64, 64), dtype=torch.float32, device="cuda")
        s.forward(pd, out, wd)
        return out.cpu().numpy().astype(np.float64)


def test_forward_matches_oracle():
    P = make_params(3)
    pb = np.random.default_rng(4).uniform(size=(2, 8)).astype(np.float32).astype(np.float64)
    got = run_forward(P, pb)
    ref = fno.forward(P, pb, HP)
    for b in range(2):
        assert rel(got[b], ref[b]) <= FORWARD_TOL, b
    # the Fourier branch matters: zeroing it changes the output by far more than the tolerance
    P0 = dict(P)
    for l in range(1, HP.layers + 1):
        P0[f"R{l}"] = np.zeros_like(P[f"R{l}"])
    assert rel(fno.forward(P0, pb, HP), ref) > 10 * FORWARD_TOL


# The fused inference kernels feed the next contraction from registers in a
# relabelled k order and compute the last layer transposed, so the fp32 sums
# differ from the training path in order only; single bf16 rounding flips
# (2^-9 relative) downstream keep the difference far below the oracle tolerance.
INFER_VS_TRAIN_TOL = 1e-3


def test_fused_inference_forward_matches_training_forward():
    P = make_params(5)
    pb = np.random.default_rng(6).uniform(size=(2, 8))
    a = run_forward(P, pb)
    with tf.Surrogate(2, training=True) as s:
        s.set_params(P)
        pd = torch.from_numpy(pb.astype(np.float32)).cuda()
        out = torch.zeros((2, 6, 64, 64, 64), dtype=torch.float32, device="cuda")
        s.forward(pd, out)
    b = out.cpu().numpy().astype(np.float64)
    for k in range(2):
        assert rel(a[k], b[k]) <= INFER_VS_TRAIN_TOL, k


def head_weights(rng, B, nb):
    """Phasor-head weights of random pulses, rounded to float32 (the GPU input)."""
    from synthetic import configs
    rows = configs.c5_params(B, seed=int(rng.integers(1 << 30)))
    w = np.array([tf.tf_fno_phasor_weights(configs.c5_pulse(r), nb) for r in rows])
    return w.astype(np.float32).astype(np.float64)


def test_padded_transform_forward_gradients_and_checkpoint_match_oracle(tmp_path):
    """Period 80 (the window extended by zeros by 16 nodes per axis) with
    the four-basis head: forward and every parameter group's gradient
    against the oracle at the same gates as the plain transform, and a
    checkpoint that carries the period into a fresh surrogate."""
    hp = fno.HP(nbasis=4, period=80)
    P = make_params(41, hp=hp)
    rng = np.random.default_rng(42)
    pb = rng.uniform(size=(2, 8)).astype(np.float32).astype(np.float64)
    w = head_weights(rng, 2, 4)
    got = run_forward(P, pb, w, period=80)
    ref = fno.forward(P, pb, hp, w=w)
    for b in range(2):
        assert rel(got[b], ref[b]) <= FORWARD_TOL, b
    assert rel(got, fno.forward(P, pb, fno.HP(nbasis=4), w=w)) > 10 * FORWARD_TOL   # the period matters
    y = (fno.forward(make_params(43, hp=hp), pb, hp, w=w) + 0.1 * rng.standard_normal((2, 6, 64, 64, 64)))
    y = y.astype(np.float32)
    L_ref, G_ref = fno.loss_and_grad(P, pb, y.astype(np.float64), hp, w=w)
    wd = torch.from_numpy(w.astype(np.float32)).cuda()
    pd = torch.from_numpy(pb.astype(np.float32)).cuda()
    with tf.Surrogate(2, training=True, nbasis=4, period=80) as s:
        s.set_params(P)
        L, g = s.loss_grad(pd, torch.from_numpy(y).cuda(), wd)
        path = tmp_path / "padded.ckpt"
        s.save(path)
    assert L == pytest.approx(L_ref, rel=FORWARD_TOL)
    G = tf.fno_unflatten(g)
    for k, r in G_ref.items():
        e = rel(G[k], r)
        cos = float(np.real(np.vdot(G[k].ravel(), r.ravel())) / (np.linalg.norm(G[k]) * np.linalg.norm(r)))
        assert e <= GRAD_TOL and cos >= GRAD_COS, (k, e, cos)
    with tf.Surrogate(2, nbasis=4) as s2:
        s2.load_checkpoint(path)
        assert s2.period == 80
        out = torch.zeros((2, 6, 64, 64, 64), dtype=torch.float32, device="cuda")
        s2.forward(pd, out, wd)
    assert np.array_equal(out.cpu().numpy(), got.astype(np.float32))


def test_four_basis_head_forward_matches_oracle():
    hp4 = fno.HP(nbasis=4)
    P = make_params(21, hp=hp4)
    rng = np.random.default_rng(22)
    pb = rng.uniform(size=(2, 8)).astype(np.float32).astype(np.float64)
    w = head_weights(rng, 2, 4)
    got = run_forward(P, pb, w)
    ref = fno.forward(P, pb, hp4, w=w)
    for b in range(2):
        assert rel(got[b], ref[b]) <= FORWARD_TOL, b


@pytest.mark.parametrize("residual, gate", [("structured", GRAD_TOL), ("white2", GRAD_TOL),
                                             ("white0.5", GRAD_TOL_WHITE)])
@pytest.mark.parametrize("nbasis", [1, 4])
def test_gradient_matches_oracle(nbasis, residual, gate):
    """Residuals: another network's output plus 0.1 white noise
    (structured), or pure white noise of 2 or 0.5 around the output."""
    hp = fno.HP(nbasis=nbasis)
    P = make_params(7, hp=hp)
    rng = np.random.default_rng(8)
    pb = rng.uniform(size=(2, 8)).astype(np.float32).astype(np.float64)
    w = head_weights(rng, 2, nbasis) if nbasis > 1 else None
    noise = rng.standard_normal((2, 6, 64, 64, 64))
    if residual == "structured":
        y = fno.forward(make_params(17, hp=hp), pb, hp, w=w) + 0.1 * noise
    else:
        y = fno.forward(P, pb, hp, w=w) + {"white2": 2.0, "white0.5": 0.5}[residual] * noise
    y = y.astype(np.float32)
    L_ref, G_ref = fno.loss_and_grad(P, pb, y.astype(np.float64), hp, w=w)
    with tf.Surrogate(2, training=True, nbasis=nbasis) as s:
        s.set_params(P)
        wd = None if w is None else torch.from_numpy(w.astype(np.float32)).cuda()
        L, g = s.loss_grad(torch.from_numpy(pb.astype(np.float32)).cuda(), torch.from_numpy(y).cuda(), wd)
    G = tf.fno_unflatten(g)
    assert L == pytest.approx(L_ref, rel=FORWARD_TOL)
    errs = {}
    for k, ref in G_ref.items():
        got = G[k]
        e = rel(got, ref)
        cos = float(np.real(np.vdot(got.ravel(), ref.ravel())) / (np.linalg.norm(got) * np.linalg.norm(ref)))
        errs[k] = (e, cos)
    print(f"nbasis {nbasis} residual {residual}: worst {max(e for e, _ in errs.values()):.2e} (gate {gate:.1e})")
    for k, (e, cos) in errs.items():
        assert e <= gate and cos >= GRAD_COS, (k, e, cos, gate)


def test_adam_steps_reduce_the_loss_and_checkpoint_roundtrips(tmp_path):
    P = make_params(9, r_scale=1.0)
    rng = np.random.default_rng(10)
    pb = rng.uniform(size=(2, 8)).astype(np.float32)
    y = np.ascontiguousarray(fno.forward(make_params(12), pb.astype(np.float64), HP), dtype=np.float32)
    pd, yd = torch.from_numpy(pb).cuda(), torch.from_numpy(y).cuda()
    with tf.Surrogate(2, training=True) as s:
        s.set_params(P)
        losses = [s.train_step(pd, yd, 1e-3) for _ in range(12)]
        path = tmp_path / "fno.ckpt"
        s.save(path)
        flat = s.get_params()
        nxt = s.train_step(pd, yd, 1e-3)
        s.load_checkpoint(path)
        assert np.array_equal(s.get_params(), flat)
        assert s.train_step(pd, yd, 1e-3) == nxt            # Adam state restored too
    assert losses[-1] < 0.7 * losses[0], losses


def test_graph_inference_replays_equal_eager_forward():
    """tf_fno_infer captures the forward pass once and replays it; every
    replay (with eager work in between, and after new parameters) must equal
    the eager forward bit for bit."""
    pb = torch.from_numpy(np.random.default_rng(15).uniform(size=(3, 8)).astype(np.float32)).cuda()
    shape = (3, 6, 64, 64, 64)
    out = torch.empty(shape, dtype=torch.float32, device="cuda")
    with tf.Surrogate(4) as s:
        for seed in (13, 14):
            s.set_params(make_params(seed))
            ref = torch.zeros(shape, dtype=torch.float32, device="cuda")
            s.forward(pb, ref)
            torch.cuda.synchronize()
            for _ in range(3):
                out.fill_(float("nan"))
                s.forward(pb, out, graph=True)
                torch.cuda.synchronize()
                junk = torch.randn(1 << 20, device="cuda").sum()
                torch.cuda.synchronize()
                del junk
                assert torch.equal(out, ref)


def read_checkpoint(path, nparams):
    """Adam step, parameters and both moments of a training checkpoint (four
    int64: magic, version, parameter count, step; then float32 parameters,
    first and second moments)."""
    raw = open(path, "rb").read()
    hdr = np.frombuffer(raw[:32], np.int64)
    body = np.frombuffer(raw[32:], np.float32).astype(np.float64)
    assert hdr[2] == nparams and body.size == 3 * nparams
    return int(hdr[3]), body[:nparams], body[nparams:2 * nparams], body[2 * nparams:]


def test_adam_steps_match_oracle_adam(tmp_path):
    """Three tf_fno_train_step updates against the oracle's float64 Adam
    (Kingma and Ba, Algorithm 1) fed the same gradients: the GPU's own
    gradient at each step (tf_fno_loss_grad, deterministic, so train_step
    sees the same values).  Parameters after every step and both moments
    after the last, element by element."""
    P = make_params(9, r_scale=1.0)
    rng = np.random.default_rng(10)
    pb = rng.uniform(size=(2, 8)).astype(np.float32)
    y = np.ascontiguousarray(fno.forward(make_params(12), pb.astype(np.float64), HP), dtype=np.float32)
    pd, yd = torch.from_numpy(pb).cuda(), torch.from_numpy(y).cuda()
    lrs = (1e-3, 3e-3, 2e-3)
    with tf.Surrogate(2, training=True) as s:
        s.set_params(P)
        p = s.get_params().astype(np.float64)
        m, v = np.zeros_like(p), np.zeros_like(p)
        gmax = np.zeros_like(p)
        for t, lr in enumerate(lrs, 1):
            _, g = s.loss_grad(pd, yd)
            _, g2 = s.loss_grad(pd, yd)
            assert np.array_equal(g, g2)
            g = g.astype(np.float64)
            gmax = np.maximum(gmax, np.abs(g))
            s.train_step(pd, yd, lr, want_loss=False)
            p, m, v = fno.adam_step(p, g, m, v, t, lr)
            got = s.get_params().astype(np.float64)
            # float32 rounding of each update (relative 1e-6) and of the stored parameters
            tol = 4 * 2.0 ** -24 * np.abs(p) + 2e-6 * t * max(lrs)
            bad = np.abs(got - p) > tol
            assert not bad.any(), (t, int(bad.sum()), float(np.abs(got - p).max()))
        path = tmp_path / "adam.ckpt"
        s.save(path)
    step, pg, mg, vg = read_checkpoint(path, p.size)
    assert step == 3
    assert np.all(np.abs(mg - m) <= 1e-6 * gmax + 1e-38)
    assert np.all(np.abs(vg - v) <= 1e-6 * v + 1e-6 * 1e-3 * gmax ** 2 + 1e-38)
    assert np.abs(pg - p).max() <= np.abs(got - p).max()


def splitmix_perms(seed, n, epochs):
    """Per-epoch Fisher-Yates permutations drawn with splitmix64 (Steele, Lea
    and Flood, OOPSLA 2014), as the library's training loop documents."""
    M = (1 << 64) - 1
    st = seed

    def nxt():
        nonlocal st
        st = (st + 0x9E3779B97F4A7C15) & M
        z = st
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    out = []
    for _ in range(epochs):
        perm = list(range(n))
        for i in range(n - 1, 0, -1):
            j = nxt() % (i + 1)
            perm[i], perm[j] = perm[j], perm[i]
        out.append(perm)
    return out


def _train_data(n, nbasis, seed):
    rng = np.random.default_rng(seed)
    P = make_params(seed, r_scale=1.0, hp=fno.HP(nbasis=nbasis))
    pb = rng.uniform(size=(n, 8)).astype(np.float32)
    y = (0.3 * rng.standard_normal((n, 6, 64, 64, 64))).astype(np.float32)
    w = head_weights(rng, n, nbasis).astype(np.float32) if nbasis > 1 else None
    return P, pb, y, w


@pytest.mark.parametrize("nbasis", [1, 4])
def test_training_run_equals_train_steps_over_its_shuffle(nbasis):
    """tf_fno_train (shuffle, gather, cosine learning rate, Adam, loss log on
    the device) against tf_fno_train_step driven from the host over the same
    permutations and learning rates: the same parameters bit for bit and the
    same per-epoch mean losses."""
    n, B, E, lr, fmin, seed = 6, 2, 2, 1e-3, 0.1, 5
    P, pb, y, w = _train_data(n, nbasis, 31)
    pd, yd = torch.from_numpy(pb).cuda(), torch.from_numpy(y).cuda()
    wd = None if w is None else torch.from_numpy(w).cuda()
    with tf.Surrogate(B, training=True, nbasis=nbasis) as s:
        s.set_params(P)
        hist = s.train(pd, yd, E, B, lr, w=wd, lr_min_frac=fmin, seed=seed, scale_targets=False)
        got = s.get_params()
    spe, total = n // B, (n // B) * E
    with tf.Surrogate(B, training=True, nbasis=nbasis) as s:
        s.set_params(P)
        means = []
        for ep, perm in enumerate(splitmix_perms(seed, n, E)):
            acc = []
            for k in range(spe):
                idx = torch.tensor(perm[k * B:(k + 1) * B], device="cuda")
                step = ep * spe + k
                a = lr * (fmin + (1 - fmin) * 0.5 * (1 + math.cos(math.pi * step / total)))
                acc.append(s.train_step(pd[idx].contiguous(), yd[idx].contiguous(), a,
                                        None if wd is None else wd[idx].contiguous()))
            means.append(sum(acc) / len(acc))
        ref = s.get_params()
    assert np.array_equal(got, ref)
    assert np.allclose(hist, means, rtol=1e-12)


def test_training_run_folds_the_target_rms_into_the_projection():
    """With lr = 0 only the scaling acts: the parameters before P2 stay as
    set, and P2 and c2 come back multiplied by the root mean square of every
    target value."""
    n = 4
    P, pb, y, _ = _train_data(n, 1, 32)
    flat0 = tf.fno_flatten(P).astype(np.float32)
    with tf.Surrogate(2, training=True) as s:
        s.set_params(P)
        s.train(torch.from_numpy(pb).cuda(), torch.from_numpy(y).cuda(), 1, 2, 0.0, seed=1)
        got = s.get_params()
    rms = float(np.sqrt(np.mean(y.astype(np.float64) ** 2)))
    off = fno_p2_offset()
    assert np.array_equal(got[:off], flat0[:off])
    assert np.allclose(got[off:], flat0[off:].astype(np.float64) * rms, rtol=2e-7, atol=0)


def fno_p2_offset():
    off = 0
    for name, shape in tf.fno_param_shapes(1):
        if name == "P2":
            return off
        off += int(np.prod(shape)) * (2 if name.startswith("R") else 1)
    raise AssertionError("no P2")


def test_eval_gives_per_window_relative_errors_of_the_forward_pass():
    n = 5
    P, pb, y, _ = _train_data(n, 1, 33)
    pd, yd = torch.from_numpy(pb).cuda(), torch.from_numpy(y).cuda()
    with tf.Surrogate(2) as s:
        s.set_params(P)
        err = s.eval(pd, yd)
        out = torch.empty_like(yd)
        for i in range(0, n, 2):
            s.forward(pd[i:i + 2].contiguous(), out[i:i + 2])
        torch.cuda.synchronize()
    o = out.cpu().numpy().astype(np.float64).reshape(n, -1)
    t = y.astype(np.float64).reshape(n, -1)
    ref = np.linalg.norm(o - t, axis=1) / np.linalg.norm(t, axis=1)
    assert np.allclose(err, ref, rtol=1e-12)
