"""Pins of the FP64 U-Net oracle of the learned Poisson part: the layer
convention against explicit loops, gradients against finite differences,
positive homogeneity of the bias-free ReLU network, and the training-sample
definition against the direct Poisson solve."""
import numpy as np
import pytest

from conftest import make_oracle
from oracle import unet_oracle as U
from paper_2109_00214_amd import workload as W


def test_layer_count_and_size():
    shapes = U.layer_shapes(4, 16, 2)
    assert len(shapes) == 15
    # 9 (2*16 + 16*16 + 16*32 + 32*32 + 32*64 + 64*64 + 64*128 + 128*128
    #    + 192*64 + 64*64 + 96*32 + 32*32 + 48*16 + 16*16) + 16
    assert U.n_params(4, 16, 2) == 486448
    assert U.padded_size(256, 512, 4) == (520, 264)


def test_conv_tap_convention_by_loops():
    """One 3x3 layer written as loops over the documented tap order equals
    the oracle's first layer (a 1-level network without ReLU effects: all
    inputs and weights positive)."""
    rng = np.random.default_rng(0)
    H = Wd = 6
    x = rng.random((1, 2, H, Wd))
    w = np.zeros(U.n_params(1, 4, 2))
    shapes = U.layer_shapes(1, 4, 2)
    w[:4 * 9 * 2] = rng.random(4 * 9 * 2)           # layer 0: [co][tap][ci]
    n1 = 4 * 9 * 4
    w[4 * 9 * 2:4 * 9 * 2 + n1] = 0.0
    for co in range(4):                               # layer 1: identity at the centre tap
        w[4 * 9 * 2 + co * 36 + 4 * 4 + co] = 1.0
    w[-4:] = 1.0                                       # 1x1: sum of the channels
    assert shapes[-1] == (1, 4, 1)
    out = U.forward(x, w, levels=1, base=4)[0, 0]
    W0 = w[:72].reshape(4, 9, 2)
    ref = np.zeros((H, Wd))
    for co in range(4):
        for y in range(H):
            for xx in range(Wd):
                s = 0.0
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        yy, xq = y + dy, xx + dx
                        if 0 <= yy < H and 0 <= xq < Wd:
                            s += np.dot(W0[co, 3 * (dy + 1) + (dx + 1)], x[0, :, yy, xq])
                ref[y, xx] += max(s, 0.0)
    np.testing.assert_allclose(out, ref, rtol=1e-12)


def test_gradients_against_finite_differences():
    rng = np.random.default_rng(1)
    levels, base = 2, 4
    x = rng.normal(size=(1, 2, 8, 8))
    w = rng.normal(size=U.n_params(levels, base, 2)) * 0.5
    dout = rng.normal(size=(1, 1, 8, 8))
    gw, gx = U.weight_gradient(x, w, dout, levels, base)
    f = lambda ww: float(np.sum(dout * U.forward(x, ww, levels, base)))  # noqa: E731
    for k in rng.choice(len(w), 25, replace=False):
        e = np.zeros_like(w)
        e[k] = 1e-6
        fd = (f(w + e) - f(w - e)) / 2e-6
        assert gw[k] == pytest.approx(fd, rel=1e-5, abs=1e-8)
    fx = lambda xx: float(np.sum(dout * U.forward(xx, w, levels, base)))  # noqa: E731
    for _ in range(10):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        e = np.zeros_like(x)
        e[idx] = 1e-6
        fd = (fx(x + e) - fx(x - e)) / 2e-6
        assert gx[idx] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_positive_homogeneity():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 2, 16, 16))
    w = rng.normal(size=U.n_params(4, 4, 2))
    a = U.forward(x, w, 4, 4)
    b = U.forward(3.5 * x, w, 4, 4)
    np.testing.assert_allclose(b, 3.5 * a, rtol=1e-10, atol=0)


def test_sample_target_is_the_solution_of_the_input():
    """Channel 0 is b of the volume-weighted system and the target its
    solution: applying the operator (from the oracle's residual, which is
    pinned separately) to the scaled target reproduces channel 0."""
    cfg = W.config("tiny", nr=16, nz=32)
    o = make_oracle(cfg, collisions_off=True)
    rng = np.random.default_rng(4)
    Q = rng.integers(0, 2 ** 44, size=(cfg.nz + 1, cfg.nr + 1))
    o.set_charge(Q)
    o.stage("poisson")
    phi = o.field()["phi"]
    j = np.arange(cfg.nz + 1)
    vac = np.repeat(((-cfg.V) + cfg.V * (j / cfg.nz))[:, None], cfg.nr + 1, axis=1)
    x, y = U.sample(o, Q, phi - vac)
    # the charge part alone, with zero electrodes, has (almost) no residual
    o2 = make_oracle(W.config("tiny", nr=16, nz=32, V=0.0), collisions_off=True)
    rn, bn = o2.poisson_residual(Q, phi - vac)
    assert rn <= 1e-10 * bn
    assert x.shape == (2, 40, 24) and y.shape == (40, 24)
    assert np.sqrt(np.mean(x[0, 1:cfg.nz, :cfg.nr + 1] ** 2)) == pytest.approx(1.0)
    assert np.sqrt(np.mean(y[1:cfg.nz, :cfg.nr + 1] ** 2)) == pytest.approx(1.0)
    assert np.all(x[:, cfg.nz + 1:] == 0) and np.all(y[cfg.nz:] == 0)


def test_bf16_rounding_helper():
    """nearest-even BF16: exact values stay, halfway cases go to even, and
    the error is at most half a BF16 ulp (2^-8 relative)"""
    import torch
    # BF16 keeps 8 significant bits: the ulp at 1 is 2^-7
    v = torch.tensor([1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 3 * 2 ** -9, -3.5, 0.0],
                     dtype=torch.float64)
    r = U.bf16_round(v).numpy()
    # halfway cases 1 + 2^-8 (-> 1) and 1 + 3 2^-8 (-> 1 + 2^-6) go to the even neighbour
    assert list(r) == [1.0 + 2 ** -7, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -3.5, 0.0]
    rng = np.random.default_rng(9)
    x = torch.as_tensor(rng.normal(size=1000) * 1e3)
    e = np.abs(U.bf16_round(x).numpy() - x.numpy()) / np.abs(x.numpy())
    assert e.max() <= 2 ** -8 + 1e-12
    # the rounded forward is the plain forward up to that rounding, and the
    # straight-through gradient is finite and close to the plain one
    xx = rng.normal(size=(1, 2, 8, 8))
    w = rng.normal(size=U.n_params(2, 4, 2)) * 0.5
    a = U.forward(xx, w, 2, 4)
    b = U.forward(xx, w, 2, 4, rounding="bf16")
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 2e-2
