"""Pins of the FP64 convolution reference: closed forms and central
differences (the backward functions must be the derivatives of the forward)."""
import numpy as np
import pytest

from oracle import conv


def test_identity_kernel_is_identity():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 4, 5, 6, 3))
    w = np.zeros((3, 27, 3))
    w[:, 13, :] = np.eye(3)  # centre tap
    assert np.abs(conv.conv3d(x, w) - x).max() == 0.0
    w1 = np.eye(3)[:, None, :]
    assert np.abs(conv.conv3d(x, w1, k=1) - x).max() == 0.0


def test_delta_input_reproduces_the_kernel():
    # A unit impulse at the centre returns the kernel mirrored in space.
    x = np.zeros((1, 5, 5, 5, 1))
    x[0, 2, 2, 2, 0] = 1.0
    rng = np.random.default_rng(1)
    w = rng.standard_normal((1, 27, 1))
    y = conv.conv3d(x, w)
    for t, (kd, kh, kw) in enumerate(conv._taps(3)):
        assert y[0, 2 - kd + 1, 2 - kh + 1, 2 - kw + 1, 0] == w[0, t, 0]


def test_stride_two_samples_even_positions():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 6, 4, 8, 2))
    w = rng.standard_normal((3, 27, 2))
    full = conv.conv3d(x, w, s=1)
    assert np.abs(conv.conv3d(x, w, s=2) - full[:, ::2, ::2, ::2, :]).max() < 1e-13


def test_upsample_and_adjoint():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 2, 3, 2, 4))
    y = conv.upsample2(x)
    assert y.shape == (1, 4, 6, 4, 4) and y[0, 3, 5, 1, 2] == x[0, 1, 2, 0, 2]
    dy = rng.standard_normal(y.shape)
    # <up(x), dy> == <x, up^T(dy)>
    assert (y * dy).sum() == pytest.approx((x * conv.upsample2_bwd(dy)).sum(), rel=1e-13)


@pytest.mark.parametrize("k,s", [(3, 1), (3, 2), (1, 1)])
def test_backward_matches_central_differences(k, s):
    rng = np.random.default_rng(4 + k + s)
    x = rng.standard_normal((2, 4, 6, 4, 3))
    w = rng.standard_normal((5, k ** 3, 3))
    b = rng.standard_normal(5)
    r = rng.standard_normal(conv.conv3d(x, w, b, k, s).shape)

    def loss(x_, w_, b_):
        return (conv.conv3d(x_, w_, b_, k, s) * r).sum()

    dx = conv.conv3d_bwd_data(r, w, x.shape, k, s)
    dw, db = conv.conv3d_bwd_weight(x, r, k, s)
    h = 1e-6
    for _ in range(12):
        idx = tuple(rng.integers(0, n) for n in x.shape)
        e = np.zeros_like(x)
        e[idx] = h
        fd = (loss(x + e, w, b) - loss(x - e, w, b)) / (2 * h)
        assert dx[idx] == pytest.approx(fd, rel=1e-6, abs=1e-8)
        idw = tuple(rng.integers(0, n) for n in w.shape)
        e = np.zeros_like(w)
        e[idw] = h
        fd = (loss(x, w + e, b) - loss(x, w - e, b)) / (2 * h)
        assert dw[idw] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    e = np.zeros_like(b)
    e[2] = h
    assert db[2] == pytest.approx((loss(x, w, b + e) - loss(x, w, b - e)) / (2 * h), rel=1e-6)


def test_bf16_rounding_ties_to_even():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5], np.float32)
    r = conv.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0              # tie -> even (1.0)
    assert r[2] == 1.0 + 2 ** -6    # tie -> even (upper)
    assert r[3] == 1.0
    assert r[4] == -2.5
