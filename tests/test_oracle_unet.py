"""Pins of the oracle's network layers (CPU only).

A single-channel stride-1 convolution equals scipy.ndimage.correlate with a
zero constant boundary; stride 2 samples the stride-1 result at even nodes;
the input and weight gradients satisfy the adjoint identities
<conv(x), dy> = <x, dgrad(dy)> = <w, wgrad(x, dy)>; trilinear up-sampling
reproduces trilinear fields and its adjoint satisfies <up(a), b> = <a, up^T(b)>.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from tests.conftest import node_coords


def grid(x, n):
    """[n^3] channel-last (x fastest) -> array indexed [k, j, i]."""
    return x.reshape(n, n, n)


def test_single_channel_conv_is_correlate():
    rng = np.random.default_rng(0)
    n = 9
    x = rng.standard_normal((n ** 3, 1))
    w = rng.standard_normal((1, 27, 1))
    y = O.conv3d_fwd(x, w)
    kern = w[0, :, 0].reshape(3, 3, 3)       # [dz][dy][dx]
    ref = ndimage.correlate(grid(x[:, 0], n), kern, mode="constant", cval=0.0)
    assert np.allclose(grid(y[:, 0], n), ref, rtol=1e-13, atol=1e-13)
    y2 = O.conv3d_fwd(x, w, stride=2)
    assert np.allclose(grid(y2[:, 0], 5), ref[::2, ::2, ::2], rtol=1e-13, atol=1e-13)


def test_multichannel_bias_relu_linearity():
    rng = np.random.default_rng(1)
    n, cin, cout = 7, 3, 4
    x = rng.standard_normal((n ** 3, cin))
    w = rng.standard_normal((cout, 27, cin))
    b = rng.standard_normal(cout)
    y = O.conv3d_fwd(x, w, b)
    ys = sum(O.conv3d_fwd(x[:, [c]], w[:, :, [c]]) for c in range(cin)) + b
    assert np.allclose(y, ys, rtol=1e-12, atol=1e-12)
    assert np.allclose(O.conv3d_fwd(x, w, b, relu=True), np.maximum(y, 0.0))


@pytest.mark.parametrize("stride", [1, 2])
def test_gradients_are_adjoints(stride):
    rng = np.random.default_rng(2 + stride)
    n, cin, cout = 9, 3, 2
    nout = (n - 1) // stride + 1
    x = rng.standard_normal((n ** 3, cin))
    w = rng.standard_normal((cout, 27, cin))
    dy = rng.standard_normal((nout ** 3, cout))
    y = O.conv3d_fwd(x, w, stride=stride)
    lhs = (y * dy).sum()
    assert lhs == pytest.approx((x * O.conv3d_dgrad(w, dy, n, stride)).sum(), rel=1e-12)
    assert lhs == pytest.approx((w * O.conv3d_wgrad(x, dy, cout, stride)).sum(), rel=1e-12)


def test_upsample_and_adjoint():
    nc = 5
    nf = 9
    Xc, Yc, Zc = node_coords(nc, 2.0)
    Xf, Yf, Zf = node_coords(nf, 2.0)
    tri = lambda X, Y, Z: 1 + X - Y + 0.5 * Z + X * Y * Z
    up = O.upsample(tri(Xc, Yc, Zc).reshape(-1, 1), nc)
    assert np.allclose(up[:, 0], tri(Xf, Yf, Zf).ravel(), atol=1e-13)
    rng = np.random.default_rng(4)
    a = rng.standard_normal((nc ** 3, 3))
    bf = rng.standard_normal((nf ** 3, 3))
    assert (O.upsample(a, nc) * bf).sum() == pytest.approx((a * O.upsample_adj(bf, nc)).sum(), rel=1e-12)
