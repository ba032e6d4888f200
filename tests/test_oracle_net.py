"""Pins for the FP64 reference of the warm-start network (CPU only): its convolution against
torch's conv2d (a library routine) in float64, its backward and loss gradients against finite
differences, and positive homogeneity of the bias-free LeakyReLU net."""
import numpy as np
import pytest

from oracle import net_ref


def rand_weights(seed, scale=0.2):
    return np.random.default_rng(seed).standard_normal(net_ref.N_PARAMS) * scale


def test_param_count():
    assert net_ref.N_PARAMS == 38592


def test_conv_matches_torch_conv2d():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    a = rng.standard_normal((5, 9, 11))
    W = rng.standard_normal((7, 5, 3, 3))
    want = torch.nn.functional.conv2d(torch.from_numpy(a)[None], torch.from_numpy(W), padding=1)[0].numpy()
    assert np.allclose(net_ref.conv3x3(a, W), want, atol=1e-12)


def test_forward_is_positively_homogeneous_and_scale_free():
    w = rand_weights(1)
    x = np.random.default_rng(2).standard_normal((3, 8, 10))
    o1, _, _ = net_ref.forward(w, x)
    o2, _, _ = net_ref.forward(w, 37.0 * x)
    assert np.allclose(o1, o2, rtol=1e-12, atol=1e-14)   # input normalisation removes the scale


def test_backward_matches_finite_differences():
    w = rand_weights(3)
    x = np.random.default_rng(4).standard_normal((3, 6, 7))
    dout = np.random.default_rng(5).standard_normal((3, 6, 7))
    g = net_ref.backward(w, x, dout)
    f = lambda ww: float((net_ref.forward(ww, x)[0] * dout).sum())
    rng = np.random.default_rng(6)
    h = 1e-6
    for k in rng.choice(w.size, 25, replace=False):
        e = np.zeros_like(w)
        e[k] = h
        fd = (f(w + e) - f(w - e)) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * max(1.0, abs(g).max())


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, 3, 20))
    x[0, :, 3] = 0.0                                            # a pinned CP is masked out
    p = rng.standard_normal((2, 3, 20))
    t = rng.standard_normal((2, 3, 20))
    L, d = net_ref.loss(x, p, t)
    assert 0.0 <= L <= 1.0
    assert np.all(d[0, :, 3] == 0.0)
    h = 1e-7
    for idx in [(0, 1, 5), (1, 2, 17), (0, 0, 0)]:
        e = np.zeros_like(p)
        e[idx] = h
        fd = (net_ref.loss(x, p + e, t)[0] - net_ref.loss(x, p - e, t)[0]) / (2 * h)
        assert abs(fd - d[idx]) < 1e-7
    # a perfect prediction up to scale has zero loss
    assert net_ref.loss(x, 3.0 * t, t)[0] < 1e-14
