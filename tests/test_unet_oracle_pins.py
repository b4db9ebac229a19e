"""Pins of the U-Net oracle against facts other than itself: a library correlation, adjoint
identities, a library bfloat16 cast, finite differences and Adam's closed form."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet_oracle as U


def rand(rng, *shape):
    return rng.standard_normal(shape)


def test_conv3x3_is_a_library_correlation_per_channel_pair():
    rng = np.random.default_rng(0)
    x, w, b = rand(rng, 2, 7, 5, 3), rand(rng, 3, 3, 3, 4), rand(rng, 4)
    out = U.conv3x3(x, w, b)
    for n in range(2):
        for co in range(4):
            ref = sum(correlate2d(x[n, :, :, ci], w[:, :, ci, co], mode="same", boundary="fill")
                      for ci in range(3)) + b[co]
            np.testing.assert_allclose(out[n, :, :, co], ref, rtol=1e-13, atol=1e-13)


def test_conv3x3_gradients_are_adjoints():
    rng = np.random.default_rng(1)
    x, w, y = rand(rng, 2, 6, 8, 5), rand(rng, 3, 3, 5, 7), rand(rng, 2, 6, 8, 7)
    lhs = np.sum(U.conv3x3(x, w) * y)
    assert abs(lhs - np.sum(x * U.conv3x3_input_grad(y, w))) <= 1e-12 * abs(lhs)
    assert abs(lhs - np.sum(w * U.conv3x3_weight_grad(x, y))) <= 1e-12 * abs(lhs)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(2)
    x, y = rand(rng, 2, 8, 6, 3), rand(rng, 2, 4, 3, 3)
    assert np.isclose(np.sum(U.avg_pool2(x) * y), np.sum(x * U.avg_pool2_grad(y)), rtol=1e-13)
    assert np.isclose(np.sum(U.upsample2(y) * x), np.sum(y * U.upsample2_grad(x)), rtol=1e-13)
    np.testing.assert_allclose(U.avg_pool2(np.ones((1, 4, 4, 1))), np.ones((1, 2, 2, 1)))


def test_bf16_rounding_matches_a_library_cast():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-8, 8, 4000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 65504.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(U.bf16(x), ref)
    assert U.bf16(1.0 + 2 ** -8) == 1.0            # tie to even


def _tiny_net(rng):
    p = U.init_params(rng)
    for k in p:                                     # non-zero biases exercise every path
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    x = np.zeros((2, 16, 16, U.IN_CH))
    x[..., :U.N_INPUTS] = rng.standard_normal((2, 16, 16, U.N_INPUTS))
    return p, x, rng.standard_normal((2, 16, 16))


def test_backward_matches_finite_differences(monkeypatch):
    """With the bf16 rounding switched off the network is smooth almost everywhere: the
    directional derivative of the loss equals <grad, direction>."""
    monkeypatch.setattr(U, "bf16", lambda v: np.asarray(v, dtype=np.float64))
    rng = np.random.default_rng(4)
    p, x, target = _tiny_net(rng)
    out, acts = U.forward(p, x)
    loss, dout = U.mse_loss(out, target)
    g = U.backward(p, acts, dout)
    d = {k: rng.standard_normal(v.shape) for k, v in p.items()}
    d["e0a.w"][:, :, U.N_INPUTS:, :] = 0.0
    h = 1e-7
    lp = U.mse_loss(U.forward({k: p[k] + h * d[k] for k in p}, x)[0], target)[0]
    lm = U.mse_loss(U.forward({k: p[k] - h * d[k] for k in p}, x)[0], target)[0]
    fd = (lp - lm) / (2 * h)
    an = sum(np.sum(g[k] * d[k]) for k in p)
    assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)


def test_backward_of_each_parameter_group(monkeypatch):
    """Per parameter group (so that a wrong index in one layer cannot hide behind the sum)."""
    monkeypatch.setattr(U, "bf16", lambda v: np.asarray(v, dtype=np.float64))
    rng = np.random.default_rng(5)
    p, x, target = _tiny_net(rng)
    out, acts = U.forward(p, x)
    _, dout = U.mse_loss(out, target)
    g = U.backward(p, acts, dout)
    h = 1e-7
    for k in ["e0a.w", "e1b.w", "e3a.b", "d2a.w", "d1a.b", "d0b.w", "head.w", "head.b"]:
        d = rng.standard_normal(p[k].shape)
        if k == "e0a.w":
            d[:, :, U.N_INPUTS:, :] = 0.0
        q = dict(p)
        q[k] = p[k] + h * d
        lp = U.mse_loss(U.forward(q, x)[0], target)[0]
        q[k] = p[k] - h * d
        lm = U.mse_loss(U.forward(q, x)[0], target)[0]
        fd, an = (lp - lm) / (2 * h), np.sum(g[k] * d)
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-12), (k, fd, an)


def test_adam_constant_gradient_closed_form():
    """For a constant gradient g, m_hat = g and v_hat = g^2 at every step, so each step moves
    the weight by lr g / (|g| + eps)."""
    w0 = {"a.w": np.array([1.0, -2.0, 0.5]), "a.b": np.array([0.3])}
    g = {"a.w": np.array([0.2, -3.0, 1e-3]), "a.b": np.array([-0.7])}
    opt = U.Adam(w0, lr=1e-2)
    for _ in range(5):
        opt.step(g)
    for k in w0:
        np.testing.assert_allclose(opt.master[k], w0[k] - 5 * 1e-2 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12)
