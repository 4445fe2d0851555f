"""Pins of the surrogate oracle: convolution against an independent library
routine (PyTorch CPU conv2d in float64), every gradient against central finite
differences, pooling/upsampling against their adjoint identities, and Adam
against its first-step closed form."""
import numpy as np
import pytest

from oracle import surrogate as S


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_conv_matches_library_conv2d():
    torch = pytest.importorskip("torch")
    r = _rng(1)
    x = r.normal(size=(2, 5, 9, 7))
    w = r.normal(size=(3, 5, 3, 3))
    b = r.normal(size=3)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b),
                                     padding=1).numpy()
    assert np.max(np.abs(S.conv3x3(x, w, b) - ref)) < 1e-12


def test_conv_gradients_match_library_autograd():
    torch = pytest.importorskip("torch")
    r = _rng(2)
    x = r.normal(size=(2, 4, 6, 5))
    w = r.normal(size=(3, 4, 3, 3))
    b = r.normal(size=3)
    dy = r.normal(size=(2, 3, 6, 5))
    xt = torch.from_numpy(x).requires_grad_()
    wt = torch.from_numpy(w).requires_grad_()
    bt = torch.from_numpy(b).requires_grad_()
    (torch.nn.functional.conv2d(xt, wt, bt, padding=1) * torch.from_numpy(dy)).sum().backward()
    dw, db = S.conv3x3_grad_weight(x, dy)
    assert np.max(np.abs(S.conv3x3_grad_input(dy, w) - xt.grad.numpy())) < 1e-12
    assert np.max(np.abs(dw - wt.grad.numpy())) < 1e-11
    assert np.max(np.abs(db - bt.grad.numpy())) < 1e-12


def test_conv_gradients_finite_differences():
    r = _rng(3)
    x = r.normal(size=(1, 3, 5, 4))
    w = r.normal(size=(2, 3, 3, 3))
    b = r.normal(size=2)
    dy = r.normal(size=(1, 2, 5, 4))
    f = lambda x_, w_, b_: float((S.conv3x3(x_, w_, b_) * dy).sum())  # noqa: E731
    dx = S.conv3x3_grad_input(dy, w)
    dw, db = S.conv3x3_grad_weight(x, dy)
    h = 1e-6
    for idx in [(0, 1, 2, 3), (0, 0, 0, 0), (0, 2, 4, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((f(x + e, w, b) - f(x - e, w, b)) / (2 * h) - dx[idx]) < 1e-7
    for idx in [(1, 2, 0, 2), (0, 0, 1, 1)]:
        e = np.zeros_like(w)
        e[idx] = h
        assert abs((f(x, w + e, b) - f(x, w - e, b)) / (2 * h) - dw[idx]) < 1e-7


def test_pool_upsample_adjoints():
    r = _rng(4)
    x = r.normal(size=(2, 3, 8, 6))
    y = r.normal(size=(2, 3, 4, 3))
    assert abs((S.avgpool2(x) * y).sum() - (x * S.avgpool2_grad(y)).sum()) < 1e-12
    assert abs((S.upsample2(y) * x).sum() - (y * S.upsample2_grad(x)).sum()) < 1e-12
    assert np.allclose(S.avgpool2(np.ones((1, 1, 4, 4))), 1.0)


def test_network_gradient_finite_differences():
    """End-to-end backward pass of the encoder-decoder against central differences
    of the MSE loss, on a 16 x 16 input (levels 16, 8, 4, 2)."""
    r = _rng(5)
    params = S.init_params(7)
    # perturb biases so that no ReLU sits exactly at its kink
    params = {k: (w, r.normal(0, 0.05, b.shape)) for k, (w, b) in params.items()}
    x = np.zeros((1, S.IN_PADDED, 16, 16))
    x[:, :S.IN_CHANNELS] = r.normal(size=(1, S.IN_CHANNELS, 16, 16))
    t = r.normal(size=(1, 1, 16, 16))
    y, cache = S.forward(params, x)
    loss, dy = S.mse(y, t)
    grads = S.backward(params, cache, dy)
    h = 1e-6
    for name, idx in [("out", (0, 3, 1, 2)), ("d0b", (5, 7, 0, 0)), ("e3a", (2, 40, 1, 1)),
                      ("e0a", (4, 1, 2, 0)), ("d2a", (10, 130, 2, 2))]:
        w, b = params[name]
        e = np.zeros_like(w)
        e[idx] = h
        lp = S.mse(S.forward({**params, name: (w + e, b)}, x)[0], t)[0]
        lm = S.mse(S.forward({**params, name: (w - e, b)}, x)[0], t)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grads[name][0][idx]) < 1e-6 * max(1.0, abs(fd)), (name, fd, grads[name][0][idx])
    for name in ("out", "e1b"):
        w, b = params[name]
        e = np.zeros_like(b)
        e[0] = h
        lp = S.mse(S.forward({**params, name: (w, b + e)}, x)[0], t)[0]
        lm = S.mse(S.forward({**params, name: (w, b - e)}, x)[0], t)[0]
        assert abs((lp - lm) / (2 * h) - grads[name][1][0]) < 1e-6


def test_adam_first_step():
    """With zero moments, the bias-corrected first Adam step is -lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = S.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
