"""FP64 reference of the convolutional surrogate (TEST INFRASTRUCTURE ONLY).

The surrogate is a small encoder-decoder that maps (solid mask, initial density,
T/Tc, wall chemical potential) to the equilibrium density field; it is not part
of the paper's method, so this file follows the textbook definitions:

  conv (3x3, stride 1, zero padding 1):
      y[n, o, i, j] = b[o] + sum_{c, u, v} w[o, c, u, v] x[n, c, i + u - 1, j + v - 1]
  its two gradients (data and weights) by the chain rule of that sum, ReLU,
  2x2 average pooling, 2x nearest-neighbour upsampling, channel concatenation,
  mean-squared error, and Adam (Kingma and Ba, 2015).

Layout NCHW, float64.  The network shape matches the GPU library's:
levels of 32, 64, 96, 128 channels, two 3x3 convolutions per level, average
pooling down, nearest upsampling and skip concatenation up, a final 3x3
convolution to one channel.  Every function is plain numpy; a matmul over the
channel axis (einsum contracted through BLAS) is the only library primitive used.
"""
from __future__ import annotations

import numpy as np

LEVELS = (32, 64, 96, 128)
IN_CHANNELS = 4      # mask, initial density, T/Tc, wall mu
IN_PADDED = 16       # the input is zero-padded to 16 channels


def conv3x3(x, w, b):
    """x [N,C,H,W], w [O,C,3,3], b [O] -> [N,O,H,W]."""
    N, C, H, W = x.shape
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((N, w.shape[0], H, W))
    for u in range(3):
        for v in range(3):
            patch = xp[:, :, u:u + H, v:v + W]                     # x[n, c, i+u-1, j+v-1]
            y += np.einsum("oc,nchw->nohw", w[:, :, u, v], patch, optimize=True)
    return y + b[None, :, None, None]


def conv3x3_grad_input(dy, w):
    """dx[n,c,i,j] = sum_{o,u,v} w[o,c,u,v] dy[n,o,i-u+1,j-v+1]."""
    N, O, H, W = dy.shape
    dyp = np.zeros((N, O, H + 2, W + 2))
    dyp[:, :, 1:-1, 1:-1] = dy
    dx = np.zeros((N, w.shape[1], H, W))
    for u in range(3):
        for v in range(3):
            patch = dyp[:, :, 2 - u:2 - u + H, 2 - v:2 - v + W]     # dy[n, o, i-u+1, j-v+1]
            dx += np.einsum("oc,nohw->nchw", w[:, :, u, v], patch, optimize=True)
    return dx


def conv3x3_grad_weight(x, dy):
    """dw[o,c,u,v] = sum_{n,i,j} dy[n,o,i,j] x[n,c,i+u-1,j+v-1]; db[o] = sum dy."""
    N, C, H, W = x.shape
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dw = np.zeros((dy.shape[1], C, 3, 3))
    for u in range(3):
        for v in range(3):
            dw[:, :, u, v] = np.einsum("nohw,nchw->oc", dy, xp[:, :, u:u + H, v:v + W], optimize=True)
    return dw, dy.sum(axis=(0, 2, 3))


def relu(x):
    return np.maximum(x, 0.0)


def avgpool2(x):
    N, C, H, W = x.shape
    return x.reshape(N, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def avgpool2_grad(dy):
    return np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def upsample2_grad(dy):
    N, C, H, W = dy.shape
    return dy.reshape(N, C, H // 2, 2, W // 2, 2).sum(axis=(3, 5))


def layer_shapes():
    """(name, in_channels, out_channels, relu) in evaluation order."""
    L = LEVELS
    s = [("e0a", IN_PADDED, L[0], True), ("e0b", L[0], L[0], True),
         ("e1a", L[0], L[1], True), ("e1b", L[1], L[1], True),
         ("e2a", L[1], L[2], True), ("e2b", L[2], L[2], True),
         ("e3a", L[2], L[3], True), ("e3b", L[3], L[3], True),
         ("d2a", L[3] + L[2], L[2], True), ("d2b", L[2], L[2], True),
         ("d1a", L[2] + L[1], L[1], True), ("d1b", L[1], L[1], True),
         ("d0a", L[1] + L[0], L[0], True), ("d0b", L[0], L[0], True),
         ("out", L[0], 1, False)]
    return s


def init_params(seed: int):
    """He-normal weights and zero biases (numpy generator; the GPU library takes its
    parameters from the caller, so this only needs to be reproducible)."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, ci, co, _ in layer_shapes():
        std = np.sqrt(2.0 / (9 * ci))
        params[name] = (rng.normal(0.0, std, (co, ci, 3, 3)), np.zeros(co))
    return params


def forward(params, x):
    """x [N,16,H,W] -> (prediction [N,1,H,W], cache of activations)."""
    cache = {"x": x}
    shapes = {n: r for n, _, _, r in layer_shapes()}

    def layer(name, inp):
        w, b = params[name]
        z = conv3x3(inp, w, b)
        a = relu(z) if shapes[name] else z
        cache[name] = (inp, a)
        return a

    e0 = layer("e0b", layer("e0a", x))
    e1 = layer("e1b", layer("e1a", avgpool2(e0)))
    e2 = layer("e2b", layer("e2a", avgpool2(e1)))
    e3 = layer("e3b", layer("e3a", avgpool2(e2)))
    d2 = layer("d2b", layer("d2a", np.concatenate([upsample2(e3), e2], axis=1)))
    d1 = layer("d1b", layer("d1a", np.concatenate([upsample2(d2), e1], axis=1)))
    d0 = layer("d0b", layer("d0a", np.concatenate([upsample2(d1), e0], axis=1)))
    y = layer("out", d0)
    return y, cache


def mse(y, t):
    """Mean squared error over all elements and its gradient."""
    d = y - t
    return float((d * d).mean()), 2.0 * d / d.size


def backward(params, cache, dy, dzs=None):
    """Gradients {name: (dw, db)} of the loss whose gradient wrt the prediction is dy.
    If dzs is a dict, it receives each layer's output gradient dz (after its ReLU)."""
    shapes = {n: r for n, _, _, r in layer_shapes()}
    grads = {}

    def back(name, da):
        inp, a = cache[name]
        dz = da * (a > 0) if shapes[name] else da
        if dzs is not None:
            dzs[name] = dz
        grads[name] = conv3x3_grad_weight(inp, dz)
        return conv3x3_grad_input(dz, params[name][0])

    L = LEVELS
    dd0 = back("out", dy)
    dcat0 = back("d0a", back("d0b", dd0))
    dd1 = upsample2_grad(dcat0[:, :L[1]])
    de0 = dcat0[:, L[1]:]
    dcat1 = back("d1a", back("d1b", dd1))
    dd2 = upsample2_grad(dcat1[:, :L[2]])
    de1 = dcat1[:, L[2]:]
    dcat2 = back("d2a", back("d2b", dd2))
    de3 = upsample2_grad(dcat2[:, :L[3]])
    de2 = dcat2[:, L[3]:]
    dp2 = back("e3a", back("e3b", de3))
    de2 = de2 + avgpool2_grad(dp2)
    dp1 = back("e2a", back("e2b", de2))
    de1 = de1 + avgpool2_grad(dp1)
    dp0 = back("e1a", back("e1b", de1))
    de0 = de0 + avgpool2_grad(dp0)
    back("e0a", back("e0b", de0))
    return grads


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of p with gradient g; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
