"""Plain CPU oracle of the learned warm start: a small U-Net, its explicit backward pass, the
mean-squared-error loss and Adam.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the benchmark's CPU leg;
never by the GPU library.  NumPy, float64 arithmetic, written for a reader: every layer is
its definition (a 3 x 3 convolution is the sum over its nine taps of shifted images times
a channel-mixing matrix), no blocking and no fusion.

The network (the warm-start model of the learned extension; the paper has none):

* encoder levels 0-3 with 32, 64, 128, 256 channels, two 3 x 3 convolutions (zero
  padding, bias, ReLU) per level, 2 x 2 average pooling between levels;
* decoder levels 2, 1, 0: 2x nearest upsampling of the coarser features, concatenation
  [upsampled, encoder skip] along channels, two 3 x 3 convolutions (bias, ReLU);
* a 1 x 1 convolution (bias, no activation) from 32 channels to 1.

Mixed precision, as the GPU computes it: weights and activations are rounded to bfloat16
(round to nearest even) where the GPU stores them; sums are exact here (float64) and FP32
on the GPU; gradients and Adam states stay in float32/float64.

Tensors are NHWC arrays (images, rows, columns, channels).  The input has 4 channels,
zero-padded to IN_CH = 32 for the first convolution.
"""
from __future__ import annotations

import numpy as np

LEVEL_CH = (32, 64, 128, 256)
IN_CH = 32          # input channels after zero padding (4 used)
N_INPUTS = 4


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


# ------------------------------------------------------------------ layers (definitions)

def conv3x3(x, w, b=None):
    """Same-size 3 x 3 convolution (cross-correlation) with zero padding.
    x: (N, H, W, Cin); w: (3, 3, Cin, Cout) indexed [dy + 1, dx + 1, ci, co]; b: (Cout,)."""
    N, H, W, _ = x.shape
    xp = np.zeros((N, H + 2, W + 2, x.shape[3]))
    xp[:, 1:-1, 1:-1, :] = x
    out = np.zeros((N, H, W, w.shape[3]))
    for ty in range(3):
        for tx in range(3):
            out += xp[:, ty:ty + H, tx:tx + W, :] @ w[ty, tx]
    if b is not None:
        out += b
    return out


def conv3x3_input_grad(dy, w):
    """Adjoint of conv3x3 in its input: dx[p] = sum_taps dy[p - tap] w[tap]^T."""
    N, H, W, _ = dy.shape
    dyp = np.zeros((N, H + 2, W + 2, dy.shape[3]))
    dyp[:, 1:-1, 1:-1, :] = dy
    dx = np.zeros((N, H, W, w.shape[2]))
    for ty in range(3):
        for tx in range(3):
            # output pixel q reads input q + (ty-1, tx-1): input pixel p gets dy[p - (ty-1, tx-1)]
            dx += dyp[:, 2 - ty:2 - ty + H, 2 - tx:2 - tx + W, :] @ w[ty, tx].T
    return dx


def conv3x3_weight_grad(x, dy):
    """dL/dw[ty, tx, ci, co] = sum_p x[p + (ty-1, tx-1), ci] dy[p, co] (zero padding)."""
    N, H, W, Cin = x.shape
    xp = np.zeros((N, H + 2, W + 2, Cin))
    xp[:, 1:-1, 1:-1, :] = x
    gw = np.zeros((3, 3, Cin, dy.shape[3]))
    for ty in range(3):
        for tx in range(3):
            xs = xp[:, ty:ty + H, tx:tx + W, :].reshape(-1, Cin)
            gw[ty, tx] = xs.T @ dy.reshape(-1, dy.shape[3])
    return gw


def avg_pool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avg_pool2_grad(dy):
    """Adjoint of avg_pool2: every input pixel gets a quarter of its window's gradient."""
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_grad(dy):
    """Adjoint of nearest upsampling: the sum over each 2 x 2 window."""
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0.0)


# ------------------------------------------------------------------ parameters

def conv_names():
    """Names and (Cin, Cout) of the 3 x 3 convolutions in forward order."""
    c = LEVEL_CH
    return [("e0a", IN_CH, c[0]), ("e0b", c[0], c[0]), ("e1a", c[0], c[1]), ("e1b", c[1], c[1]),
            ("e2a", c[1], c[2]), ("e2b", c[2], c[2]), ("e3a", c[2], c[3]), ("e3b", c[3], c[3]),
            ("d2a", c[3] + c[2], c[2]), ("d2b", c[2], c[2]), ("d1a", c[2] + c[1], c[1]), ("d1b", c[1], c[1]),
            ("d0a", c[1] + c[0], c[0]), ("d0b", c[0], c[0])]


def init_params(rng, scale=1.0):
    """He-normal weights (rounded to bf16), zero biases; the 1 x 1 head starts small."""
    p = {}
    for name, cin, cout in conv_names():
        fan_in = 9 * (N_INPUTS if name == "e0a" else cin)
        w = rng.standard_normal((3, 3, cin, cout)) * np.sqrt(2.0 / fan_in) * scale
        if name == "e0a":
            w[:, :, N_INPUTS:, :] = 0.0          # padded input channels
        p[name + ".w"] = bf16(w)
        p[name + ".b"] = np.zeros(cout)
    p["head.w"] = bf16(rng.standard_normal(LEVEL_CH[0]) * 0.01)
    p["head.b"] = np.zeros(1)
    return p


# ------------------------------------------------------------------ network

def forward(p, x):
    """x: (N, H, W, IN_CH) bf16-valued input.  Returns the output (N, H, W) and the saved
    activations (bf16-valued, as stored by the GPU)."""
    acts = {"x": x}

    def cbr(name, inp):
        y = bf16(relu(conv3x3(inp, p[name + ".w"], p[name + ".b"])))
        acts[name] = y
        return y

    e0 = cbr("e0b", cbr("e0a", x))
    e1 = cbr("e1b", cbr("e1a", bf16(avg_pool2(e0))))
    e2 = cbr("e2b", cbr("e2a", bf16(avg_pool2(e1))))
    e3 = cbr("e3b", cbr("e3a", bf16(avg_pool2(e2))))
    d2 = cbr("d2b", cbr("d2a", np.concatenate([upsample2(e3), e2], axis=3)))
    d1 = cbr("d1b", cbr("d1a", np.concatenate([upsample2(d2), e1], axis=3)))
    d0 = cbr("d0b", cbr("d0a", np.concatenate([upsample2(d1), e0], axis=3)))
    out = d0 @ p["head.w"] + p["head.b"][0]
    return out, acts


def mse_loss(out, target):
    """Mean over all pixels of (out - target)^2 and its gradient."""
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(p, acts, dout):
    """Gradients of every parameter for the output gradient dout (N, H, W).  Activation
    gradients are kept in float64 (the GPU keeps them in FP32) and rounded to bf16 where
    they enter a convolution's matrix products."""
    g = {}
    d0 = acts["d0b"]
    g["head.w"] = np.einsum("nhwc,nhw->c", d0, dout)
    g["head.b"] = np.array([dout.sum()])
    dd0 = dout[..., None] * p["head.w"]

    def cbr_back(name, inp, dy):
        # ReLU', then bf16: the matrix cores take the gradient as bf16 (sums stay exact)
        dpre = bf16(dy * (acts[name] > 0))
        g[name + ".w"] = conv3x3_weight_grad(inp, dpre)
        g[name + ".b"] = dpre.sum(axis=(0, 1, 2))
        return conv3x3_input_grad(dpre, p[name + ".w"])

    def split(dcat, c_up):
        return dcat[..., :c_up], dcat[..., c_up:]

    c = LEVEL_CH
    x = acts["x"]
    e0, e1, e2, e3 = acts["e0b"], acts["e1b"], acts["e2b"], acts["e3b"]
    d1, d2 = acts["d1b"], acts["d2b"]
    # decoder level 0
    dcat0 = cbr_back("d0a", np.concatenate([upsample2(d1), e0], axis=3), cbr_back("d0b", acts["d0a"], dd0))
    dup1, de0 = split(dcat0, c[1])
    dd1 = upsample2_grad(dup1)
    dcat1 = cbr_back("d1a", np.concatenate([upsample2(d2), e1], axis=3), cbr_back("d1b", acts["d1a"], dd1))
    dup2, de1 = split(dcat1, c[2])
    dd2 = upsample2_grad(dup2)
    dcat2 = cbr_back("d2a", np.concatenate([upsample2(e3), e2], axis=3), cbr_back("d2b", acts["d2a"], dd2))
    dup3, de2 = split(dcat2, c[3])
    de3 = upsample2_grad(dup3)
    # encoder, from the bottom: each level's output also feeds the next level's pooling
    dp2 = cbr_back("e3a", bf16(avg_pool2(e2)), cbr_back("e3b", acts["e3a"], de3))
    de2 = de2 + avg_pool2_grad(dp2)
    dp1 = cbr_back("e2a", bf16(avg_pool2(e1)), cbr_back("e2b", acts["e2a"], de2))
    de1 = de1 + avg_pool2_grad(dp1)
    dp0 = cbr_back("e1a", bf16(avg_pool2(e0)), cbr_back("e1b", acts["e1a"], de1))
    de0 = de0 + avg_pool2_grad(dp0)
    cbr_back("e0a", x, cbr_back("e0b", acts["e0a"], de0))
    g["e0a.w"][:, :, N_INPUTS:, :] = 0.0            # padded input channels are not trained
    return g


# ------------------------------------------------------------------ Adam (Kingma and Ba, 2015)

class Adam:
    """Adam with bias correction: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).  Master weights in float64;
    the network uses their bf16 rounding (biases stay full precision)."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.master = {k: np.array(v, dtype=np.float64) for k, v in params.items()}
        self.m = {k: np.zeros_like(v) for k, v in self.master.items()}
        self.v = {k: np.zeros_like(v) for k, v in self.master.items()}
        self.lr, self.b1, self.b2, self.eps, self.t = lr, b1, b2, eps, 0

    def step(self, grads):
        self.t += 1
        for k, gk in grads.items():
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * gk
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * gk * gk
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            self.master[k] = self.master[k] - self.lr * mh / (np.sqrt(vh) + self.eps)

    def params(self):
        return {k: (v if k.endswith(".b") else bf16(v)) for k, v in self.master.items()}
