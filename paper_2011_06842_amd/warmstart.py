"""Learned warm start: data collection and training through the C ABI (fewha_solve_aug,
fewha_warmstart_input, fewha_apply_piece and the fewha_unet_* calls).  The solves, the network
inputs, the nodal fields and the network's forward and backward passes run in the library's
HIP kernels; this module orders the calls, forms the training target as the difference of two
coefficient vectors (a torch subtraction) and normalises the samples on the host (NumPy).

A sample pairs, for one frame transition i -> i+1 of a slope sequence,
  input  [W^-1 c_i, W^-1 J^-1 r, h / 20 km, gamma] per layer node, with c_i the coefficients the
         deployed solver produced for frame i and r = b_{i+1} - M c_i the new true residual,
  target W^-1 (c*_{i+1} - c_i), with c*_{i+1} a converged solve of frame i+1,
both normalised by their root-mean-square values (kept with the model as the warm start's
scales)."""
from __future__ import annotations

import numpy as np

from ._lib import PIECE_WINV, UNetContext


def layer_groups(spec):
    """U-Net image groups of a system: consecutive layers of equal grid size."""
    groups = []
    for lay in spec.layers:
        if groups and groups[-1][1] == lay.n:
            groups[-1] = (groups[-1][0] + 1, lay.n)
        else:
            groups.append((1, lay.n))
    return groups


def collect(spec, plain, truth, slopes, device="cuda"):
    """Samples of one slope sequence.  `plain` is the deployed solver's context (its frames
    give c_i), `truth` a context converged far below the deployment tolerance (its frames
    give c*_{i+1}); both start at frame 0.  Returns raw (unnormalised) host arrays
    x (T-1, N, 4) and y (T-1, N)."""
    import torch
    dt = torch.float64 if spec.precision == "fp64" else torch.float32
    xs, ys = [], []
    c_prev = None
    for t in range(slopes.shape[0]):
        s = torch.from_numpy(np.ascontiguousarray(slopes[t])).to(device=device, dtype=dt)
        c_star = truth.fewha_solve_aug(s)
        if c_prev is not None:
            x = plain.fewha_warmstart_input((1.0, 1.0), c_prev, s).cpu().numpy()
            y = plain.fewha_apply_piece(PIECE_WINV, (c_star - c_prev).contiguous()).float().cpu().numpy()
            xs.append(x)
            ys.append(y)
        c_prev = plain.fewha_solve_aug(s).clone()
    return np.stack(xs), np.stack(ys)


def scales_of(x, y):
    """Root-mean-square normalisation of the two field inputs and of the target."""
    rms = lambda a: float(np.sqrt(np.mean(np.square(a, dtype=np.float64)))) or 1.0
    return rms(x[..., 0]), rms(x[..., 1]), rms(y)


def normalise(x, y, scales):
    sc, sr, so = scales
    xn = x.copy()
    xn[..., 0] /= sc
    xn[..., 1] /= sr
    return xn, y / so


def train(spec, x, y, batch, epochs, lr=1e-3, seed=0, params=None, device="cuda", log=None):
    """Adam on the normalised samples (x (S, N, 4), y (S, N)) in minibatches of `batch`
    frames; returns the trained network's parameters (device FP32) and the loss history."""
    import torch
    groups = [(n * batch, size) for n, size in layer_groups(spec)]
    net = UNetContext(groups, lr=lr, device=device)
    if params is None:
        params = init_params(net.n_params, spec, seed, device)
    net.set_params(params)
    rng = np.random.default_rng(seed)
    losses = []
    n = x.shape[0] - x.shape[0] % batch
    for ep in range(epochs):
        order = rng.permutation(x.shape[0])[:n]
        for b0 in range(0, n, batch):
            idx = order[b0:b0 + batch]
            xb = torch.from_numpy(_group_major(spec, x[idx], 4)).to(device)
            yb = torch.from_numpy(_group_major(spec, y[idx], 1)).to(device)
            losses.append(float(net.backward(xb, yb).cpu().numpy()[0]))
            net.adam_step()
        if log:
            log(f"epoch {ep}: loss {np.mean(losses[-max(1, n // batch):]):.4g}")
    return net.get_params(), losses


def _group_major(spec, a, ch):
    """(B, N[, ch]) frames -> the network's order: for each group of equal-size layers, every
    frame's images of that group, one after the other."""
    out = []
    o = 0
    for cnt, size in layer_groups(spec):
        k = cnt * size * size
        out.append(a[:, o:o + k].reshape(-1))
        o += k
    return np.ascontiguousarray(np.concatenate(out), dtype=np.float32)


def init_params(n_params, spec, seed, device="cuda"):
    """He-normal 3 x 3 weights (fan-in 9 Cin; 4 live input channels for the first layer),
    zero biases, a zero output layer (the untrained network predicts no correction)."""
    import torch
    rng = np.random.default_rng(seed)
    ch = (32, 64, 128, 256)
    convs = [(32, ch[0]), (ch[0], ch[0]), (ch[0], ch[1]), (ch[1], ch[1]), (ch[1], ch[2]), (ch[2], ch[2]),
             (ch[2], ch[3]), (ch[3], ch[3]), (ch[3] + ch[2], ch[2]), (ch[2], ch[2]), (ch[2] + ch[1], ch[1]),
             (ch[1], ch[1]), (ch[1] + ch[0], ch[0]), (ch[0], ch[0])]
    parts = []
    for k, (cin, cout) in enumerate(convs):
        fan = 9 * (4 if k == 0 else cin)
        w = rng.standard_normal((3, 3, cin, cout)) * np.sqrt(2.0 / fan)
        if k == 0:
            w[:, :, 4:, :] = 0.0
        parts += [w.ravel(), np.zeros(cout)]
    parts += [np.zeros(32), np.zeros(1)]
    v = np.concatenate(parts).astype(np.float32)
    if v.size != n_params:
        raise ValueError(f"parameter count {v.size} != network's {n_params}")
    return torch.from_numpy(v).to(device)


def inference_net(spec, params, device="cuda"):
    """A one-frame network for fewha_solve_aug_ws with the given parameters."""
    net = UNetContext(layer_groups(spec), device=device)
    net.set_params(params)
    return net
