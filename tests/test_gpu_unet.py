"""Warm-start U-Net on the GPU (bf16 matrix cores, FP32 accumulation) against its CPU oracle
on the same bf16-valued weights and inputs.  Both sides round to bf16 at the same points,
so the remaining differences are FP32 versus exact sums (an occasional one-ulp bf16 flip
that the following layers carry): the bars are relative L2 errors, written per test."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import unet_oracle as U
import paper_2011_06842_amd as fw

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GROUPS = [(2, 32), (3, 16)]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def flat(p):
    parts = []
    for name, _, _ in U.conv_names():
        parts += [p[name + ".w"].ravel(), p[name + ".b"]]
    parts += [p["head.w"], p["head.b"]]
    return np.concatenate(parts)


def unflat(v):
    out, o = {}, 0
    for name, cin, cout in U.conv_names():
        n = 9 * cin * cout
        out[name + ".w"] = v[o:o + n].reshape(3, 3, cin, cout)
        o += n
        out[name + ".b"] = v[o:o + cout]
        o += cout
    out["head.w"], out["head.b"] = v[o:o + 32], v[o + 32:o + 33]
    return out


def setup_case(seed=0, groups=GROUPS):
    rng = np.random.default_rng(seed)
    p = U.init_params(rng)
    for k in p:
        if k.endswith(".b"):
            p[k] = (0.05 * rng.standard_normal(p[k].shape)).astype(np.float32).astype(np.float64)
    p["head.w"] = U.bf16(0.2 * rng.standard_normal(32))
    xs, ts = [], []
    for n, s in groups:
        xs.append(rng.standard_normal((n, s, s, 4)).astype(np.float32))
        ts.append(rng.standard_normal((n, s, s)).astype(np.float32))
    return p, xs, ts


def oracle_inputs(x):
    xi = np.zeros(x.shape[:3] + (U.IN_CH,))
    xi[..., :4] = U.bf16(x)
    return xi


def gpu_net(p, groups=GROUPS):
    net = fw.UNetContext(groups, lr=1e-3, device=DEV)
    net.set_params(torch.from_numpy(flat(p).astype(np.float32)).to(DEV))
    return net


def dev_cat(arrs):
    return torch.from_numpy(np.concatenate([a.ravel() for a in arrs]).astype(np.float32)).to(DEV)


def test_parameter_round_trip_and_sizes():
    p, _, _ = setup_case()
    net = gpu_net(p)
    v = flat(p)
    assert net.n_params == v.size
    assert net.nodes == sum(n * s * s for n, s in GROUPS)
    back = net.get_params().cpu().numpy()
    np.testing.assert_array_equal(back, v.astype(np.float32))


def test_forward_matches_oracle():
    p, xs, _ = setup_case(1)
    net = gpu_net(p)
    out = net.forward(dev_cat(xs)).cpu().numpy()
    ref = np.concatenate([U.forward(p, oracle_inputs(x))[0].ravel() for x in xs])
    assert rel(out, ref) <= 5e-3, rel(out, ref)


def _oracle_grads(p, xs, ts):
    outs, actss = [], []
    for x in xs:
        o, a = U.forward(p, oracle_inputs(x))
        outs.append(o)
        actss.append(a)
    total = sum(o.size for o in outs)
    loss = sum(float(np.sum((o - t) ** 2)) for o, t in zip(outs, ts)) / total
    g = None
    for o, t, a in zip(outs, ts, actss):
        gi = U.backward(p, a, 2.0 * (o - t) / total)
        g = gi if g is None else {k: g[k] + gi[k] for k in g}
    return loss, g


def _oracle_self_sensitivity(p, xs, ts, gref):
    """How far the oracle's own gradients move when every value is perturbed at the FP32
    rounding level (relative 2^-24) before it is rounded to bf16: the intrinsic noise of a
    bf16 backward pass, against which the GPU's FP32 sums are judged."""
    orig = U.bf16
    rng = np.random.default_rng(0)
    U.bf16 = lambda v: orig(np.asarray(v, dtype=np.float64) * (1 + 2.0 ** -24 * rng.standard_normal(np.shape(v))))
    try:
        _, gp = _oracle_grads(p, xs, ts)
    finally:
        U.bf16 = orig
    return {k: rel(gp[k], gref[k]) for k in gref}


def test_backward_matches_oracle_per_parameter_group():
    """Bar per parameter group: twice the oracle's own deviation under FP32-sized
    perturbations (deep layers carry a few percent of bf16 noise), plus 1e-3."""
    p, xs, ts = setup_case(2)
    net = gpu_net(p)
    loss = net.backward(dev_cat(xs), dev_cat(ts)).cpu().numpy()[0]
    g = unflat(net.get_grads().cpu().numpy().astype(np.float64))
    ref_loss, gref = _oracle_grads(p, xs, ts)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    np.testing.assert_array_equal(g["e0a.w"][:, :, U.N_INPUTS:, :], 0.0)   # padded input channels
    noise = _oracle_self_sensitivity(p, xs, ts, gref)
    bad = {k: (rel(g[k], gref[k]), noise[k]) for k in gref if rel(g[k], gref[k]) > 2 * noise[k] + 1e-3}
    assert not bad, bad
    assert rel(g["head.w"], gref["head.w"]) <= 1e-3 and rel(g["d0b.w"], gref["d0b.w"]) <= 1e-2


def test_backward_with_many_chunk_partials_matches_oracle():
    """Two 128^2 images: the weight gradients are summed from 512 (32-channel level), 128, 64 and
    fewer chunk partials, so the fixed-order reduction spreads an entry's eight running sums over
    eight, four, two and one threads; same bars as the test above."""
    groups = [(2, 128)]
    p, xs, ts = setup_case(5, groups)
    net = gpu_net(p, groups)
    loss = net.backward(dev_cat(xs), dev_cat(ts)).cpu().numpy()[0]
    g = unflat(net.get_grads().cpu().numpy().astype(np.float64))
    ref_loss, gref = _oracle_grads(p, xs, ts)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    noise = _oracle_self_sensitivity(p, xs, ts, gref)
    bad = {k: (rel(g[k], gref[k]), noise[k]) for k in gref if rel(g[k], gref[k]) > 2 * noise[k] + 1e-3}
    assert not bad, bad


def test_adam_step_matches_oracle_on_the_same_gradients():
    p, xs, ts = setup_case(3)
    net = gpu_net(p)
    net.backward(dev_cat(xs), dev_cat(ts))
    g = unflat(net.get_grads().cpu().numpy().astype(np.float64))
    net.adam_step()
    w = unflat(net.get_params().cpu().numpy().astype(np.float64))
    opt = U.Adam({k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}, lr=1e-3)
    opt.step(g)
    for k in p:
        np.testing.assert_allclose(w[k], opt.master[k], rtol=1e-5, atol=1e-7, err_msg=k)


def _oracle_training(p, xs, ts, steps, perturb=False):
    """The oracle's loss after each of `steps` Adam steps on the same batch (bf16 network,
    FP64 master weights); perturb: every value is perturbed by a relative 2^-24 before its bf16
    rounding (the oracle's own sensitivity)."""
    orig = U.bf16
    rng = np.random.default_rng(1)
    if perturb:
        U.bf16 = lambda v: orig(np.asarray(v, dtype=np.float64) * (1 + 2.0 ** -24 * rng.standard_normal(np.shape(v))))
    try:
        opt = U.Adam({k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}, lr=1e-3)
        losses = []
        for _ in range(steps):
            loss, g = _oracle_grads(opt.params(), xs, ts)
            losses.append(loss)
            opt.step(g)
    finally:
        U.bf16 = orig
    return losses


def test_training_follows_the_oracle():
    """40 Adam steps on the GPU against the same 40 steps of the oracle.  bf16 trajectories
    part slowly (one-ulp flips carry), so the bar on every step's loss is three times the
    oracle's own drift under FP32-sized perturbations, plus 2 %; and training lowers the loss by
    at least 30 %."""
    p, xs, ts = setup_case(4)
    net = gpu_net(p)
    x, t = dev_cat(xs), dev_cat(ts)
    losses = []
    for _ in range(40):
        losses.append(float(net.backward(x, t).cpu().numpy()[0]))
        net.adam_step()
    ref = _oracle_training(p, xs, ts, 40)
    pert = _oracle_training(p, xs, ts, 40, perturb=True)
    drift = [abs(a - b) / b for a, b in zip(pert, ref)]
    rows = [(k, losses[k], ref[k], drift[k]) for k in range(0, 40, 8)] + [(39, losses[-1], ref[-1], drift[-1])]
    print("step, GPU loss, oracle loss, oracle drift:", rows)
    for k in range(40):
        assert abs(losses[k] - ref[k]) <= (3 * max(drift[:k + 1]) + 0.02) * ref[k], rows
    assert losses[-1] < 0.7 * losses[0], rows
