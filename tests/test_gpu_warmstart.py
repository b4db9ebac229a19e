"""Learned warm start inside the frame solve (fewha_solve_aug_ws), through the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import AugmentedReconstructor, OracleSystem
import paper_2011_06842_amd as fw
from paper_2011_06842_amd import warmstart as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def test_zero_correction_warm_start_matches_plain_oracle_frames():
    """An untrained network (zero output layer) predicts no correction: (e, M e) = 0, the
    line search takes no step, and the frames are the plain frames of the oracle up to
    rounding (FP64, 10 iterations)."""
    spec = synth.config_small()
    seq = synth.make_sequence(spec, 6, seed=11)
    ctx = fw.FewhaContext(spec, device=DEV)
    net = W.inference_net(spec, W.init_params(
        fw.UNetContext(W.layer_groups(spec), device=DEV).n_params, spec, 0, DEV), DEV)
    ref = AugmentedReconstructor(OracleSystem(spec))
    info = ctx.new_info()
    for t in range(6):
        c = ctx.fewha_solve_aug_ws(net, (1.0, 1.0, 1.0), dev(seq[t]), info=info)
        torch.cuda.synchronize()
        c_ref, _ = ref.solve(seq[t])
        assert rel(c.cpu().numpy(), c_ref) <= 1e-10, t
        gi = fw.decode_info(info)
        assert gi["flags"] == 4                      # the zero correction is never taken
    assert ctx.fewha_frame_iterations() == spec.max_iter


def _pattern_params(sign):
    """U-Net parameters whose output is input-independent and exactly representable: every
    convolution is zero except d0a's bias (channel 0: 0.75) and d0b's nine taps from channel 0
    to channel 0 (0.125 each), so d0b's channel 0 is 0.09375 times the number of taps inside
    the image (9 inside, 6 on an edge, 4 in a corner); the head maps it to sign (0.5 v - 0.25).
    Every value is a short dyadic fraction, so the bf16 network and the oracle agree bit for
    bit, and the correction has a border pattern (nonzero detail coefficients)."""
    from oracle import unet_oracle as U
    p = U.init_params(np.random.default_rng(0))
    for k in p:
        p[k] = np.zeros_like(p[k])
    p["d0a.b"][0] = 0.75
    p["d0b.w"][:, :, 0, 0] = 0.125
    p["head.w"][0] = 0.5 * sign
    p["head.b"][0] = -0.25 * sign
    flat = []
    for name, _, _ in U.conv_names():
        flat += [p[name + ".w"].ravel(), p[name + ".b"]]
    flat += [p["head.w"], p["head.b"]]
    return p, np.concatenate(flat).astype(np.float32)


def _oracle_correction(spec, p):
    """The oracle network as the correction; these parameters make its output independent of
    the input, so it is evaluated once (on the first frame's inputs) and reused."""
    from oracle import unet_oracle as U
    cache = []

    def corr(x):
        if not cache:
            out = []
            o = 0
            for cnt, size in W.layer_groups(spec):
                k = cnt * size * size
                xi = np.zeros((cnt, size, size, U.IN_CH))
                xi[..., :U.N_INPUTS] = U.bf16(x[o:o + k].reshape(cnt, size, size, U.N_INPUTS))
                out.append(U.forward(p, xi)[0].ravel())
                o += k
            cache.append(np.concatenate(out))
        return cache[0]
    return corr


def test_nonzero_correction_warm_start_matches_oracle_frames():
    """A fixed nonzero correction (a border pattern, exact on both sides): the packing into the
    network, the unpacking, e = W d, M e, the line search tau and the c / r update, then the
    frame's augmented PCG, all equal the oracle's warm-started frames at 1e-10 (FP64); the
    frames that take the step (tau > 0) and those that do not are the same on both sides, and
    at least one takes it."""
    spec = synth.config_small()
    seq = synth.make_sequence(spec, 6, seed=12)
    sysm = OracleSystem(spec)
    scales = (1.0, 1.0, 0.25)
    best = None
    for sign in (1.0, -1.0):   # the sign under which the oracle takes the most steps
        p, _ = _pattern_params(sign)
        ref = AugmentedReconstructor(sysm)
        taken = sum(ref.solve(seq[t], correction=_oracle_correction(spec, p), scales=scales)[1]["tau"] > 0
                    for t in range(6))
        if best is None or taken > best[0]:
            best = (taken, sign)
    assert best[0] >= 1
    p, flat = _pattern_params(best[1])
    net = W.inference_net(spec, torch.from_numpy(flat).to(DEV), DEV)
    ctx = fw.FewhaContext(spec, device=DEV)
    ref = AugmentedReconstructor(sysm)
    info = ctx.new_info()
    for t in range(6):
        c = ctx.fewha_solve_aug_ws(net, scales, dev(seq[t]), info=info)
        torch.cuda.synchronize()
        c_ref, i_ref = ref.solve(seq[t], correction=_oracle_correction(spec, p), scales=scales)
        gi = fw.decode_info(info)
        assert rel(c.cpu().numpy(), c_ref) <= 1e-10, (t, rel(c.cpu().numpy(), c_ref))
        assert (gi["flags"] & 4 == 0) == (i_ref["tau"] > 0), (t, gi, i_ref)


@pytest.mark.parametrize("precision, tol_c, tol_r", [("fp64", 1e-7, 1e-7), ("fp32", 1e-6, 2e-4)])
def test_warmstart_input_matches_oracle(precision, tol_c, tol_r):
    """fewha_warmstart_input: [W^-1 c / s_c, W^-1 J^-1 (b - M c) / s_r, h / 20 km, gamma] per
    node, against the oracle's inputs (FP32 output: the bars are FP32 rounding, and for the
    residual column in split precision the FP32 operator's error on b - M c)."""
    from oracle import warm_start_inputs
    spec = synth.config_small().copy(precision=precision)
    seq = synth.make_sequence(spec, 2, seed=13)
    sysm = OracleSystem(spec)
    dt = np.float64 if precision == "fp64" else np.float32
    ref = AugmentedReconstructor(sysm)
    c0, _ = ref.solve(seq[0].astype(dt).astype(np.float64))
    c0 = c0.astype(dt).astype(np.float64)
    s1 = seq[1].astype(dt).astype(np.float64)
    ctx = fw.FewhaContext(spec, device=DEV)
    x = ctx.fewha_warmstart_input((2.0, 0.5), dev(c0).to(ctx.dtype), dev(s1).to(ctx.dtype)).cpu().numpy()
    want = warm_start_inputs(sysm, c0, sysm.rhs(s1) - sysm.apply_M(c0, ref.D), ref.Jinv, 2.0, 0.5)
    assert rel(x[:, 0], want[:, 0]) <= tol_c
    assert rel(x[:, 1], want[:, 1]) <= tol_r
    np.testing.assert_array_equal(x[:, 2:], want[:, 2:].astype(np.float32))


def test_trained_warm_start_against_plain_augmented_pcg():
    """Train on converged solves of two sequences, evaluate on a third at equal final
    residual (tolerance mode): every frame crosses the tolerance with and without the warm
    start; the iterations to the first crossing are reported."""
    tol, cap = 1e-3, 120
    cal = [synth.config_small() for _ in range(3)]
    seqs = [synth.make_sequence(sp, 24, seed=s) for sp, s in zip(cal, (21, 22, 23))]
    base = cal[0]                                   # its noise weights serve every sequence
    spec = base.copy(rel_tol=tol, max_iter=cap)
    truth_spec = base.copy(rel_tol=1e-6, max_iter=256)
    xs, ys = [], []
    for sq in seqs[:2]:
        x, y = W.collect(spec, fw.FewhaContext(spec, device=DEV), fw.FewhaContext(truth_spec, device=DEV), sq, DEV)
        xs.append(x)
        ys.append(y)
    x, y = np.concatenate(xs), np.concatenate(ys)
    scales = W.scales_of(x, y)
    xn, yn = W.normalise(x, y, scales)
    params, losses = W.train(spec, xn, yn, batch=4, epochs=25, lr=1e-3)
    assert losses[-1] < 0.7 * losses[0], (losses[0], losses[-1])     # training makes progress
    net = W.inference_net(spec, params, DEV)
    plain = fw.FewhaContext(spec, device=DEV)
    warm = fw.FewhaContext(spec, device=DEV)
    ip, iw = plain.new_info(), warm.new_info()
    its_p, its_w, accepted = [], [], 0
    for t in range(seqs[2].shape[0]):
        s = dev(seqs[2][t])
        plain.fewha_solve_aug(s, info=ip)
        warm.fewha_solve_aug_ws(net, scales, s, info=iw)
        gp, gw = fw.decode_info(ip), fw.decode_info(iw)
        assert gp["flags"] & 2 == 0 and gw["flags"] & 2 == 0, t     # tolerance met by both
        # a frame runs on to the next host check (every 4 iterations) after its first crossing,
        # and the CG residual norm is not monotone: the final residual stays near the tolerance
        assert gp["rel_res"] <= 1.5 * tol and gw["rel_res"] <= 1.5 * tol, (t, gp, gw)
        if t > 0:
            its_p.append(gp["iters"])
            its_w.append(gw["iters"])
            accepted += 0 if gw["flags"] & 4 else 1
    print(f"\nwarm start: iterations to {tol:g} plain {np.mean(its_p):.2f}, warm {np.mean(its_w):.2f}, "
          f"accepted {accepted}/{len(its_w)}; training loss {losses[0]:.3g} -> {losses[-1]:.3g}")
    assert accepted >= len(its_w) // 2
    assert np.mean(its_w) <= np.mean(its_p) + 2.0
