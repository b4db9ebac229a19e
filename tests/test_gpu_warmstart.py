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
