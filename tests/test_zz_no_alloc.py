"""fewha_apply_A_noalloc through the C ABI: the same y = M x as fewha_apply_A, with the
intermediates in the library's static device array; two calls in a row on contexts of
decreasing size (the array keeps the first call's contents), then a system whose
intermediates do not fit (rejected, nothing launched)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
import paper_2011_06842_amd as fw

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_apply_equals_apply_A_on_two_calls(precision):
    big = synth.config_elt_mcao(precision=precision)
    synth.make_sequence(big, 1, seed=6)          # calibrates the noise weights
    small = synth.config_small()
    synth.make_sequence(small, 1, seed=5)
    small.precision = precision
    rng = np.random.default_rng(3)
    for spec in (big, small):                    # the second call has the smaller input
        ctx = fw.FewhaContext(spec, device=DEV)
        x = torch.from_numpy(rng.standard_normal(ctx.N)).to(device=DEV, dtype=ctx.dtype)
        y_ref = ctx.fewha_apply_A(x)
        y = torch.full_like(y_ref, float("nan"))
        ctx.fewha_apply_A_noalloc(x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), (spec.name, float((y - y_ref).abs().max()))


def test_noalloc_rejects_systems_beyond_the_static_array():
    spec = synth.config_elt_mcao(precision="fp64", other_n=256)   # 9 x 256^2: 22 MB of intermediates
    for w in spec.wfs:
        w.weight = np.ones(2 * w.n_sub * w.n_sub)
    N = sum(l.n ** 2 for l in spec.layers)
    ctx = fw.FewhaContext(spec, device=DEV, precond_inv=np.ones(N))
    x = torch.zeros(ctx.N, dtype=ctx.dtype, device=DEV)
    y = torch.full_like(x, 7.0)
    with pytest.raises(fw.FewhaError) as e:
        ctx.fewha_apply_A_noalloc(x, y)
    assert "FEWHA_E_NOMEM" in str(e.value) and "16 MiB" in str(e.value)
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
