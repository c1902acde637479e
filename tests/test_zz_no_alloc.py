"""The allocation-free mobility product (pse_mobility_apply_noalloc) against
the handle-based product on the same inputs: two calls in a row, the second
with fewer particles, both bit for bit equal to pse_mobility_apply."""
import numpy as np
import pytest

from paper_1709_06946_amd import inputs, pse

from gpu_common import dev, host, packing

pytestmark = pytest.mark.gpu


def _case(N, phi, precision, parts, seed):
    import torch
    x, L = packing(N, phi, inputs.SEED_BASE + seed)
    q = np.random.default_rng(seed).normal(size=(N, 11))
    kw = dict(grid=32, tol=1e-3, precision=precision)
    h = pse.PSE(N, L, **kw)
    ref = torch.zeros((N, 11), dtype=torch.float64, device='cuda:0')
    h.mobility_apply(dev(x), dev(q), ref, parts)
    h.close()
    # zeros like ref: with PSE_ES_BLOCK the product leaves components 0-5 of
    # out untouched
    out = torch.zeros((N, 11), dtype=torch.float64, device='cuda:0')
    pse.mobility_apply_noalloc(pse.make_params(N, L, **kw), dev(x), dev(q), out, parts)
    return host(out), host(ref)


@pytest.mark.parametrize('precision', [pse.PSE_FP64, pse.PSE_MIXED])
@pytest.mark.parametrize('parts', [pse.PSE_REAL | pse.PSE_WAVE,
                                   pse.PSE_REAL | pse.PSE_WAVE | pse.PSE_ES_BLOCK])
def test_noalloc_product_equals_handle_product(precision, parts):
    for N, seed in ((160, 31), (100, 32)):      # second call smaller
        print(f'noalloc case N={N} precision={precision} parts={parts}', flush=True)
        out, ref = _case(N, 0.1, precision, parts, seed)
        assert np.isfinite(out).all()
        assert np.array_equal(out, ref), np.abs(out - ref).max()


def test_noalloc_product_too_large_is_refused():
    import torch
    N = 100
    x, L = packing(N, 0.1, inputs.SEED_BASE + 33)
    q = torch.zeros((N, 11), dtype=torch.float64, device='cuda:0')
    out = torch.zeros_like(q)
    with pytest.raises(pse.PSEError, match='scratch'):
        pse.mobility_apply_noalloc(pse.make_params(N, L, grid=128), dev(x), q, out)
