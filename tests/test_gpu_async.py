"""Asynchronous handles (pse_params.async_calls = 1): Krylov solves checked on
the device, no host synchronisation inside a call, so that whole steps can
be captured into a graph and replayed.

* One step of an asynchronous handle equals (bit for bit) the step of a
  synchronous handle from the same state and noise: the device picks the
  same iteration of each solve as the host would.
* Steps captured into one graph (torch.cuda.graph on the handle's stream,
  noise counter from the device, PSE_STEP_DEVICE) and replayed twice give
  the positions of the same steps made by eager calls, bit for bit.
* The device statistics and status word: a non-finite position is flagged.
"""
import numpy as np
import pytest

from paper_1709_06946_amd import inputs, pse

from gpu_common import dev, host, packing

pytestmark = pytest.mark.gpu

N, PHI, DT, SEED = 100, 0.1, 1e-3, 4242


def _setup(seed=SEED + 1):
    x, L = packing(N, PHI, inputs.SEED_BASE + 120)
    FL = inputs.forces_torques(N, seed)
    return x, L, FL


@pytest.mark.parametrize('precision', [pse.PSE_FP64, pse.PSE_MIXED])
def test_async_step_equals_sync_step(precision):
    import torch
    x, L, FL = _setup()
    kw = dict(grid=32, tol=1e-3, precision=precision, gmres_tol=1e-6)
    hs = pse.PSE(N, L, **kw)
    xs = dev(x)
    rc, st = hs.constrained_step(xs, dev(FL), DT, seed=SEED, step=3)
    assert rc == 0 and st['converged'] == 1
    s = torch.cuda.Stream()
    # as many refinement passes as the synchronous solve took (it stops at
    # the first pass that meets the tolerance; the asynchronous one runs all)
    if precision == pse.PSE_MIXED:
        kw['refine_passes'] = st['refine_passes']
    ha = pse.PSE(N, L, stream=s.cuda_stream, async_calls=1, **kw)
    with torch.cuda.stream(s):
        xa = dev(x)
        FLa = dev(FL)
    s.synchronize()
    rc_a, none = ha.constrained_step(xa, FLa, DT, seed=SEED, step=3)
    assert rc_a == 0 and none is None
    sa = ha.stats()
    print(f'sync {st}\nasync {sa}', flush=True)
    assert np.array_equal(host(xa), host(xs))
    assert sa['converged'] == 1 and sa['status'] == 0
    assert sa['lanczos_iters'] == st['lanczos_iters']
    assert sa['gmres_iters'] == st['gmres_iters']
    assert sa['fp64_residual'] == pytest.approx(st['fp64_residual'], rel=1e-12)
    hs.close()
    ha.close()


@pytest.mark.parametrize('precision', [pse.PSE_FP64, pse.PSE_MIXED])
def test_captured_steps_replay_like_eager_steps(precision):
    import torch
    K = 3
    x, L, FL = _setup()
    kw = dict(grid=32, tol=1e-3, precision=precision, gmres_tol=1e-6, async_calls=1)
    # eager reference: 2K asynchronous steps with explicit step numbers
    he = pse.PSE(N, L, **kw)
    xe, FLe = dev(x), dev(FL)
    ref = []
    for k in range(2 * K):
        he.constrained_step(xe, FLe, DT, seed=SEED, step=k)
        if k % K == K - 1:
            he.synchronize()          # the handle's own stream, not torch's
            ref.append(host(xe))
    assert he.stats()['converged'] == 1
    he.close()
    s = torch.cuda.Stream()
    hg = pse.PSE(N, L, stream=s.cuda_stream, **kw)
    with torch.cuda.stream(s):
        xg, FLg = dev(x), dev(FL)
        x0 = xg.clone()
        # warm-up (explicit step number: the device counter stays at 0)
        hg.constrained_step(xg, FLg, DT, seed=SEED, step=77)
        xg.copy_(x0)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode='thread_local'):
        for _ in range(K):
            hg.constrained_step(xg, FLg, DT, seed=SEED, step=pse.PSE_STEP_DEVICE)
    torch.cuda.synchronize()
    assert np.array_equal(host(xg), x)          # capture ran nothing
    for r in range(2):
        print(f'replay {r}', flush=True)
        g.replay()
        torch.cuda.synchronize()
        got = host(xg)
        assert np.array_equal(got, ref[r]), np.abs(got - ref[r]).max()
        st = hg.stats()
        assert st['converged'] == 1 and st['status'] == 0
        # eager work of the program between replays
        tmp = torch.ones(1000, device='cuda:0').sum()
        torch.cuda.synchronize()
        assert float(tmp) == 1000.0
    del g
    hg.close()


def test_async_status_flags_nonfinite_position():
    import torch
    x, L, FL = _setup()
    x = x.copy()
    x[7, 1] = np.nan
    h = pse.PSE(N, L, grid=32, tol=1e-3, async_calls=1)
    xd = dev(x)
    h.constrained_step(xd, dev(FL), DT, seed=SEED, step=0)
    st = h.stats()
    assert st['status'] & pse.PSE_STATUS_NONFINITE_POS
    h.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize('precision', [pse.PSE_FP64, pse.PSE_MIXED])
def test_step_graph_through_the_abi(precision):
    """pse_set_krylov / pse_step_graph_*: one synchronous step, then the
    handle switched to asynchronous calls with the learned iteration counts
    and one captured step replayed three times; the positions equal those of
    three eager asynchronous steps with explicit step numbers 1, 2, 3."""
    import torch
    x, L, FL = _setup()
    kw = dict(grid=32, tol=1e-3, precision=precision, gmres_tol=1e-6)
    outs = []
    for mode in ('graph', 'eager'):
        h = pse.PSE(N, L, **kw)
        xd, FLd = dev(x), dev(FL)
        rc, st = h.constrained_step(xd, FLd, DT, seed=SEED, step=0)
        assert rc == 0
        passes = max(1, st['refine_passes'])
        caps = (st['lanczos_iters'] + 1, st['gmres_iters'] // passes + 3, passes)
        h.set_krylov(1, *caps, next_step=1)
        if mode == 'graph':
            g = h.step_graph(xd, FLd, DT, seed=SEED, steps=1)
            for _ in range(3):
                g.launch()
                h.synchronize()
                sg = h.stats()
                assert sg['converged'] == 1 and sg['status'] == 0
            g.close()
        else:
            for k in (1, 2, 3):
                h.constrained_step(xd, FLd, DT, seed=SEED, step=k)
            assert h.stats()['converged'] == 1
        torch.cuda.synchronize()
        outs.append(host(xd))
        h.close()
    assert np.array_equal(outs[0], outs[1])
