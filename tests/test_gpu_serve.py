"""Served form: requests of different N and volume fraction admitted by
device footprint onto one GPU, running concurrently (after a synchronous
first step, each request's steps are replays of one captured graph of the
whole step).  Each request's result is the same alone and in the mix, bit
for bit: nothing in a request's work depends on the others."""
import numpy as np
import pytest

from paper_1709_06946_amd import inputs

pytestmark = pytest.mark.gpu

REQS = [(300, 0.1), (500, 0.2), (800, 0.1), (1200, 0.15), (400, 0.3)]


def _requests():
    out = []
    for i, (n, phi) in enumerate(REQS):
        x, L = inputs.packing(n, phi, seed=inputs.SEED_BASE + 200 + i)
        FL = inputs.forces_torques(n, inputs.SEED_BASE + 300 + i)
        out.append((x, L, FL, 1000 + i))
    return out


def _run(server, reqs, precision, steps=4):
    from paper_1709_06946_amd import pse
    ids = [server.submit(x, L, FL=FL, steps=steps, seed=seed, grid=pse.grid_for(L),
                         gmres_tol=1e-6, lanczos_tol=1e-3, precision=precision)
           for x, L, FL, seed in reqs]
    res = []
    for rid in ids:
        info = server.wait(rid)
        x, lat = server.result(rid)
        res.append((info, x, lat))
    return res


@pytest.mark.parametrize('precision', [0, 1])
def test_alone_equals_mix_and_budget_respected(precision):
    from paper_1709_06946_amd import pse
    reqs = _requests()
    alone = []
    s1 = pse.PSEServer(max_active=1)
    for r in reqs:
        alone.append(_run(s1, [r], precision)[0])
    s1.close()
    sizes = sorted(i[0]['bytes'] for i in alone)
    budget = sizes[-1] + sizes[-2] + sizes[0]          # at most ~3 at once
    s2 = pse.PSEServer(budget_bytes=budget, max_active=4)
    mix = _run(s2, reqs, precision)
    st = s2.stats()
    s2.close()
    assert st['completed'] == len(reqs) and st['failed'] == 0
    assert st['peak_used'] <= budget
    assert 2 <= st['peak_active'] <= 4
    for (ia, xa, la), (im, xm, lm), (x0, L, FL, seed) in zip(alone, mix, reqs):
        assert ia['status'] == 0 and im['status'] == 0
        da = xa - x0
        da -= L * np.rint(da / L)
        dm = xm - x0
        dm -= L * np.rint(dm / L)
        err = np.abs(da - dm).max() / np.abs(da).max()
        print(len(x0), 'alone vs mix', err, 'latency ms', np.round(lm, 2))
        assert np.array_equal(xa, xm), err
        assert len(lm) == 4 and np.all(lm > 0)
    # requests overlapped in time on the device
    spans = sorted((i['t_admit'], i['t_done']) for i, _, _ in mix)
    assert any(spans[k + 1][0] < spans[k][1] for k in range(len(spans) - 1))


def test_creates_and_copies_overlapping_captures_do_not_fail():
    """Many short requests, six at a time, in both precisions: handles are
    created, filled and freed by some workers while others capture their
    constraint-operator graphs.  Those calls and the captures are kept apart
    by the library, so no request fails and every result is finite."""
    from paper_1709_06946_amd import pse
    reqs = []
    for i in range(18):
        n = 400 + 150 * (i % 7)
        x, L = inputs.packing(n, 0.1 + 0.05 * (i % 5), seed=inputs.SEED_BASE + 400 + i)
        reqs.append((x, L, inputs.forces_torques(n, inputs.SEED_BASE + 500 + i)))
    srv = pse.PSEServer(max_active=6)
    ids = [srv.submit(x, L, FL=FL, steps=3, seed=2000 + i, grid=pse.grid_for(L),
                      precision=pse.PSE_MIXED if i % 2 else pse.PSE_FP64)
           for i, (x, L, FL) in enumerate(reqs)]
    for rid in ids:
        info = srv.wait(rid)
        x, lat = srv.result(rid)
        assert info['status'] >= 0 and np.isfinite(x).all() and len(lat) == 3
    st = srv.stats()
    srv.close()
    print('peak active', st['peak_active'], 'completed', st['completed'])
    assert st['failed'] == 0 and st['completed'] == 18
    assert st['peak_active'] >= 2
