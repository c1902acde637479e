"""Benchmark: stresslet-constrained PSE Brownian dynamics steps on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One "step" is one full mid-point step of the method (Sec. III.D): Lanczos
M_r^(1/2), wave-space M_w^(1/2), half step, GMRES on the stresslet
constraint, final mobility product and position update.  The default workload
is N = 10,000 hard spheres (a = 1) at phi = 0.3 in a 128^3 grid, eps = 1e-3,
dt = 1e-3, with random non-overlapping positions and N(0, 1) forces/torques.
Beside the FP64 headline: the mixed-precision form on the same workload, the
RPY-level comparison system (forces only, no constraint) and its cost ratio,
the served form (a Poisson stream of independent simulations of different N
and phi with p50/p99 per-step latency), and the FP64 oracle on host cores.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ('particle-steps/s (FTS Brownian, rel.err 1e-3) vs FP64; '
          'served p50/p99 step latency')
HBM_PEAK_GBS = 8000.0


def run_form(w, precision, steps, warmup, seed, prof_steps=2, deriv_gridding=0):
    """Times `steps` steps with the stage profiler off (the throughput), then
    runs `prof_steps` more with it on (stage times, launch durations)."""
    import torch

    from paper_1709_06946_amd import pse
    N = w['N']
    h = pse.PSE(N, w['L'], grid=w['grid'], tol=w['eps'], precision=precision,
                lanczos_tol=w['lanczos_tol'], gmres_tol=w['gmres_tol'],
                deriv_gridding=deriv_gridding)
    x = torch.tensor(w['x'], device='cuda:0')
    FL = torch.tensor(w['FL'], device='cuda:0')
    for k in range(warmup):
        h.constrained_step(x, FL, w['dt'], seed=seed, step=k)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        rc, st = h.constrained_step(x, FL, w['dt'], seed=seed, step=warmup + k)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k, st in enumerate(stats):
        print(f'# step {k} lanczos={st["lanczos_iters"]} gmres={st["gmres_iters"]} '
              f'res={st["fp64_residual"]:.2e}', file=sys.stderr, flush=True)
    h.profile(1)
    for k in range(prof_steps):
        h.constrained_step(x, FL, w['dt'], seed=seed, step=warmup + steps + k)
    torch.cuda.synchronize()
    h.profile(0)
    prof = h.profile_read()
    bracket = prof.pop('bracket', {'total_ms': 0.0})['total_ms']
    noop = prof.pop('bracket_noop', {'total_ms': 0.0})['total_ms']
    d = h.derived
    h.close()
    dt = t1 - t0
    return dict(value=N * steps / dt, ms_per_step=1e3 * dt / steps, prof=prof, stats=stats,
                prof_steps=prof_steps, bracket_us=(1e3 * bracket, 1e3 * noop),
                derived=dict(grid=d.grid, support=d.support, xi=d.xi, rcut=d.rcut,
                             deriv_gridding=d.deriv_gridding,
                             eta_s=d.eta_s), finite=bool(torch.isfinite(x).all()))


def run_rpy(w, steps, warmup, seed):
    """The RPY-level comparison system (forces only, Sec. IV) on the same
    workload in FP64: Euler-Maruyama steps with the split sampler on the
    force-velocity block and the same forces' translational part."""
    import torch

    from paper_1709_06946_amd import pse
    N = w['N']
    h = pse.PSE(N, w['L'], grid=w['grid'], tol=w['eps'], precision=pse.PSE_FP64,
                lanczos_tol=w['lanczos_tol'])
    x = torch.tensor(w['x'], device='cuda:0')
    F = torch.tensor(w['FL'][:, 0:3].copy(), device='cuda:0')
    for k in range(warmup):
        h.rpy_step(x, F, w['dt'], seed=seed, step=k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lz = []
    for k in range(steps):
        _, st = h.rpy_step(x, F, w['dt'], seed=seed, step=warmup + k)
        lz.append(st['lanczos_iters'])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h.close()
    return dict(value=round(N * steps / dt, 1), ms_per_step=round(1e3 * dt / steps, 3),
                lanczos_iters=lz)


STAGE_KERNELS = {
    'fft': 'fft_xy_plane_kernel (x-y transform of one z-plane, both directions)',
    'fft_large': 'fft_x_r2c/c2r_kernel and fft_lines_kernel (x and y passes)',
    'kspace': 'kspace_fused_kernel (z transform, k-space kernel, inverse z transform)',
    'spread': 'spread_list_kernel', 'interp': 'interp_kernel', 'real': 'real_pair_kernel',
}


def roofline(prof, traffic_file=None, grid=128, bracket_us=(0.0, 0.0)):
    """The stage with the largest total time: algorithmic bytes per launch over
    the average event-timed launch duration, against the HBM peak; traffic is
    the HBM bytes per launch from the committed counter summary, if it was
    taken on the current sources (else null).  The durations have the event
    time of an empty bracket (bracket_us[0]) subtracted; bracket_us[1], the
    time of a bracket around an empty kernel, is reported beside it."""
    from paper_1709_06946_amd import profsum
    dom = max(prof, key=lambda k: prof[k]['total_ms'])
    p = prof[dom]
    per_launch_bytes = p['alg_bytes'] / p['launches']
    per_launch_s = p['total_ms'] / p['launches'] / 1e3
    achieved = per_launch_bytes / per_launch_s / 1e9
    traffic = profsum.recorded_traffic(dom, traffic_file) if traffic_file else None
    return dom, dict(bound='hbm', achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit='GB/s',
                     frac=round(achieved / HBM_PEAK_GBS, 4),
                     traffic=None if traffic is None else round(traffic),
                     kernel=STAGE_KERNELS.get('fft_large' if dom == 'fft' and grid > 128
                                              else dom, dom),
                     stage=dom, launches=p['launches'],
                     avg_us=round(1e6 * per_launch_s, 2),
                     event_bracket_us=round(bracket_us[0], 2),
                     event_noop_bracket_us=round(bracket_us[1], 2),
                     alg_bytes_per_launch=round(per_launch_bytes))


def cpu_baseline():
    """The FP64 oracle's mid-point step on a bounded sample of the workload:
    N = 100 spheres at the same phi = 0.3, tolerance and dt (the dense oracle
    costs O(N^3); its particle-steps/s at N = 100 bounds it from above)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import integrator
    from paper_1709_06946_amd import inputs, pse
    N, phi, grid = 100, 0.3, 48
    x, L = inputs.packing(N, phi, seed=inputs.SEED_BASE + 50)
    d = pse.derive(pse.make_params(N, L, grid=grid, tol=1e-3))
    FL = inputs.forces_torques(N, 1)
    psi1 = inputs.real_noise(N, 2)
    psi2 = inputs.wave_noise(grid, 3)
    t0 = time.perf_counter()
    reps = 0
    while True:
        integrator.midpoint_step(x, FL, psi1, psi2, 1e-3, L, grid, d.xi, xi_total=7.0 / L)
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps >= 5:
            break
    dt = (time.perf_counter() - t0) / reps
    cores = max([i.get('num_threads', 1) for i in threadpool_info()] + [1])
    return dict(value=round(N / dt, 2), unit='particle-steps/s', cores=int(cores),
                kind='oracle',
                sample=f'{reps} oracle mid-point step(s) at N=100, phi=0.3, 48^3 k-set, '
                       f'eps=1e-3, dt=1e-3 ({dt:.2f} s per step)')


def served(n_req, steps, max_active, n_max, rate_hz, seed):
    """Served form: a Poisson stream of independent simulations with N
    log-uniform in [1e3, n_max] and phi uniform in [0.05, 0.45], each `steps`
    mixed-precision constrained steps at eps = 1e-3, admitted by device
    footprint and run concurrently.  The same requests are also run one at a
    time (no overlap) for comparison."""
    import numpy as np

    from paper_1709_06946_amd import inputs, pse
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(n_max)))))
        phi = float(rng.uniform(0.05, 0.45))
        x, L = inputs.packing(n, phi, seed=seed + 10 + i)
        reqs.append(dict(x=x, L=L, FL=inputs.forces_torques(n, seed + 5000 + i), n=n, phi=phi,
                         grid=pse.grid_for(L), seed=seed + 9000 + i))
    gaps = rng.exponential(1.0 / rate_hz, size=n_req)

    def run(active, arrivals):
        srv = pse.PSEServer(max_active=active)
        t0 = time.perf_counter()
        ids = []
        for r, g in zip(reqs, gaps):
            if arrivals:
                time.sleep(g)
            ids.append(srv.submit(r['x'], r['L'], FL=r['FL'], steps=steps, dt=1e-3,
                                  seed=r['seed'], grid=r['grid'], precision=pse.PSE_MIXED))
        lat, waits, errors = [], [], []
        for rid in ids:
            try:
                info = srv.wait(rid)
            except pse.PSEError as e:       # reported below, not fatal to the bench
                errors.append(str(e))
                srv.release(rid)
                continue
            _, l = srv.result(rid)
            lat.extend(l.tolist())
            waits.append(info['t_admit'] - info['t_submit'])
            srv.release(rid)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat = np.asarray(lat) if lat else np.full(1, np.nan)
        waits = np.asarray(waits) if waits else np.full(1, np.nan)
        return dict(particle_steps_per_s=round(st['particle_steps'] / wall, 1),
                    wall_s=round(wall, 3), p50_step_ms=round(float(np.percentile(lat, 50)), 3),
                    p99_step_ms=round(float(np.percentile(lat, 99)), 3),
                    p50_admit_wait_ms=round(1e3 * float(np.percentile(waits, 50)), 3),
                    peak_active=st['peak_active'], peak_used_GB=round(st['peak_used'] / 1e9, 3),
                    completed=st['completed'], failed=st['failed'], errors=errors[:3])

    for r in reqs[:1]:      # warm the library (code objects, tables)
        srv = pse.PSEServer(max_active=1)
        srv.wait(srv.submit(r['x'], r['L'], FL=r['FL'], steps=1, grid=r['grid'],
                            precision=pse.PSE_MIXED))
        srv.close()
    conc = run(max_active, True)
    serial = run(1, False)
    return dict(requests=n_req, steps_per_request=steps, n_range=[1000, n_max],
                phi_range=[0.05, 0.45], arrival_rate_hz=rate_hz, max_active=max_active,
                dtype='f32+f64', tol=1e-3,
                total_particles=int(sum(r['n'] for r in reqs)),
                concurrent=conc, one_at_a_time=serial)


def copy_calibration(mib=1024, reps=3):
    """A plain device copy of known size, for scaling HBM byte counters
    (FETCH_SIZE / WRITE_SIZE under rocprofv3 --pmc): each copy reads and
    writes `mib` MiB."""
    import torch
    a = torch.ones(mib * 2**20 // 8, dtype=torch.float64, device='cuda:0')
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_mib=mib, reps=reps, bytes_each_way=mib * 2**20)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=10)
    ap.add_argument('--warmup', type=int, default=2)
    ap.add_argument('--workload', default='n10000_phi0.3_g128')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-mixed', action='store_true')
    ap.add_argument('--no-served', action='store_true')
    ap.add_argument('--no-rpy', action='store_true')
    ap.add_argument('--deriv-gridding', type=int, default=0,
                    help='gridding of the constraint operator: 0 library default, '
                         '1 moments, 2 derivative')
    ap.add_argument('--copy-calibration', action='store_true',
                    help='only run a 1 GiB device copy (counter calibration)')
    ap.add_argument('--served-requests', type=int, default=16)
    ap.add_argument('--served-steps', type=int, default=20)
    ap.add_argument('--served-nmax', type=int, default=20000)
    ap.add_argument('--served-active', type=int, default=4)
    ap.add_argument('--served-rate', type=float, default=40.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f'bench.py runs on one GPU only (--gpus {args.gpus} requested): the method '
              'here is the single-GPU hot path; see the sharding notes in DESIGN.md.',
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    from paper_1709_06946_amd import inputs, pse
    w = inputs.workload(args.workload)
    seed = w['seed']
    fp64 = run_form(w, pse.PSE_FP64, args.steps, args.warmup, seed,
                    deriv_gridding=args.deriv_gridding)
    traffic_file = os.path.join(ROOT, 'profiles', f'hbm_traffic_{args.workload}_fp64.md')
    dom, roof = roofline(fp64['prof'], traffic_file, w['grid'], fp64['bracket_us'])
    mixed = None
    if not args.no_mixed:
        m = run_form(w, pse.PSE_MIXED, args.steps, args.warmup, seed,
                     deriv_gridding=args.deriv_gridding)
        mdom, mroof = roofline(m['prof'], None, w['grid'], m['bracket_us'])
        mixed = dict(value=round(m['value'], 1), ms_per_step=round(m['ms_per_step'], 3),
                     speedup_vs_fp64=round(m['value'] / fp64['value'], 3), dtype='f32+f64',
                     roofline=mroof,
                     gmres_iters=[s['gmres_iters'] for s in m['stats']],
                     fp64_residual=[s['fp64_residual'] for s in m['stats']])
    gm = [s['gmres_iters'] for s in fp64['stats']]
    lz = [s['lanczos_iters'] for s in fp64['stats']]
    out = dict(
        metric=METRIC, value=round(fp64['value'], 1), unit='particle-steps/s', n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=round(fp64['ms_per_step'], 3),
        higher_is_better=True, scaling='weak', vs_baseline=None, dtype='f64',
        data='synthetic',
        config=dict(workload=args.workload, N=w['N'], phi=w['phi'], L=round(w['L'], 4),
                    grid=w['grid'], tol=w['eps'], dt=w['dt'], gmres_tol=w['gmres_tol'],
                    lanczos_tol=w['lanczos_tol'],
                    derived={k: v for k, v in fp64['derived'].items()}),
        roofline=roof,
        krylov=dict(lanczos_iters=lz, gmres_iters=gm),
        stages_ms={k: round(v['total_ms'] / fp64['prof_steps'], 3)
                   for k, v in fp64['prof'].items()},
        mixed=mixed,
    )
    if not args.no_rpy:
        r = run_rpy(w, args.steps, args.warmup, seed)
        r['fts_over_rpy'] = round(r['value'] / fp64['value'], 2)
        out['rpy'] = r
    if not args.no_served:
        out['served'] = served(args.served_requests, args.served_steps, args.served_active,
                               args.served_nmax, args.served_rate, seed + 777)
    if not args.no_cpu_baseline:
        out['cpu_baseline'] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
