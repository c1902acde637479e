"""Benchmark: stresslet-constrained PSE Brownian dynamics steps on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One "step" is one full mid-point step of the method (Sec. III.D): Lanczos
M_r^(1/2), wave-space M_w^(1/2), half step, GMRES on the stresslet
constraint, final mobility product and position update.  The default workload
is N = 10^6 hard spheres (a = 1) at phi = 0.1 in a 512^3 grid, eps = 1e-3,
Lanczos to 1e-3, GMRES to 1e-4 with FP64 residual refinement, in the mixed
precision form (FP32 grids, FFTs, k-space, gridding and pair sums; FP64
Krylov scalars, positions and residual), with random non-overlapping
positions and N(0, 1) forces/torques.  Beside the headline: the plain FP64
form on the same workload and the difference of the two forms' velocities
from the same state and noise, the N = 10^4, phi = 0.3, 128^3 workload in
both forms, the RPY-level comparison system (forces only, no constraint) and
its cost ratio, the served form (a Poisson stream of independent simulations
of different N and phi with p50/p99 per-step latency), and the FP64 oracle on
host cores.  Prints one JSON line.
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


def make_handle(w, precision, deriv_gridding=0):
    from paper_1709_06946_amd import pse
    return pse.PSE(w['N'], w['L'], grid=w['grid'], tol=w['eps'], precision=precision,
                   lanczos_tol=w['lanczos_tol'], gmres_tol=w['gmres_tol'],
                   deriv_gridding=deriv_gridding)


def run_form(w, precision, steps, warmup, seed, prof_steps=2, deriv_gridding=0):
    """Times `steps` steps with the stage profiler off (the throughput), then
    runs `prof_steps` more with it on (stage times, launch durations)."""
    import torch

    N = w['N']
    h = make_handle(w, precision, deriv_gridding)
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
        print(f'# {w["name"]} precision={precision} step {k} lanczos={st["lanczos_iters"]} '
              f'gmres={st["gmres_iters"]} res={st["fp64_residual"]:.2e}', file=sys.stderr,
              flush=True)
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


def run_graph(w, precision, steps, warmup, seed):
    """The same steps as replays of one captured graph of the whole step: a
    synchronous first step gives the Krylov iteration counts, the handle is
    switched to device-checked solves with those counts plus a margin, and
    one captured step is replayed per step (one host launch per step)."""
    import torch
    N = w['N']
    h = make_handle(w, precision)
    x = torch.tensor(w['x'], device='cuda:0')
    FL = torch.tensor(w['FL'], device='cuda:0')
    _, st = h.constrained_step(x, FL, w['dt'], seed=seed, step=0)
    passes = max(1, st['refine_passes'])
    caps = (st['lanczos_iters'] + 1, st['gmres_iters'] // passes + 3, passes)
    h.set_krylov(1, *caps, next_step=1)
    g = h.step_graph(x, FL, w['dt'], seed=seed, steps=1)
    for _ in range(warmup):
        g.launch()
    h.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.launch()
    h.synchronize()
    dt = time.perf_counter() - t0
    last = h.stats()
    g.close()
    h.close()
    return dict(value=round(N * steps / dt, 1), ms_per_step=round(1e3 * dt / steps, 3),
                caps=dict(lanczos=caps[0], gmres=caps[1], refine_passes=caps[2]),
                last_step=dict(converged=last['converged'], status=last['status'],
                               gmres_iters=last['gmres_iters'],
                               fp64_residual=last['fp64_residual']))


def form_difference(w, seed, deriv_gridding=0):
    """Velocity of one constrained step from the workload's initial positions
    with the same noise (internal Philox stream, same seed and step) in the
    FP64 and the mixed form: the relative difference of the velocities and of
    the stresslets isolates the precision effect at this size."""
    import torch

    from paper_1709_06946_amd import pse
    out = {}
    for prec in (pse.PSE_FP64, pse.PSE_MIXED):
        h = make_handle(w, prec, deriv_gridding)
        x = torch.tensor(w['x'], device='cuda:0')
        FL = torch.tensor(w['FL'], device='cuda:0')
        U = torch.empty((w['N'], 3), dtype=torch.float64, device='cuda:0')
        S = torch.empty((w['N'], 5), dtype=torch.float64, device='cuda:0')
        h.constrained_step(x, FL, w['dt'], seed=seed, step=10**6, velocity=U, stresslet=S)
        torch.cuda.synchronize()
        out[prec] = (U.cpu(), S.cpu())
        h.close()
        del x, FL, U, S
    (u64, s64), (u32, s32) = out[pse.PSE_FP64], out[pse.PSE_MIXED]
    return dict(velocity_rel_diff=float((u32 - u64).norm() / u64.norm()),
                stresslet_rel_diff=float((s32 - s64).norm() / s64.norm()))


def run_rpy(w, precision, steps, warmup, seed):
    """The RPY-level comparison system (forces only, Sec. IV) on the same
    workload: Euler-Maruyama steps with the split sampler on the
    force-velocity block and the same forces' translational part."""
    import torch

    from paper_1709_06946_amd import pse
    N = w['N']
    h = pse.PSE(N, w['L'], grid=w['grid'], tol=w['eps'], precision=precision,
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


# Kernels of each stage of the library's stage profiler.
STAGE_KERNELS = {
    'fft': 'fft_xy_plane_kernel (x-y transform of one z-plane, both directions)',
    'fft_large': 'fft_x_r2c/c2r_kernel and fft_lines_kernel (x and y passes)',
    'kspace': 'kspace_fused_kernel (z transform, k-space kernel, inverse z transform)',
    'spread': 'spread_list_kernel and spread_deriv_kernel',
    'interp': 'interp_kernel and interp_deriv_kernel', 'real': 'real_pair_kernel',
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


def stage_fracs(prof):
    """Per stage: algorithmic bytes over event-timed duration, as a fraction
    of the HBM peak, and the stage's total time per profiled run."""
    out = {}
    for k, p in prof.items():
        if p['total_ms'] <= 0 or p['alg_bytes'] <= 0:
            continue
        gbs = p['alg_bytes'] / (p['total_ms'] / 1e3) / 1e9
        out[k] = dict(total_ms=round(p['total_ms'], 3), launches=p['launches'],
                      achieved_GBs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


def host_cpu():
    """CPU model and logical core count of the host."""
    model = 'unknown'
    try:
        with open('/proc/cpuinfo') as fh:
            for line in fh:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(phi):
    """The FP64 oracle's mid-point step on a bounded sample of the workload:
    N = 100 spheres at the workload's volume fraction, tolerance and dt, on
    the 32^3 k-set of that box (the dense oracle costs O(N^3); its
    particle-steps/s at N = 100 bounds it from above)."""
    from threadpoolctl import threadpool_info

    from oracle import integrator
    from paper_1709_06946_amd import inputs, pse
    N, grid = 100, 32
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
        if time.perf_counter() - t0 > 15.0 or reps >= 8:
            break
    dt = (time.perf_counter() - t0) / reps
    cores = max([i.get('num_threads', 1) for i in threadpool_info()] + [1])
    model, nproc = host_cpu()
    return dict(value=round(N / dt, 2), unit='particle-steps/s', cores=int(cores),
                kind='oracle', cpu_model=model, nproc=nproc,
                sample=f'{reps} oracle mid-point step(s) at N=100, phi={phi}, L={L:.2f}, '
                       f'32^3 k-set, eps=1e-3, dt=1e-3 ({dt:.2f} s per step)')


def _make_request(args):
    """One served request's inputs (run in a worker process)."""
    i, n, phi, seed = args
    from paper_1709_06946_amd import inputs, pse
    x, L = inputs.packing(n, phi, seed=seed + 10 + i)
    return dict(x=x, L=L, FL=inputs.forces_torques(n, seed + 5000 + i), n=n, phi=phi,
                grid=pse.grid_for(L), seed=seed + 9000 + i)


def served(n_req, steps, max_active, n_max, rate_frac, seed, workers=8):
    """Served form: a Poisson stream of independent simulations with N
    log-uniform in [1e3, n_max] and phi uniform in [0.05, 0.45], each `steps`
    mixed-precision constrained steps at eps = 1e-3, admitted by device
    footprint and run concurrently.  The same requests are run one at a time
    and all submitted at once (no arrival gaps) with and without overlap: the
    overlapped run's rate is the capacity, and the Poisson arrival rate of the
    latency run is rate_frac times it.  Inputs are generated before any run."""
    import concurrent.futures

    import numpy as np

    from paper_1709_06946_amd import pse
    rng = np.random.default_rng(seed)
    spec = []
    for i in range(n_req):
        n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(n_max)))))
        spec.append((i, n, float(rng.uniform(0.05, 0.45)), seed))
    gaps01 = rng.exponential(1.0, size=n_req)
    t0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers) as ex:
        reqs = list(ex.map(_make_request, spec))
    t_inputs = time.perf_counter() - t0

    def run(active, gaps):
        srv = pse.PSEServer(max_active=active)
        t0 = time.perf_counter()
        ids = []
        for r, g in zip(reqs, gaps):
            if g > 0:
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
    serial = run(1, np.zeros(n_req))
    saturated = run(max_active, np.zeros(n_req))
    capacity = n_req / saturated['wall_s']
    rate = rate_frac * capacity
    conc = run(max_active, gaps01 / rate)
    return dict(requests=n_req, steps_per_request=steps, n_range=[1000, n_max],
                phi_range=[0.05, 0.45], dtype='f32+f64', tol=1e-3, max_active=max_active,
                capacity_req_per_s=round(capacity, 3), arrival_rate_req_per_s=round(rate, 3),
                arrival_rate_frac_of_capacity=rate_frac,
                total_particles=int(sum(r['n'] for r in reqs)),
                input_generation_s=round(t_inputs, 1),
                concurrent=conc, concurrent_all_at_once=saturated, one_at_a_time=serial)


def copy_rate_gbs(mib=1024, reps=20):
    """Read + write rate of a plain 1 GiB device copy (torch copy_, events on
    the current stream): the streaming rate HBM gives a kernel that reads and
    writes every byte once, beside the published peak."""
    import torch
    a = torch.ones(mib * 2**20 // 4, dtype=torch.float32, device='cuda:0')
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * mib * 2**20 / (ms * 1e-3) / 1e9


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


FORM_NAME = {0: 'fp64', 1: 'mixed'}
FORM_DTYPE = {0: 'f64', 1: 'f32+f64'}


def form_summary(r, other=None):
    out = dict(value=round(r['value'], 1), ms_per_step=round(r['ms_per_step'], 3),
               gmres_iters=[s['gmres_iters'] for s in r['stats']],
               lanczos_iters=[s['lanczos_iters'] for s in r['stats']],
               fp64_residual=[s['fp64_residual'] for s in r['stats']])
    if other is not None:
        out['speedup_vs_other'] = round(r['value'] / other['value'], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=10)
    ap.add_argument('--warmup', type=int, default=2)
    ap.add_argument('--workload', default='n1000000_phi0.1_g512')
    ap.add_argument('--secondary', default='n10000_phi0.3_g128',
                    help='second workload run in both forms ("" to skip)')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-other-form', action='store_true',
                    help='skip the second precision form of the headline workload')
    ap.add_argument('--no-served', action='store_true')
    ap.add_argument('--no-rpy', action='store_true')
    ap.add_argument('--deriv-gridding', type=int, default=0,
                    help='gridding of the constraint operator: 0 library default, '
                         '1 moments, 2 derivative')
    ap.add_argument('--copy-calibration', action='store_true',
                    help='only run a 1 GiB device copy (counter calibration)')
    ap.add_argument('--served-requests', type=int, default=24)
    ap.add_argument('--served-steps', type=int, default=20)
    ap.add_argument('--served-nmax', type=int, default=200000)
    ap.add_argument('--served-active', type=int, default=4)
    ap.add_argument('--served-rate-frac', type=float, default=0.75)
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
    prec = w['precision']
    other_prec = pse.PSE_FP64 if prec == pse.PSE_MIXED else pse.PSE_MIXED
    head = run_form(w, prec, args.steps, args.warmup, seed,
                    deriv_gridding=args.deriv_gridding)
    traffic_file = os.path.join(ROOT, 'profiles',
                                f'hbm_traffic_{args.workload}_{FORM_NAME[prec]}.md')
    dom, roof = roofline(head['prof'], traffic_file, w['grid'], head['bracket_us'])
    # context for the HBM fraction: what a plain device copy reaches here
    roof['copy_GBs'] = round(copy_rate_gbs(), 1)
    roof['frac_of_copy'] = round(roof['achieved'] / roof['copy_GBs'], 4)
    out = dict(
        metric=METRIC, value=round(head['value'], 1), unit='particle-steps/s', n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=round(head['ms_per_step'], 3),
        higher_is_better=True, scaling='weak', vs_baseline=None, dtype=FORM_DTYPE[prec],
        data='synthetic',
        config=dict(workload=args.workload, N=w['N'], phi=w['phi'], L=round(w['L'], 4),
                    grid=w['grid'], tol=w['eps'], dt=w['dt'], gmres_tol=w['gmres_tol'],
                    lanczos_tol=w['lanczos_tol'], form=FORM_NAME[prec],
                    derived={k: v for k, v in head['derived'].items()}),
        roofline=roof,
        krylov=dict(lanczos_iters=[s['lanczos_iters'] for s in head['stats']],
                    gmres_iters=[s['gmres_iters'] for s in head['stats']],
                    fp64_residual=[s['fp64_residual'] for s in head['stats']]),
        stages_ms={k: round(v['total_ms'] / head['prof_steps'], 3)
                   for k, v in head['prof'].items()},
        stage_hbm=stage_fracs(head['prof']),
    )
    if not args.no_other_form:
        o = run_form(w, other_prec, args.steps, args.warmup, seed,
                     deriv_gridding=args.deriv_gridding)
        _, oroof = roofline(o['prof'], None, w['grid'], o['bracket_us'])
        s = form_summary(o, head)
        s.update(dtype=FORM_DTYPE[other_prec], roofline=oroof)
        out[FORM_NAME[other_prec]] = s
        out['form_difference'] = form_difference(w, seed, args.deriv_gridding)
    if args.secondary:
        w2 = inputs.workload(args.secondary)
        sec = dict(workload=args.secondary, N=w2['N'], phi=w2['phi'], grid=w2['grid'])
        r64 = run_form(w2, pse.PSE_FP64, args.steps, args.warmup, w2['seed'])
        r32 = run_form(w2, pse.PSE_MIXED, args.steps, args.warmup, w2['seed'])
        sec['fp64'] = form_summary(r64)
        sec['mixed'] = form_summary(r32, r64)
        g64 = run_graph(w2, pse.PSE_FP64, args.steps, args.warmup, w2['seed'])
        g64['speedup_vs_eager'] = round(g64['value'] / r64['value'], 3)
        g32 = run_graph(w2, pse.PSE_MIXED, args.steps, args.warmup, w2['seed'])
        g32['speedup_vs_eager'] = round(g32['value'] / r32['value'], 3)
        sec['graph'] = dict(fp64=g64, mixed=g32)
        traffic2 = os.path.join(ROOT, 'profiles',
                                f'hbm_traffic_{args.secondary}_{FORM_NAME[0]}.md')
        _, sec['fp64']['roofline'] = roofline(r64['prof'], traffic2, w2['grid'],
                                              r64['bracket_us'])
        out['secondary'] = sec
    if not args.no_rpy:
        r = run_rpy(w, prec, args.steps, args.warmup, seed)
        r['fts_over_rpy'] = round(r['value'] / head['value'], 2)
        r['dtype'] = FORM_DTYPE[prec]
        out['rpy'] = r
    if not args.no_served:
        out['served'] = served(args.served_requests, args.served_steps, args.served_active,
                               args.served_nmax, args.served_rate_frac, seed + 777)
    if not args.no_cpu_baseline:
        out['cpu_baseline'] = cpu_baseline(w['phi'])
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
