"""Seeded synthetic inputs: hard-sphere packings, forces/torques and noise.

This module holds no part of the method's arithmetic; it only draws inputs.
Both the tests (oracle side and library side) and the benchmark take their
inputs from here, so the two sides always see identical arrays.

The packings stand in for the random hard-sphere suspensions the paper
measures on (Sec. IV, phi = 0.1 - 0.5): non-overlapping spheres of radius a
placed uniformly at random in a periodic cube by random sequential addition
(candidates drawn in batches; a candidate is rejected if it overlaps a placed
sphere or an earlier candidate of its batch).
"""
import numpy as np

SEED_BASE = 1709069460

# Workloads: sphere count, volume fraction, grid, tolerance, time step.
WORKLOADS = {
    'n100_phi0.1_g32': dict(N=100, phi=0.1, grid=32, eps=1e-3, dt=1e-3,
                            gmres_tol=1e-6, lanczos_tol=1e-3, index=0),
    'n100_phi0.01_g32': dict(N=100, phi=0.01, grid=32, eps=1e-3, dt=1e-3,
                             gmres_tol=1e-6, lanczos_tol=1e-3, index=0),
    'n10000_phi0.3_g128': dict(N=10_000, phi=0.3, grid=128, eps=1e-3, dt=1e-3,
                               gmres_tol=1e-6, lanczos_tol=1e-3, index=1),
    'n1000000_phi0.1_g512': dict(N=1_000_000, phi=0.1, grid=512, eps=1e-3,
                                 dt=1e-3, gmres_tol=1e-4, lanczos_tol=1e-3,
                                 index=2),
}
# the dense suspension over its tolerance sweep (eps, grid)
for _eps, _g in ((1e-2, 128), (1e-3, 192), (1e-4, 256), (1e-5, 384)):
    WORKLOADS[f'n200000_phi0.45_g{_g}'] = dict(N=200_000, phi=0.45, grid=_g, eps=_eps,
                                               dt=1e-3, gmres_tol=1e-4, lanczos_tol=1e-3,
                                               index=3)


def box_length(N, phi, a=1.0):
    """Side of the periodic cube holding N spheres of radius a at fraction phi."""
    return (N * 4.0 / 3.0 * np.pi * a**3 / phi) ** (1.0 / 3.0)


def rsa_packing(N, phi, a=1.0, seed=SEED_BASE, batch=None):
    """(positions (N, 3) in [0, L)^3, L) of N non-overlapping spheres."""
    L = box_length(N, phi, a)
    rng = np.random.default_rng(seed)
    nc = max(1, int(np.floor(L / (2.0 * a))))
    cs = L / nc
    cap = 16
    cells = np.full((nc, nc, nc, cap), -1, dtype=np.int64)
    count = np.zeros((nc, nc, nc), dtype=np.int64)
    x = np.empty((N, 3))
    n = 0
    d2min = (2.0 * a) ** 2
    offs = np.stack(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1],
                                indexing='ij'), -1).reshape(-1, 3)
    if batch is None:
        batch = max(64, min(N // 20, nc**3 // 8))
    tries = 0

    def neighbours(table, ci):
        nb = (ci[:, None, :] + offs[None, :, :]) % nc                # (B,27,3)
        return table[nb[..., 0], nb[..., 1], nb[..., 2]]             # (B,27,cap)

    while n < N:
        tries += 1
        if tries > 100000:
            raise RuntimeError('random sequential addition did not converge')
        B = batch
        c = rng.uniform(0.0, L, (B, 3))
        ci = np.minimum((c / cs).astype(np.int64), nc - 1)
        # overlap with placed spheres
        occ = neighbours(cells, ci)
        valid = occ >= 0
        d = c[:, None, None, :] - x[np.where(valid, occ, 0)]
        d -= L * np.rint(d / L)
        bad = (valid & ((d**2).sum(-1) < d2min)).any(axis=(1, 2))
        # overlap with earlier candidates of the same batch (cell hash)
        flat = (ci[:, 0] * nc + ci[:, 1]) * nc + ci[:, 2]
        order = np.argsort(flat, kind='stable')
        fs = flat[order]
        start = np.searchsorted(fs, fs, side='left')
        rank = np.arange(B) - start
        capb = int(rank.max()) + 1
        tb = np.full((nc, nc, nc, capb), -1, dtype=np.int64)
        tb.reshape(-1, capb)[fs, rank] = order
        occ = neighbours(tb, ci)
        valid = (occ >= 0) & (occ < np.arange(B)[:, None, None])
        d = c[:, None, None, :] - c[np.where(valid, occ, 0)]
        d -= L * np.rint(d / L)
        bad |= (valid & ((d**2).sum(-1) < d2min)).any(axis=(1, 2))
        ok = np.nonzero(~bad)[0][:N - n]
        for j in ok:
            cx, cy, cz = ci[j]
            if count[cx, cy, cz] >= cap:
                raise RuntimeError('cell capacity exceeded')
            cells[cx, cy, cz, count[cx, cy, cz]] = n
            count[cx, cy, cz] += 1
            x[n] = c[j]
            n += 1
    return x, L


def relaxed_packing(N, phi, a=1.0, seed=SEED_BASE, margin=1e-3,
                    max_iter=20000):
    """(positions, L) of N non-overlapping spheres at a dense fraction.

    Centres are drawn uniformly at random and overlapping pairs are then
    pushed apart along their line of centres (each by half the overlap, plus
    a relative margin) until no pair is closer than 2a.  Used where random
    sequential addition is impractically slow (phi above ~0.2)."""
    L = box_length(N, phi, a)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, L, (N, 3))
    nc = max(1, int(np.floor(L / (2.0 * a))))
    cs = L / nc
    target = 2.0 * a * (1.0 + margin)
    offs = np.stack(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1],
                                indexing='ij'), -1).reshape(-1, 3)
    for it in range(max_iter):
        ci = np.minimum((x / cs).astype(np.int64), nc - 1)
        flat = (ci[:, 0] * nc + ci[:, 1]) * nc + ci[:, 2]
        order = np.argsort(flat, kind='stable')
        fs = flat[order]
        start = np.searchsorted(fs, fs, side='left')
        rank = np.arange(N) - start
        cap = int(rank.max()) + 1
        table = np.full((nc**3, cap), -1, dtype=np.int64)
        table[fs, rank] = order
        table = table.reshape(nc, nc, nc, cap)
        moved = np.zeros_like(x)
        for s0 in range(0, N, 65536):
            idx = np.arange(s0, min(N, s0 + 65536))
            nb = (ci[idx, None, :] + offs[None]) % nc
            occ = table[nb[..., 0], nb[..., 1], nb[..., 2]].reshape(idx.size, -1)
            occ = np.where(occ > idx[:, None], occ, -1)    # each pair once
            i_, j_ = np.nonzero(occ >= 0)
            pi, pj = idx[i_], occ[i_, j_]
            if pi.size == 0:
                continue
            pair = np.unique(pi * N + pj)
            pi, pj = pair // N, pair % N
            d = x[pi] - x[pj]
            d -= L * np.rint(d / L)
            r = np.sqrt((d**2).sum(1))
            m = r < 2.0 * a
            if not m.any():
                continue
            pi, pj, d, r = pi[m], pj[m], d[m], r[m]
            u = d / np.maximum(r, 1e-12)[:, None]
            push = 0.5 * (target - r)[:, None] * u
            np.add.at(moved, pi, push)
            np.add.at(moved, pj, -push)
        if not moved.any():
            return x, L
        x = (x + moved) % L
    raise RuntimeError('overlap relaxation did not converge')


LATTICE_N = 200_000   # from this size on, packings are jittered lattices


def jittered_lattice(N, phi, a=1.0, seed=SEED_BASE):
    """Non-overlapping spheres for very large N: N distinct random sites of
    the m^3 cubic lattice (m = ceil(N^(1/3))) of the box, each displaced
    uniformly by at most half the gap (spacing - 2a) per axis, so that no
    two spheres overlap; the volume fraction is exactly phi.  Needs a lattice
    spacing above 2a (phi below about 0.47)."""
    L = box_length(N, phi, a)
    m = int(np.ceil(N ** (1.0 / 3.0) - 1e-9))
    s = L / m
    if s <= 2.0 * a:
        raise ValueError('volume fraction too high for a jittered lattice')
    rng = np.random.default_rng(seed)
    sites = rng.choice(m**3, size=N, replace=False)
    ijk = np.stack([sites % m, (sites // m) % m, sites // (m * m)], axis=1)
    half_gap = 0.5 * (s - 2.0 * a) * (1.0 - 1e-9)
    x = (ijk + 0.5) * s + rng.uniform(-half_gap, half_gap, size=(N, 3))
    return np.mod(x, L), L


def packing(N, phi, a=1.0, seed=SEED_BASE):
    """Random non-overlapping packing: sequential addition for dilute
    suspensions, overlap relaxation for dense ones, a jittered lattice from
    LATTICE_N spheres on (sequential addition is too slow there)."""
    if N >= LATTICE_N:
        return jittered_lattice(N, phi, a, seed)
    if phi <= 0.2:
        return rsa_packing(N, phi, a, seed)
    return relaxed_packing(N, phi, a, seed)


def forces_torques(N, seed):
    """F and L per particle, i.i.d. N(0, 1) per component: (N, 6)."""
    return np.random.default_rng(seed).normal(size=(N, 6))


def real_noise(N, seed):
    """psi1 for the real-space sampler, i.i.d. N(0, 1): (N, 11)."""
    return np.random.default_rng(seed).normal(size=(N, 11))


def wave_noise(Ng, seed):
    """Complex wave noise (3, Ng, Ng, Ng//2 + 1); real and imaginary parts
    i.i.d. N(0, 1/2).  Only the canonical half space is read by consumers."""
    rng = np.random.default_rng(seed)
    shape = (3, Ng, Ng, Ng // 2 + 1)
    s = np.sqrt(0.5)
    return (rng.normal(scale=s, size=shape)
            + 1j * rng.normal(scale=s, size=shape))


def workload(name, seed_offset=0):
    """Positions, box, forces and noise of a named workload."""
    w = dict(WORKLOADS[name])
    base = SEED_BASE + w['index'] + seed_offset
    x, L = packing(w['N'], w['phi'], seed=base)
    w.update(name=name, x=x, L=L, FL=forces_torques(w['N'], base + 1),
             seed=base + 2)
    return w
