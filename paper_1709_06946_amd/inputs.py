"""Seeded synthetic inputs: hard-sphere packings, forces/torques and noise.

This module holds no part of the method's arithmetic; it only draws inputs.
Both the tests (oracle side and library side) and the benchmark take their
inputs from here, so the two sides always see identical arrays.

The packings stand in for the random hard-sphere suspensions the paper
measures on (Sec. IV, phi = 0.1 - 0.5): non-overlapping spheres of radius a
placed uniformly at random in a periodic cube.  Below CPACK_N spheres, random
sequential addition in numpy (candidates drawn in batches; a candidate is
rejected if it overlaps a placed sphere or an earlier candidate of its batch)
for phi <= 0.2, overlap relaxation of uniform centres above.  From CPACK_N
on, the compiled generator (packing.c): random sequential addition for
phi <= 0.3; above, sequential addition at the reduced radius that gives
phi = 0.3, compression to the target fraction and hard-sphere Monte Carlo
sweeps.
"""
import numpy as np

SEED_BASE = 1709069460

# Workloads: sphere count, volume fraction, grid, tolerance, time step and
# the precision form they are run in (0 FP64, 1 mixed).
WORKLOADS = {
    'n100_phi0.1_g32': dict(N=100, phi=0.1, grid=32, eps=1e-3, dt=1e-3,
                            gmres_tol=1e-6, lanczos_tol=1e-3, index=0, precision=0),
    'n100_phi0.01_g32': dict(N=100, phi=0.01, grid=32, eps=1e-3, dt=1e-3,
                             gmres_tol=1e-6, lanczos_tol=1e-3, index=0, precision=0),
    'n10000_phi0.3_g128': dict(N=10_000, phi=0.3, grid=128, eps=1e-3, dt=1e-3,
                               gmres_tol=1e-6, lanczos_tol=1e-3, index=1, precision=0),
    'n1000000_phi0.1_g512': dict(N=1_000_000, phi=0.1, grid=512, eps=1e-3,
                                 dt=1e-3, gmres_tol=1e-4, lanczos_tol=1e-3,
                                 index=2, precision=1),
}
# the dense suspension over its tolerance sweep (eps, grid)
for _eps, _g in ((1e-2, 128), (1e-3, 192), (1e-4, 256), (1e-5, 384)):
    WORKLOADS[f'n200000_phi0.45_g{_g}'] = dict(N=200_000, phi=0.45, grid=_g, eps=_eps,
                                               dt=1e-3, gmres_tol=1e-4, lanczos_tol=1e-3,
                                               index=3, precision=1)


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


# From this size on, packings come from the compiled generator (packing.c):
# random sequential addition up to phi = 0.3, and above it sequential
# addition at the radius that gives phi = 0.3 followed by compression (radius
# set to a, overlapping pairs pushed apart until none is left).
CPACK_N = 2000
RSA_PHI_MAX = 0.3

_pack_lib = None


def _packing_lib():
    global _pack_lib
    if _pack_lib is None:
        import ctypes
        import os
        from . import build
        if not os.path.exists(build.PACK_LIB):
            build.build_packing()
        lib = ctypes.CDLL(build.PACK_LIB)
        lib.pack_rsa.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_uint64, ctypes.c_void_p]
        lib.pack_compressed.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p]
        _pack_lib = lib
    return _pack_lib


def compiled_packing(N, phi, a=1.0, seed=SEED_BASE):
    """(positions, L): random sequential addition (phi <= 0.3) or sequential
    addition at phi = 0.3 then compression to phi, by the compiled
    generator."""
    L = box_length(N, phi, a)
    x = np.empty((N, 3))
    lib = _packing_lib()
    if phi <= RSA_PHI_MAX:
        rc = lib.pack_rsa(N, L, a, seed % 2**64, x.ctypes.data)
    else:
        rc = lib.pack_compressed(N, L, a, RSA_PHI_MAX, seed % 2**64, x.ctypes.data)
    if rc != 0:
        raise RuntimeError(f'packing generator failed ({rc}) at N={N}, phi={phi}')
    return x, L


def packing(N, phi, a=1.0, seed=SEED_BASE):
    """Random non-overlapping packing: for small N sequential addition for
    dilute suspensions and overlap relaxation for dense ones; from CPACK_N
    spheres on, the compiled generator."""
    if N >= CPACK_N:
        return compiled_packing(N, phi, a, seed)
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
