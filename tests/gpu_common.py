"""Shared helpers of the GPU tests (inputs, error norms, oracle caching)."""
import functools

import numpy as np

from paper_1709_06946_amd import inputs

BLOCKS = {'U': slice(0, 3), 'Omega': slice(3, 6), 'E': slice(6, 11)}


def rel_err(y, ref):
    y, ref = np.asarray(y), np.asarray(ref)
    d = np.linalg.norm(ref)
    return np.linalg.norm(y - ref) / (d if d > 0 else 1.0)


def block_errors(y, ref):
    return {k: rel_err(np.asarray(y)[:, s], np.asarray(ref)[:, s]) for k, s in BLOCKS.items()}


@functools.lru_cache(maxsize=None)
def packing(N, phi, seed):
    x, L = inputs.packing(N, phi, seed=seed)
    return x, L


def dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to('cuda:0')


def host(t):
    return t.detach().cpu().numpy()
