"""Seeded synthetic inputs for the decoder: seeds, noise strengths, lattice sizes.

This module holds no decoder arithmetic: it only produces the seeds and
parameters that both the GPU path and the CPU oracle consume.  The workloads
mirror the paper's numerics (Sec. 7): i.i.d. bit-flip noise of strength p on
every link of an L x L periodic lattice, decoded with v = 3.

Seed recipe: seed_i = (config_id << 40) | (p_index << 32) | i.
"""
from __future__ import annotations

import numpy as np

T_MAX_DEFAULT = 4096


def seeds(config_id: int, p_index: int, n: int, start: int = 0) -> np.ndarray:
    """uint64 seeds (config_id << 40) | (p_index << 32) | i for i in [start, start+n)."""
    i = np.arange(start, start + n, dtype=np.uint64)
    return (np.uint64(config_id) << np.uint64(40)) | (np.uint64(p_index) << np.uint64(32)) | i


# The five workloads: L = lattice size, p = noise strength(s), n = samples.
CONFIGS = {
    1: dict(name="toric L=16 p=0.01", L=16, p=[0.01], n=1000, T_max=4096),
    2: dict(name="toric L=64 p in {0.005,0.01,0.02}", L=64, p=[0.005, 0.01, 0.02], n=10000,
            T_max=4096),
    3: dict(name="toric L=256 p=0.01", L=256, p=[0.01], n=4096, T_max=4096),
    4: dict(name="mixed L in {32..512}, p~U[0.001,0.03]", L=[32, 64, 128, 256, 512],
            n=[256, 64, 16, 4, 1], p_range=(0.001, 0.03), T_max=4096),
    5: dict(name="learned scheduling L=256/1024 p=0.01", L=[256, 1024], p=[0.01], n=[4096, 1024],
            train_n=200000, train_p=(0.005, 0.02), T_max=4096),
}


def mixed_batch(config_id: int = 4, rng_seed: int = 4):
    """Mixed-size batch: per-class counts proportional to 1/L^2 (262144 sites per
    class) and p_i ~ U[0.001, 0.03] from numpy PCG64(rng_seed).

    Returns (L int32[n], p float64[n], seeds uint64[n]) in class order.
    """
    cfg = CONFIGS[config_id]
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    Ls, ps, ss = [], [], []
    for k, (L, n) in enumerate(zip(cfg["L"], cfg["n"])):
        Ls.append(np.full(n, L, dtype=np.int32))
        ps.append(rng.uniform(cfg["p_range"][0], cfg["p_range"][1], size=n))
        ss.append(seeds(config_id, k, n))
    return np.concatenate(Ls), np.concatenate(ps), np.concatenate(ss)
