"""Seeded synthetic inputs for LR-QAOA simulation runs.

This module only draws inputs: complete-graph edge weights and the per-run
settings (qubit count, depth, ramp slopes, shot count, seeds).  It holds none
of the simulation arithmetic, so both the GPU path and the oracle may use it.

The paper (arXiv:2604.26423, Sec. II-G) builds one weighted complete graph
per size with weights uniform on [0, 1] and publishes its instances
externally.  Those are not available here, so these seeded instances stand in
for them: weights are i.i.d. uniform on {0.1, 0.2, ..., 1.0}, stored as
integers in tenths (1..10) so the cut value of every basis state is an exact
integer.  Edges are listed in lexicographic order (0,1), (0,2), ..., (n-2,n-1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


def n_edges(n: int) -> int:
    return n * (n - 1) // 2


def complete_graph_tenths(n: int, seed: int) -> np.ndarray:
    """Edge weights of K_n in tenths, i.i.d. uniform on 1..10, lexicographic."""
    rng = np.random.default_rng(seed)
    return rng.integers(1, 11, size=n_edges(n), dtype=np.int32)


@dataclass(frozen=True)
class Run:
    """One simulation run: instance, depth and ramp slopes, shots."""
    name: str
    n: int
    seed: int
    p: int
    delta_gamma: float
    delta_beta: float
    shots: int = 0
    precision: str = "c64"

    def weights(self) -> np.ndarray:
        return complete_graph_tenths(self.n, self.seed)


# The five workload families.  Shot seeds equal the instance seed.
SMALL = Run("K12_p3", n=12, seed=0, p=3, delta_gamma=0.6, delta_beta=0.6, shots=1000,
            precision="c128")
MEDIUM = Run("K26_p3", n=26, seed=1, p=3, delta_gamma=0.6, delta_beta=0.6, shots=10000)
LARGE = Run("K32_p3", n=32, seed=2, p=3, delta_gamma=0.6, delta_beta=0.6, shots=10000)
LARGE_SWEEP: List[Run] = [
    Run(f"K32_p{p}_d{d}", n=32, seed=2, p=p, delta_gamma=d, delta_beta=d)
    for p in (3, 10) for d in (0.3, 0.6, 0.9)
]
HUGE = Run("K34_p3", n=34, seed=3, p=3, delta_gamma=0.6, delta_beta=0.6, shots=100000)
HUGE_GRAD = Run("K33_p3_grad", n=33, seed=3, p=3, delta_gamma=0.6, delta_beta=0.6)
# single-GPU depth sweep at 30 qubits (the paper's one single-GPU workload)
SWEEP30: List[Run] = [Run(f"K30_p{p}", n=30, seed=5, p=p, delta_gamma=0.6, delta_beta=0.6)
                      for p in (3, 6, 10, 50, 100)]


@dataclass(frozen=True)
class BatchItem:
    n: int
    p: int
    delta_gamma: float
    delta_beta: float
    seed: int

    def weights(self) -> np.ndarray:
        return complete_graph_tenths(self.n, self.seed)


def batch(count: int = 512, master_seed: int = 4, n_lo: int = 14, n_hi: int = 22,
          depths=(3, 5, 10)) -> List[BatchItem]:
    """Uneven batch: n ~ U{n_lo..n_hi}, p ~ U{depths}, slopes ~ U[0.2, 1.0].

    Circuit i draws its graph from seed 1000 + i.
    """
    rng = np.random.default_rng(master_seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ps = rng.choice(np.asarray(depths), size=count)
    dg = rng.uniform(0.2, 1.0, size=count)
    db = rng.uniform(0.2, 1.0, size=count)
    return [BatchItem(int(ns[i]), int(ps[i]), float(dg[i]), float(db[i]), 1000 + i)
            for i in range(count)]


def random_angles(p: int, seed: int, scale: float = 1.0) -> tuple:
    """Arbitrary per-layer gate angles for tests that do not follow a ramp."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(-scale, scale, size=p), rng.uniform(-scale, scale, size=p))


# Noise (Sec. II-C, Fig. 1): depolarizing rate eps after every two-qubit gate.
@dataclass(frozen=True)
class NoiseRun:
    name: str
    n: int
    seed: int
    p: int
    delta: float      # ramp slope, delta_gamma = delta_beta
    eps: float
    ntraj: int

    def weights(self) -> np.ndarray:
        return complete_graph_tenths(self.n, self.seed)


# throughput shape: the paper's largest noisy size, 10 layers, many trajectories
NOISE_BENCH = NoiseRun("K12_p10_eps0.003", n=12, seed=2, p=10, delta=0.6, eps=0.003, ntraj=65536)
