"""Seeded synthetic knapsack workloads.

This module only draws problem instances (item values and weights, capacity,
population size, QIEO seed, generation budget, arrival times).  It holds none
of the QIEO arithmetic and is the one module that both the CPU oracle's tests
and the GPU library's tests, smoke check and benchmark import.

The paper's own instances and its generator are not published (Sec. IV-A only
gives the (Np, Ng) grid); these generators stand in for them with the value
distributions stated per workload below.  Item draws use numpy's PCG64 keyed
by (instance seed, purpose tag), so they are fixed by the seed alone.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TAG_WEIGHT, TAG_VALUE, TAG_SHAPE, TAG_ARRIVAL = 1, 2, 3, 4


@dataclass
class Instance:
    """One 0/1 knapsack problem plus the QIEO run parameters."""
    values: np.ndarray          # int32 [Ng]
    weights: np.ndarray         # int32 [Ng]
    capacity: int
    n_pop: int
    seed: int                   # key of the QIEO uniform draws
    generations: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_items(self) -> int:
        return int(self.values.size)

    @property
    def genes(self) -> int:
        return self.n_pop * self.n_items


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(tag)])


def correlated_items(n_items: int, wmax: int, offset: int, seed: int):
    """Weights uniform in [1, wmax]; value = weight + offset; C = floor(sum/2)."""
    w = _rng(seed, TAG_WEIGHT).integers(1, wmax + 1, size=n_items, dtype=np.int64)
    v = w + offset
    cap = int(w.sum() // 2)
    return v.astype(np.int32), w.astype(np.int32), cap


def independent_items(n_items: int, lo: int, hi: int, seed: int):
    """Weights and values independently uniform in [lo, hi]; C = floor(sum/2)."""
    w = _rng(seed, TAG_WEIGHT).integers(lo, hi + 1, size=n_items, dtype=np.int64)
    v = _rng(seed, TAG_VALUE).integers(lo, hi + 1, size=n_items, dtype=np.int64)
    cap = int(w.sum() // 2)
    return v.astype(np.int32), w.astype(np.int32), cap


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int, size=None):
    u = rng.random(size)
    x = np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo))))
    return np.clip(x, lo, hi).astype(np.int64)


# --- the single-instance workloads -----------------------------------------

def small_instance() -> Instance:
    """Ng=100, weights U[1,10], value = weight+5, Np=16, 500 generations, seed 0."""
    v, w, cap = correlated_items(100, 10, 5, seed=0)
    return Instance(v, w, cap, 16, 0, 500, name="qieo-knapsack Np=16 Ng=100")


def medium_instance() -> Instance:
    """Ng=10,000, weights U[1,10], value = weight+5, Np=1024, 1000 generations, seed 1."""
    v, w, cap = correlated_items(10_000, 10, 5, seed=1)
    return Instance(v, w, cap, 1024, 1, 1000, name="qieo-knapsack Np=1024 Ng=10000")


def large_instance(n_pop: int = 4096, n_items: int = 200_000) -> Instance:
    """Ng=200,000, weights U[1,100], value = weight+10, Np=4096, 200 generations, seed 2."""
    v, w, cap = correlated_items(n_items, 100, 10, seed=2)
    return Instance(v, w, cap, n_pop, 2, 200,
                    name="qieo-knapsack Np=%d Ng=%d" % (n_pop, n_items))


# --- the batched workload ---------------------------------------------------

def batch_instances(count: int = 512, first_seed: int = 1000, generations: int = 500):
    """Ragged batch: Ng log-uniform in [50, 20000], Np from {32,64,128,256},
    values and weights independently U[1,100], C = floor(sum(w)/2)."""
    out = []
    for k in range(count):
        seed = first_seed + k
        r = _rng(seed, TAG_SHAPE)
        ng = int(log_uniform_int(r, 50, 20_000))
        n_pop = int((32, 64, 128, 256)[int(r.integers(0, 4))])
        v, w, cap = independent_items(ng, 1, 100, seed)
        out.append(Instance(v, w, cap, n_pop, seed, generations, name="batch-%d" % k))
    return out


# --- the serving workload ---------------------------------------------------

@dataclass
class Request:
    arrival_s: float
    instance: Instance


def serving_requests(count: int = 20_000, rate_per_s: float = 500.0,
                     first_seed: int = 100_000, arrival_seed: int = 500):
    """Poisson arrivals; Ng log-uniform in [100, 100000]; Np uniform over
    {64,...,1024}; generation budget uniform in [200, 2000]; weights U[1,10],
    value = weight + 5, C = floor(sum/2)."""
    ar = _rng(arrival_seed, TAG_ARRIVAL)
    gaps = ar.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(count):
        seed = first_seed + k
        r = _rng(seed, TAG_SHAPE)
        ng = int(log_uniform_int(r, 100, 100_000))
        n_pop = int((64, 128, 256, 512, 1024)[int(r.integers(0, 5))])
        gens = int(r.integers(200, 2001))
        v, w, cap = correlated_items(ng, 10, 5, seed)
        out.append(Request(float(t[k]), Instance(v, w, cap, n_pop, seed, gens,
                                                 name="req-%d" % k)))
    return out


def random_instance(n_items: int, n_pop: int, seed: int, generations: int = 10,
                    wmax: int = 10, offset: int = 5) -> Instance:
    """Correlated instance of arbitrary shape (used for ragged test sizes)."""
    v, w, cap = correlated_items(n_items, wmax, offset, seed)
    return Instance(v, w, cap, n_pop, seed, generations,
                    name="rand Np=%d Ng=%d" % (n_pop, n_items))
