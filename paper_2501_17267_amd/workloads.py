"""Seeded synthetic workloads: seeds, sizes and schedules, nothing else.

This module is shared by the tests, the benchmark and the oracle-side
checks.  It holds none of the method's arithmetic: it only derives 64-bit
seeds (with the splitmix64 finaliser, Steele-Lea-Flood 2014) and lists the
shapes of the five workloads.  Every instance it names is a synthetic
tile-planted stand-in (class "T6": every tile has all six faces frustrated)
generated on demand by either implementation from (L, class, seed).

Workload shapes (sizes as in the annealing experiments of App. D, made
concrete for one GPU):
  sa_small   1 instance, L=4, 64 restarts x 1000 sweeps, beta 0.1 -> 3.0 linear
  sa_batch   16 instances at each of L = 8, 12, 16; 1024 replicas; 256 sweeps
  pt         L=12; 32 temperatures, beta geometric 0.2 -> 3.0; 128 runs; 2000 steps
  uneven     4096 instances, L in {6,8,10,12,16,20}, 64 replicas, 128..1024 sweeps
  serve      Poisson 2000 req/s; L even in [8, 32] (95 %) or 64 (5 %);
             sweeps log-uniform 64..4096; one replica per request
"""
from __future__ import annotations

from dataclasses import dataclass, field

MASTER_SEED = 0x250117267
MASK64 = (1 << 64) - 1
T6 = 6  # class code: number of frustrated faces per tile

WORKLOAD_IDS = {"sa_small": 1, "sa_batch": 2, "pt": 3, "uneven": 4, "serve": 5, "fragment": 6, "tn": 7}


def mix64(x: int) -> int:
    """splitmix64 output function applied to x + golden gamma (one draw)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def instance_seed(workload: str, k: int) -> int:
    wid = WORKLOAD_IDS[workload]
    return mix64((MASTER_SEED + (wid << 40) + k) & MASK64)


def philox_seed(workload: str) -> int:
    wid = WORKLOAD_IDS[workload]
    return mix64((MASTER_SEED ^ (wid << 56)) & MASK64)


@dataclass(frozen=True)
class InstanceSpec:
    L: int
    seed: int
    chain: int          # fourth Philox counter word of this instance's chains
    cls: int = T6


@dataclass(frozen=True)
class SAWorkload:
    name: str
    instances: tuple
    n_rep: int
    n_sweeps: int
    beta0: float = 0.1
    beta1: float = 3.0
    kind: int = 0          # 0 linear, 1 geometric
    seed: int = 0


def sa_small() -> SAWorkload:
    inst = (InstanceSpec(4, instance_seed("sa_small", 0), 0),)
    return SAWorkload("sa_small", inst, 64, 1000, seed=philox_seed("sa_small"))


def sa_batch(sizes=(8, 12, 16), per_size=16, n_rep=1024, n_sweeps=256) -> SAWorkload:
    insts = []
    k = 0
    for L in sizes:
        for _ in range(per_size):
            insts.append(InstanceSpec(L, instance_seed("sa_batch", k), k))
            k += 1
    return SAWorkload("sa_batch", tuple(insts), n_rep, n_sweeps, seed=philox_seed("sa_batch"))


@dataclass(frozen=True)
class PTWorkload:
    name: str
    instance: InstanceSpec
    T: int
    beta0: float
    beta1: float
    n_runs: int
    n_steps: int
    seed: int


def pt(n_runs=128, n_steps=2000, L=12, T=32) -> PTWorkload:
    return PTWorkload("pt", InstanceSpec(L, instance_seed("pt", 0), 0), T, 0.2, 3.0,
                      n_runs, n_steps, philox_seed("pt"))


@dataclass(frozen=True)
class UnevenJob:
    inst: InstanceSpec
    n_rep: int
    n_sweeps: int


def uneven(n_inst=4096, n_rep=64, sizes=(6, 8, 10, 12, 16, 20),
           budgets=(128, 256, 512, 1024)) -> tuple:
    """Jobs of the uneven batch: L and sweep budget drawn from the seed."""
    jobs = []
    for k in range(n_inst):
        s = instance_seed("uneven", k)
        L = sizes[mix64(s ^ 0x1) % len(sizes)]
        S = budgets[mix64(s ^ 0x2) % len(budgets)]
        jobs.append(UnevenJob(InstanceSpec(L, s, k), n_rep, S))
    return tuple(jobs)


def uneven_seed() -> int:
    return philox_seed("uneven")


@dataclass(frozen=True)
class FragmentSetting:
    name: str
    core: int
    halo: int
    replicas: int
    n_sweeps: int
    order: int = 1          # diagonal wavefront
    beta0: float = 0.1
    beta1: float = 3.0


def fragment_settings():
    """The meta-heuristic as measured: the paper's fragment edge l = 5 with
    one decimated spin per fragment, and a cheaper block form (2^3 cores in
    4^3 fragments)."""
    return (FragmentSetting("l5_single_spin", 1, 2, 8, 100),
            FragmentSetting("l4_block8", 2, 1, 8, 50))


def fragment_instances(L: int, n: int = 20):
    return tuple(InstanceSpec(L, instance_seed("fragment", 1000 * L + k), k) for k in range(n))


def tn_instances(L: int, n: int = 20):
    """Instances of the tensor-network meta-heuristic study (one decimation
    each, deterministic: no counter words)."""
    return tuple(InstanceSpec(L, instance_seed("tn", 1000 * L + k), k) for k in range(n))
