"""Seeded synthetic workloads of the GMF-FLBM hot path.

This module holds no arithmetic of the method: it names the lattice sizes,
relaxation times, k_B T and seeds of the workloads, and draws seeded random
perturbations that tests hand to both the library and the oracle.  The paper's
own runs (Results section) use an equilibrium fluid at rho = 1 started at rest;
the workloads below have that structure at the sizes the benchmarks use.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TAU_CHOICES = (0.51, 0.6, 0.8, 1.0, 2.0, 5.0)


@dataclass
class Box:
    n: tuple
    tau: float
    kbt: float
    seed: int
    rho0: float = 1.0


@dataclass
class Workload:
    name: str
    boxes: list
    steps: int
    warmup: int = 0
    precision: str = "fp32"          # "fp32" (shifted) or "fp64" (plain)
    sample_every: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return int(sum(np.prod(b.n) for b in self.boxes))


def small_parity() -> Workload:
    """16^3 periodic box, rho0 = 1, tau = 1, k_B T = 1e-4, seed 1, 200 steps, FP64."""
    return Workload("d3q27_16cube_fp64_tau1", [Box((16, 16, 16), 1.0, 1e-4, 1)], steps=200,
                    precision="fp64", sample_every=1)


def tau_sweep(precision: str = "fp32") -> Workload:
    """64^3 at tau in {0.51, 0.6, 1, 2, 5}, k_B T = 1e-4, seed 1 each, 2000 warm-up + 20000 steps."""
    return Workload(f"d3q27_64cube_5tau_{precision}",
                    [Box((64, 64, 64), t, 1e-4, 1) for t in (0.51, 0.6, 1.0, 2.0, 5.0)],
                    steps=20000, warmup=2000, precision=precision, sample_every=10)


def bandwidth_headline(precision: str = "fp32") -> Workload:
    """256^3, rho0 = 1, tau = 0.8, k_B T = 1e-4, seed 1, 2000 steps."""
    return Workload(f"d3q27_256cube_{precision}_tau0.8", [Box((256, 256, 256), 0.8, 1e-4, 1)], steps=2000,
                    warmup=50, precision=precision)


def ensemble_taus(seed: int = 2601) -> list:
    """tau of the 64 ensemble replicas, drawn uniformly from TAU_CHOICES with a
    seeded numpy generator (32 at 32^3, then 16 at 48^3, then 16 at 64^3)."""
    rng = np.random.default_rng(seed)
    return [TAU_CHOICES[i] for i in rng.integers(0, len(TAU_CHOICES), size=64)]


def ensemble() -> Workload:
    """32 replicas at 32^3, 16 at 48^3 and 16 at 64^3, seeds 1..64, k_B T = 1e-4, 5000 steps."""
    taus = ensemble_taus()
    sizes = [32] * 32 + [48] * 16 + [64] * 16
    boxes = [Box((s, s, s), taus[i], 1e-4, i + 1) for i, s in enumerate(sizes)]
    return Workload("d3q27_ensemble_64rep_fp32", boxes, steps=5000, precision="fp32", sample_every=10)


def precision_stress(precision: str = "fp32") -> Workload:
    """512^3 at tau = 0.55, k_B T = 1e-5, seed 1, 500 steps, plus the embedded 16^3 box with the same
    (seed, tau, k_B T) run in the same launch."""
    return Workload(f"d3q27_512cube_{precision}_tau0.55",
                    [Box((512, 512, 512), 0.55, 1e-5, 1), Box((16, 16, 16), 0.55, 1e-5, 1)],
                    steps=500, precision=precision, sample_every=10)


def perturbed_populations(weights, n_nodes: int, rho0: float = 1.0, amp: float = 0.02, seed: int = 0,
                          velocity: float = 0.0) -> np.ndarray:
    """Canonical populations f[i*N + n] = w_i rho0 (1 + amp U(-1,1)) (1 + velocity c-independent
    scale); a seeded random non-equilibrium state with density, momentum and stress
    fluctuations.  `weights` are the 27 lattice weights in the interface order."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64).reshape(27, 1)
    f = w * rho0 * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(27, n_nodes)))
    if velocity:
        f *= 1.0 + velocity * rng.uniform(-1.0, 1.0, size=(1, n_nodes))
    return np.ascontiguousarray(f.reshape(-1))


def sample_nodes(n_nodes: int, count: int, seed: int = 0) -> np.ndarray:
    """Distinct node indices for sampled comparisons, always including the box corners."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(n_nodes, size=min(count, n_nodes), replace=False)
    return np.unique(np.concatenate([pick, [0, n_nodes - 1]])).astype(np.int64)
