"""Named synthetic workloads and their seeds.

Every stream is derived from ``np.random.SeedSequence([SEED_ROOT, workload_id,
sequence_id])`` so that a workload is reproducible bit for bit from its three
integers.  Workload ids:

1. diffusion 20^3 (n = 8,000), 8 systems, damage 5% x U[0.5, 1].
2. elasticity 40^3 Q1 (n = 201,720), 20 systems, damage 5% x U[0.7, 1].
3. elasticity 100^3 Q1 (n = 3,060,300), 30 systems.
4. batched diffusion: 256 sequences, n ~ U[5e3, 2e5], 10 systems each.
5. serving elasticity: 64 clients, dofs ~ U[1e4, 5e5], 50 systems each.
"""

from __future__ import annotations

import numpy as np

from .diffusion import DiffusionSequence
from .elasticity import ElasticitySequence

SEED_ROOT = 13017530


def config_diffusion_20(seq_id: int = 0, n_systems: int = 8, N: int = 20):
    return DiffusionSequence((N, N, N), n_systems, (SEED_ROOT, 1, seq_id), damage_frac=0.05,
                             damage_range=(0.5, 1.0))


def config_elasticity(E: int, n_systems: int, workload_id: int = 2, seq_id: int = 0):
    return ElasticitySequence(E, n_systems, (SEED_ROOT, workload_id, seq_id))


def batched_diffusion_sizes(count: int = 256, lo: float = 5e3, hi: float = 2e5, workload_id: int = 4):
    """Grid shapes (Nx, Ny, Nz) with n ~ U[lo, hi]; Nx = Ny = round(n^(1/3))."""
    rng = np.random.default_rng(np.random.SeedSequence((SEED_ROOT, workload_id, 1 << 20)))
    shapes = []
    for n in rng.uniform(lo, hi, size=count):
        nx = max(2, int(round(n ** (1.0 / 3.0))))
        nz = max(2, int(round(n / (nx * nx))))
        shapes.append((nx, nx, nz))
    return shapes


def serving_elasticity_sizes(count: int = 64, lo: float = 1e4, hi: float = 5e5, workload_id: int = 5):
    """Mesh sizes E with 3*E*(E+1)^2 dofs closest to a draw from U[lo, hi]."""
    rng = np.random.default_rng(np.random.SeedSequence((SEED_ROOT, workload_id, 1 << 20)))
    Es = np.arange(2, 80)
    dofs = 3 * Es * (Es + 1) ** 2
    out = []
    for t in rng.uniform(lo, hi, size=count):
        out.append(int(Es[np.argmin(np.abs(dofs - t))]))
    return out


def make_sequence(kind: str, size, n_systems: int, workload_id: int, seq_id: int = 0):
    """Generic constructor: kind 'diffusion' (size = (Nx, Ny, Nz)) or 'elasticity' (size = E)."""
    if kind == "diffusion":
        dmg = (0.5, 1.0)
        return DiffusionSequence(size, n_systems, (SEED_ROOT, workload_id, seq_id), damage_frac=0.05,
                                 damage_range=dmg)
    if kind == "elasticity":
        return ElasticitySequence(int(size), n_systems, (SEED_ROOT, workload_id, seq_id))
    raise ValueError(f"unknown workload kind {kind!r}")
