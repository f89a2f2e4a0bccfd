"""Seeded synthetic workloads: sequences of sparse SPD systems A^(k) x = b^(k).

This module only builds inputs (sparsity patterns, matrix values, right-hand
sides).  It contains none of the solver's arithmetic and is the one piece of
code that both the CPU oracle (under ``oracle/``) and the HIP library
(``paper_1301_7530_amd``) are fed from.

The paper's own workloads (FETI interface problems on meshes that are not
available, Section 5) are replaced by two families of assembled operators
with the same character (3D, heterogeneous, slowly changing from one system
to the next, as the multiresolution setting of Section 1 and Section 3
assumes):

* ``diffusion``: cell-centred 7-point finite volumes, lognormal cell
  coefficients, one unknown per cell (scalar CSR).
* ``elasticity``: Q1 hexahedral linear elasticity on a cube with one clamped
  face and stiff random inclusions (3x3 nodal block CSR, i.e. BSR).
* ``newton``: the elasticity cube in a secant loop, each matrix built from
  the strains of the previous solution (the nonlinear sequences of the
  paper's Sections 5.2 and 5.3, made synthetic).

Sequences perturb a random subset of cells/elements at every step
(cumulative "damage"), and draw a fresh Gaussian right-hand side per system.
"""

from .diffusion import diffusion_matrix, DiffusionSequence
from .elasticity import q1_reference_stiffness, elasticity_matrix, ElasticitySequence, bsr_to_csr
from .newton import NewtonSequence, centre_strain, softening
from .workloads import (
    SEED_ROOT,
    make_sequence,
    config_diffusion_20,
    config_elasticity,
    batched_diffusion_sizes,
    serving_elasticity_sizes,
)

__all__ = [
    "diffusion_matrix",
    "DiffusionSequence",
    "q1_reference_stiffness",
    "elasticity_matrix",
    "ElasticitySequence",
    "bsr_to_csr",
    "NewtonSequence",
    "centre_strain",
    "softening",
    "SEED_ROOT",
    "make_sequence",
    "config_diffusion_20",
    "config_elasticity",
    "batched_diffusion_sizes",
    "serving_elasticity_sizes",
]
