"""A sequence whose matrices evolve from the computed solutions.

The paper's second and third experiments (Sections 5.2 and 5.3) solve the
tangent systems of nonlinear loops: each matrix depends on the displacement
computed for the previous one.  This workload reproduces that dependence
synthetically on the elasticity cube of ``elasticity.py``: a secant loop of
a damaging material under an increasing load.

System k has the element moduli E_e^(k) = E_e^(0) g(eps_e^(k-1) / s), where
E^(0) are the moduli of the undamaged cube with its stiff inclusions,
eps_e^(k-1) the equivalent strain at the centre of element e of the
displacement solved for system k-1 (eps^(-1) = 0), s the 90th percentile of
the strains of the first solution (so that about a tenth of the cube starts
to soften), and g(t) = max(g_min, 1 / (1 + c (t - 1)_+^2)) a smooth
softening.  The right-hand side is an increasing load b^(k) = (1 + k/4) f:
a uniform pull along +x on every free node plus a seeded N(0, 0.1) part.

Only inputs are built here (moduli, matrix values, right-hand sides); the
strain of a displacement is the workload's own physics.  Use:

    seq = NewtonSequence(E, n_systems, seed)
    vals, b = seq.system(0); x = solve(...); seq.advance(x)
    vals, b = seq.system(1); ...
"""

from __future__ import annotations

import numpy as np

from .elasticity import ElasticitySequence, elasticity_blocks


def centre_strain(E: int, x: np.ndarray) -> np.ndarray:
    """Equivalent strain sqrt(e_xx^2 + e_yy^2 + e_zz^2 + (g_xy^2 + g_yz^2 + g_xz^2)/2)
    at the centre of every element of the E^3 cube, indexed [ez, ey, ex],
    for the free-dof displacement x (clamped face x = 0 has u = 0)."""
    n1 = E + 1
    h = 1.0 / E
    u = np.zeros((n1, n1, n1, 3))
    u[:, :, 1:, :] = np.asarray(x, dtype=np.float64).reshape(n1, n1, E, 3)
    # centre derivatives of the trilinear shape functions: dN_a/dx_i = s_ai / (4h)
    e = np.zeros((6, E, E, E))
    for az in (0, 1):
        for ay in (0, 1):
            for ax in (0, 1):
                ua = u[az : az + E, ay : ay + E, ax : ax + E, :]
                sx, sy, sz = 2 * ax - 1, 2 * ay - 1, 2 * az - 1
                e[0] += sx * ua[..., 0]
                e[1] += sy * ua[..., 1]
                e[2] += sz * ua[..., 2]
                e[3] += sy * ua[..., 0] + sx * ua[..., 1]
                e[4] += sz * ua[..., 1] + sy * ua[..., 2]
                e[5] += sz * ua[..., 0] + sx * ua[..., 2]
    e /= 4.0 * h
    return np.sqrt(e[0] ** 2 + e[1] ** 2 + e[2] ** 2 + 0.5 * (e[3] ** 2 + e[4] ** 2 + e[5] ** 2))


def softening(t: np.ndarray, c: float = 4.0, g_min: float = 0.05) -> np.ndarray:
    return np.maximum(g_min, 1.0 / (1.0 + c * np.maximum(t - 1.0, 0.0) ** 2))


class NewtonSequence:
    """Secant loop of a damaging elastic cube (see the module docstring)."""

    block = 3

    def __init__(self, E, n_systems, seed, load_noise=0.1):
        self.base = ElasticitySequence(E, 1, seed)
        self.E = self.base.E
        self.n_systems = int(n_systems)
        self.row_ptr, self.col_idx = self.base.row_ptr, self.base.col_idx
        self.n, self.nb, self.nnzb, self.nnz = self.base.n, self.base.nb, self.base.nnzb, self.base.nnz
        rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(4)[3])
        f = np.zeros((self.nb, 3))
        f[:, 0] = 1.0 / self.nb
        f += load_noise / self.nb * rng.standard_normal((self.nb, 3))
        self._f = f.ravel()
        self._mod0 = self.base.moduli(0)
        self._mods = [self._mod0]
        self._scale = None
        self.strains = []

    def moduli(self, k):
        if k >= len(self._mods):
            raise ValueError(f"system {k} needs the solution of system {k - 1} (call advance)")
        return self._mods[k]

    def rhs(self, k):
        return (1.0 + 0.25 * k) * self._f

    def system(self, k):
        """(blocks float64[nnzb*9], b float64[n]) of system k."""
        blocks = elasticity_blocks(self.moduli(k), self.base._kref, self.nnzb)
        return blocks.reshape(-1), self.rhs(k)

    def advance(self, x):
        """Record the solution of the latest system; defines the next one."""
        eps = centre_strain(self.E, x)
        if self._scale is None:
            self._scale = float(np.quantile(eps, 0.9))
        self.strains.append(eps)
        self._mods.append(self._mod0 * softening(eps / self._scale))

    def csr(self, k):
        from .elasticity import bsr_to_csr

        blocks, b = self.system(k)
        rp, ci, v = bsr_to_csr(self.row_ptr, self.col_idx, blocks.reshape(-1, 3, 3))
        return rp, ci, v, b
