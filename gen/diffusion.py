"""Cell-centred 7-point finite-volume diffusion operator on an Nx x Ny x Nz grid.

Unknown i sits in cell (x, y, z) with i = x + Nx*(y + Ny*z), h = 1.  The face
between two neighbouring cells carries the harmonic transmissibility
2*k_i*k_j/(k_i + k_j); a face on the domain boundary (Dirichlet) carries k_i.
With unit coefficients this is exactly the textbook 7-point Laplacian
(6 on the diagonal, -1 off it), which the closed-form tests rely on.

The result is symmetric positive definite (strictly diagonally dominant on
boundary rows, irreducible).  Columns of each CSR row are sorted ascending.
"""

from __future__ import annotations

import numpy as np

# neighbour offsets in ascending column order: -z, -y, -x, self, +x, +y, +z
_OFFS = ((0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1))


def _pattern(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    valid = []
    for ox, oy, oz in _OFFS:
        valid.append(
            (x + ox >= 0) & (x + ox < nx) & (y + oy >= 0) & (y + oy < ny) & (z + oz >= 0) & (z + oz < nz)
        )
    valid = np.stack([v.ravel() for v in valid], axis=1)  # [n, 7]
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    cols = np.stack([idx + ox + nx * (oy + ny * oz) for ox, oy, oz in _OFFS], axis=1)
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[valid].astype(np.int32)
    return row_ptr, col_idx, valid


def diffusion_matrix(k: np.ndarray):
    """Assemble the operator for cell coefficients ``k`` of shape (Nz, Ny, Nx).

    Returns (row_ptr int64[n+1], col_idx int32[nnz], values float64[nnz]).
    """
    k = np.asarray(k, dtype=np.float64)
    nz, ny, nx = k.shape
    row_ptr, col_idx, valid = _pattern((nx, ny, nz))
    vals = np.zeros((nz, ny, nx, 7), dtype=np.float64)
    diag = np.zeros((nz, ny, nx), dtype=np.float64)
    # axis 2 = x, 1 = y, 0 = z; slot of the minus/plus neighbour in _OFFS
    for axis, (sm, sp) in ((2, (2, 4)), (1, (1, 5)), (0, (0, 6))):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        k_lo, k_hi = k[tuple(lo)], k[tuple(hi)]
        t = 2.0 * k_lo * k_hi / (k_lo + k_hi)
        vals[tuple(lo) + (sp,)] = -t
        vals[tuple(hi) + (sm,)] = -t
        diag[tuple(lo)] += t
        diag[tuple(hi)] += t
        # Dirichlet faces at both ends of this axis
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = slice(0, 1)
        last[axis] = slice(-1, None)
        diag[tuple(first)] += k[tuple(first)]
        diag[tuple(last)] += k[tuple(last)]
    vals[..., 3] = diag
    values = vals.reshape(-1, 7)[valid]
    return row_ptr, col_idx, values


class DiffusionSequence:
    """A sequence of diffusion systems with cumulative random damage.

    System 0 has k = exp(N(0,1)) per cell.  For every later system a random
    ``damage_frac`` of the cells (without replacement) has its coefficient
    multiplied by U[lo, hi]; the damage accumulates.  Each system draws its
    own right-hand side b ~ N(0, 1).

    ``seed`` is a numpy SeedSequence entropy tuple; it is spawned into three
    independent streams (coefficients, damage, right-hand sides).
    """

    block = 1

    def __init__(self, shape, n_systems, seed, damage_frac=0.05, damage_range=(0.5, 1.0)):
        self.shape = tuple(int(s) for s in shape)  # (Nx, Ny, Nz)
        self.n_systems = int(n_systems)
        ss = np.random.SeedSequence(seed)
        s_coef, s_dmg, s_rhs = ss.spawn(3)
        nx, ny, nz = self.shape
        self.n = nx * ny * nz
        self._rng_dmg = np.random.default_rng(s_dmg)
        self._rng_rhs = np.random.default_rng(s_rhs)
        self._k0 = np.exp(np.random.default_rng(s_coef).standard_normal((nz, ny, nx)))
        self.damage_frac = damage_frac
        self.damage_range = damage_range
        self.row_ptr, self.col_idx, _ = _pattern(self.shape)
        self.nnz = int(self.row_ptr[-1])
        self.nnzb = self.nnz
        self._coefs = [self._k0]
        self._rhs = []

    def coefficients(self, k):
        while len(self._coefs) <= k:
            prev = self._coefs[-1].ravel().copy()
            cnt = int(round(self.damage_frac * self.n))
            cells = self._rng_dmg.choice(self.n, size=cnt, replace=False)
            prev[cells] *= self._rng_dmg.uniform(*self.damage_range, size=cnt)
            self._coefs.append(prev.reshape(self._k0.shape))
        return self._coefs[k]

    def rhs(self, k):
        while len(self._rhs) <= k:
            self._rhs.append(self._rng_rhs.standard_normal(self.n))
        return self._rhs[k]

    def system(self, k):
        """(values float64[nnz], b float64[n]) of system k (0-based)."""
        _, _, values = diffusion_matrix(self.coefficients(k))
        return values, self.rhs(k)

    def csr(self, k):
        """(row_ptr, col_idx, values, b) of system k, scalar CSR."""
        values, b = self.system(k)
        return self.row_ptr, self.col_idx, values, b
