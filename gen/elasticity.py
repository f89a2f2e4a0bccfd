"""Q1 hexahedral linear elasticity on the unit cube, 3x3 nodal blocks.

The cube [0,1]^3 is cut into E^3 cubic elements of side h = 1/E.  Every
element is isotropic with Poisson ratio nu and its own Young modulus E_e, so
its stiffness is E_e * K_ref, K_ref being the 24x24 stiffness of a cube of
side h and unit modulus integrated with 2x2x2 Gauss points.  Nodes on the
face x = 0 are clamped and their degrees of freedom eliminated.

Free node (ix, iy, iz), ix in 1..E, iy, iz in 0..E, has index
p = (ix-1) + E*(iy + (E+1)*iz) and dofs 3p, 3p+1, 3p+2 (u_x, u_y, u_z).
The operator is returned as block CSR (BSR) with 3x3 row-major blocks and
ascending block columns; ``bsr_to_csr`` expands it to scalar CSR.
"""

from __future__ import annotations

import numpy as np

_GP = 1.0 / np.sqrt(3.0)


def q1_reference_stiffness(h: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """24x24 stiffness of a cube of side ``h`` with unit Young modulus.

    Local node a = ax + 2*ay + 4*az sits at corner (ax, ay, az)*h; dof 3a+d
    is its displacement along axis d.  Strains are ordered
    (xx, yy, zz, xy, yz, xz) with engineering shear.
    """
    lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = 1.0 / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[[0, 1, 2], [0, 1, 2]] += 2.0 * mu
    D[[3, 4, 5], [3, 4, 5]] = mu
    corners = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=np.float64)
    sgn = 2.0 * corners - 1.0  # reference coordinates of the corners, +-1
    K = np.zeros((24, 24))
    detj = (h / 2.0) ** 3
    for gz in (-_GP, _GP):
        for gy in (-_GP, _GP):
            for gx in (-_GP, _GP):
                g = np.array([gx, gy, gz])
                f = 1.0 + sgn * g  # [8, 3]
                dN = np.empty((8, 3))
                dN[:, 0] = sgn[:, 0] * f[:, 1] * f[:, 2] / 8.0
                dN[:, 1] = f[:, 0] * sgn[:, 1] * f[:, 2] / 8.0
                dN[:, 2] = f[:, 0] * f[:, 1] * sgn[:, 2] / 8.0
                dN *= 2.0 / h
                B = np.zeros((6, 24))
                for a in range(8):
                    dx, dy, dz = dN[a]
                    c = 3 * a
                    B[0, c] = dx
                    B[1, c + 1] = dy
                    B[2, c + 2] = dz
                    B[3, c], B[3, c + 1] = dy, dx
                    B[4, c + 1], B[4, c + 2] = dz, dy
                    B[5, c], B[5, c + 2] = dz, dx
                K += B.T @ D @ B * detj
    return 0.5 * (K + K.T)


def _offsets():
    # ascending block-column order: oz major, then oy, then ox
    return [(ox, oy, oz) for oz in (-1, 0, 1) for oy in (-1, 0, 1) for ox in (-1, 0, 1)]


def _pattern(E: int):
    """Validity mask [n_free_nodes, 27] and block CSR pattern for an E^3 mesh."""
    n1 = E + 1
    iz, iy, ix = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(1, n1), indexing="ij")
    valid = []
    cols = []
    p = (ix - 1) + E * (iy + n1 * iz)
    for ox, oy, oz in _offsets():
        qx, qy, qz = ix + ox, iy + oy, iz + oz
        v = (qx >= 1) & (qx <= E) & (qy >= 0) & (qy <= E) & (qz >= 0) & (qz <= E)
        valid.append(v.ravel())
        cols.append((p + ox + E * (oy + n1 * oz)).ravel())
    valid = np.stack(valid, axis=1)
    cols = np.stack(cols, axis=1)
    nb = valid.shape[0]
    row_ptr = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(valid.sum(axis=1), out=row_ptr[1:])
    col_idx = cols[valid].astype(np.int32)
    return row_ptr, col_idx, valid


_asm_lib = None


def _asm():
    global _asm_lib
    if _asm_lib is None:
        import ctypes

        from .build import ensure_built

        L = ctypes.CDLL(ensure_built())
        D = ctypes.POINTER(ctypes.c_double)
        L.gen_elasticity_blocks.restype = None
        L.gen_elasticity_blocks.argtypes = [ctypes.c_int, D, D, D]
        _asm_lib = L
    return _asm_lib


def elasticity_blocks(moduli: np.ndarray, kref: np.ndarray, nnzb: int) -> np.ndarray:
    """Blocks float64[nnzb, 3, 3] in block-CSR order, assembled by the C
    helper (same sums, same rounding as ``elasticity_matrix``)."""
    import ctypes

    mod = np.ascontiguousarray(moduli, dtype=np.float64)
    kr = np.ascontiguousarray(kref, dtype=np.float64)
    out = np.empty((nnzb, 3, 3), dtype=np.float64)
    D = ctypes.POINTER(ctypes.c_double)
    _asm().gen_elasticity_blocks(mod.shape[0], mod.ctypes.data_as(D), kr.ctypes.data_as(D), out.ctypes.data_as(D))
    return out


def elasticity_matrix(moduli: np.ndarray, nu: float = 0.3, kref: np.ndarray | None = None):
    """Assemble for element moduli of shape (E, E, E) indexed [ez, ey, ex]
    (vectorised numpy; the reference for the C helper).

    Returns (block_row_ptr int64[nb+1], block_col int32[nnzb],
    blocks float64[nnzb, 3, 3]) with nb = E*(E+1)^2 free nodes.
    """
    moduli = np.asarray(moduli, dtype=np.float64)
    E = moduli.shape[0]
    if kref is None:
        kref = q1_reference_stiffness(1.0 / E, nu)
    n1 = E + 1
    full = np.zeros((n1, n1, n1, 27, 3, 3), dtype=np.float64)
    offs = {o: i for i, o in enumerate(_offsets())}
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        for b in range(8):
            bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
            oi = offs[(bx - ax, by - ay, bz - az)]
            blk = kref[3 * a : 3 * a + 3, 3 * b : 3 * b + 3]
            full[az : az + E, ay : ay + E, ax : ax + E, oi] += moduli[..., None, None] * blk
    row_ptr, col_idx, valid = _pattern(E)
    blocks = full[:, :, 1:].reshape(-1, 27, 3, 3)[valid]
    return row_ptr, col_idx, blocks


def bsr_to_csr(block_row_ptr, block_col, blocks):
    """Expand 3x3 BSR to scalar CSR with ascending columns.

    Scalar row 3i+d holds, for every block (rank r in block row i), the three
    entries of the block's row d, at offset 3r+e within the row.
    """
    block_row_ptr = np.asarray(block_row_ptr, dtype=np.int64)
    block_col = np.asarray(block_col)
    blocks = np.asarray(blocks, dtype=np.float64).reshape(-1, 3, 3)
    nb = len(block_row_ptr) - 1
    cnt = np.diff(block_row_ptr)
    nnzb = len(block_col)
    row_ptr = np.zeros(3 * nb + 1, dtype=np.int64)
    np.cumsum(np.repeat(3 * cnt, 3), out=row_ptr[1:])
    first = np.repeat(block_row_ptr[:-1], cnt)
    rank = np.arange(nnzb, dtype=np.int64) - first
    rowlen = np.repeat(3 * cnt, cnt)
    d = np.arange(3)[None, :, None]
    e = np.arange(3)[None, None, :]
    pos = 9 * first[:, None, None] + d * rowlen[:, None, None] + 3 * rank[:, None, None] + e
    out_cols = np.empty(9 * nnzb, dtype=np.int32)
    out_vals = np.empty(9 * nnzb, dtype=np.float64)
    out_cols[pos.ravel()] = np.broadcast_to(3 * block_col.astype(np.int64)[:, None, None] + e, (nnzb, 3, 3)).ravel()
    out_vals[pos.ravel()] = blocks.ravel()
    return row_ptr, out_cols, out_vals


class ElasticitySequence:
    """A sequence of elasticity systems with cumulative random damage.

    System 0: ``n_incl`` cubic inclusions of modulus ``e_incl`` are placed at
    random positions (they may overlap) in a matrix of modulus 1; their side
    (in elements) is chosen so that together they fill about ``incl_frac``
    of the volume, as in the paper's heterogeneous cube with 4x4x4 cubic
    inclusions (Section 5.1).  Every later system multiplies the modulus of
    a random ``damage_frac`` of the elements by U[lo, hi] (secant modulus of
    damaged elements), cumulatively.  Each system draws its own right-hand
    side b ~ N(0, 1) per free dof.
    """

    block = 3

    def __init__(self, E, n_systems, seed, nu=0.3, incl_frac=0.10, e_incl=1.0e3, n_incl=64,
                 damage_frac=0.05, damage_range=(0.7, 1.0)):
        self.E = int(E)
        self.n_systems = int(n_systems)
        self.nu = nu
        ss = np.random.SeedSequence(seed)
        s_coef, s_dmg, s_rhs = ss.spawn(3)
        E_ = self.E
        rng = np.random.default_rng(s_coef)
        side = min(E_, max(1, int(round(E_ * (incl_frac / n_incl) ** (1.0 / 3.0)))))
        mod = np.ones((E_, E_, E_))
        for _ in range(n_incl):
            z, y, x = rng.integers(0, E_ - side + 1, size=3)
            mod[z : z + side, y : y + side, x : x + side] = e_incl
        self.incl_side = side
        self._mod = [mod]
        self._rng_dmg = np.random.default_rng(s_dmg)
        self._rng_rhs = np.random.default_rng(s_rhs)
        self.damage_frac = damage_frac
        self.damage_range = damage_range
        self.row_ptr, self.col_idx, _ = _pattern(self.E)
        self.nb = len(self.row_ptr) - 1
        self.n = 3 * self.nb
        self.nnzb = int(self.row_ptr[-1])
        self.nnz = 9 * self.nnzb
        self._kref = q1_reference_stiffness(1.0 / self.E, nu)
        self._rhs = []

    def moduli(self, k):
        while len(self._mod) <= k:
            prev = self._mod[-1].ravel().copy()
            ne = prev.size
            cnt = int(round(self.damage_frac * ne))
            els = self._rng_dmg.choice(ne, size=cnt, replace=False)
            prev[els] *= self._rng_dmg.uniform(*self.damage_range, size=cnt)
            self._mod.append(prev.reshape(self._mod[0].shape))
        return self._mod[k]

    def rhs(self, k):
        while len(self._rhs) <= k:
            self._rhs.append(self._rng_rhs.standard_normal(self.n))
        return self._rhs[k]

    def system(self, k):
        """(blocks float64[nnzb*9] row-major 3x3, b float64[n]) of system k."""
        blocks = elasticity_blocks(self.moduli(k), self._kref, self.nnzb)
        return blocks.reshape(-1), self.rhs(k)

    def csr(self, k):
        """(row_ptr, col_idx, values, b) of system k expanded to scalar CSR."""
        blocks, b = self.system(k)
        rp, ci, v = bsr_to_csr(self.row_ptr, self.col_idx, blocks.reshape(-1, 3, 3))
        return rp, ci, v, b
