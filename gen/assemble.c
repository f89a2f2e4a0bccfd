/*
 * Input generation only: assembly of the Q1 elasticity operator's 3x3
 * blocks from element moduli, in block-CSR order.  Holds no solver
 * arithmetic.  It reproduces, bit for bit, the summation order of the
 * vectorised numpy assembly in elasticity.py (for each block, the
 * contributions of the element corners in ascending corner number, each a
 * product modulus * reference-block entry added to a running sum from 0).
 *
 * Free node (ix, iy, iz), ix in 1..E, iy, iz in 0..E, is block row
 * p = (ix-1) + E*(iy + (E+1)*iz).  Its blocks follow the 27 neighbour
 * offsets in ascending order (oz, then oy, then ox, each -1..1), keeping
 * the neighbours that are free nodes.  Local corner a = ax + 2 ay + 4 az of
 * element (ex, ey, ez) sits at node (ex+ax, ey+ay, ez+az).
 */
#include <stdint.h>

void gen_elasticity_blocks(int E, const double* mod, const double* kref, double* out) {
    const int n1 = E + 1;
    int64_t pos = 0;
    for (int iz = 0; iz <= E; ++iz)
        for (int iy = 0; iy <= E; ++iy)
            for (int ix = 1; ix <= E; ++ix)
                for (int oz = -1; oz <= 1; ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox) {
                            const int qx = ix + ox, qy = iy + oy, qz = iz + oz;
                            if (qx < 1 || qx > E || qy < 0 || qy > E || qz < 0 || qz > E) continue;
                            double blk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                            for (int a = 0; a < 8; ++a) {
                                const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
                                const int bx = ax + ox, by = ay + oy, bz = az + oz;
                                if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                                const int ex = ix - ax, ey = iy - ay, ez = iz - az;
                                if (ex < 0 || ex >= E || ey < 0 || ey >= E || ez < 0 || ez >= E) continue;
                                const int b = bx + 2 * by + 4 * bz;
                                const double m = mod[((int64_t)ez * E + ey) * E + ex];
                                for (int d = 0; d < 3; ++d)
                                    for (int f = 0; f < 3; ++f) blk[3 * d + f] += m * kref[(3 * a + d) * 24 + 3 * b + f];
                            }
                            for (int t = 0; t < 9; ++t) out[pos * 9 + t] = blk[t];
                            ++pos;
                        }
    (void)n1;
}
