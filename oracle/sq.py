"""Structure factor of the blob centres (Results section, Eq. Sfactor), plain
FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring): used by the tests and
the benchmark's checks, never by the product path.

Wavevectors of a sheared box.  The periodic images of a Lees-Edwards box
with offset delta sit at R + a Lx x + b (Ly y + delta x) + c Lz z for integer
a, b, c.  A wavevector gives the same phase at every image -- so that S(q)
does not depend on which image of a particle is stored -- exactly when
    q . Lx x = 2 pi mx,   q . (Ly y + delta x) = 2 pi my,   q . Lz z = 2 pi mz
for integers (mx, my, mz), i.e.
    qx = 2 pi mx / Lx,   qy = (2 pi my - qx delta) / Ly,   qz = 2 pi mz / Lz.
S(q) = |sum_c exp(-i q . R_c)|^2 / C for one configuration of C particles;
the average over configurations is the caller's.
"""
import math

import numpy as np


def le_wavevectors(box, delta, m):
    """(nq, 3) wavevectors of the integer triples m (nq, 3) for a box
    (Lx, Ly, Lz) at Lees-Edwards offset delta."""
    m = np.asarray(m, dtype=np.float64).reshape(-1, 3)
    Lx, Ly, Lz = (float(b) for b in box)
    qx = 2.0 * math.pi * m[:, 0] / Lx
    qy = (2.0 * math.pi * m[:, 1] - qx * float(delta)) / Ly
    qz = 2.0 * math.pi * m[:, 2] / Lz
    return np.stack([qx, qy, qz], axis=1)


def structure_factor(box, delta, pos, m, chunk=65536):
    """S(q) for each triple of m, positions pos (C, 3), by the definition:
    the real and imaginary parts of sum_c exp(-i q . R_c), summed in order
    over chunks of particles, squared and divided by C."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    q = le_wavevectors(box, delta, m)
    re = np.zeros(len(q))
    im = np.zeros(len(q))
    for a in range(0, len(pos), chunk):
        ph = pos[a:a + chunk] @ q.T          # (chunk, nq) phases q . R_c
        re += np.cos(ph).sum(axis=0)
        im -= np.sin(ph).sum(axis=0)
    return (re * re + im * im) / len(pos)


def grid_triples(nx, my_max, mz=0):
    """The triples of the (qx, qy) grid in the library's output order:
    mx = 0..nx-1 (rows), my = -my_max..my_max (columns), fixed mz."""
    mx, my = np.meshgrid(np.arange(nx), np.arange(-my_max, my_max + 1), indexing="ij")
    return np.stack([mx.ravel(), my.ravel(), np.full(mx.size, mz)], axis=1)
