"""Oracle casting constraint (Sec. 3.7).  TEST INFRASTRUCTURE ONLY.

Once a casting direction is chosen, the topological level-set field is made
non-decreasing along it, on either side of a parting plane, so that the
extracted topology has no cavity the mould cannot reach.  Reading used here:
the element field phi lives on an nx x ny x nz grid (element e = ex + nx (ey +
ny ez)); the casting axis is a and the parting plane lies before element
index p along a (0 <= p <= n_a).  On the side j >= p the field may not increase
away from the plane (toward +a), on the side j < p it may not increase toward
-a.  The projection is the smallest such field that is >= phi: along every
line of elements parallel to a, the running maximum taken from each far end
toward the plane.  Taking the maximum (never lowering a value) keeps every
element at least as high in the ranking as before.

The projected field is constant along plateaus (runs of equal running
maxima).  A topology cut through a plateau has no cavity only if the plateau
is cut nearer-to-the-plane first, so the extraction ranks equal values by the
distance of the element from the parting plane along the axis
(parting_distance: j - p on the side j >= p, p - 1 - j on the side j < p)
before the element index.
"""
from __future__ import annotations

import numpy as np


def cast_project(phi, dims, axis, parting):
    nx, ny, nz = (int(d) for d in dims)
    n = (nx, ny, nz)[axis]
    if not 0 <= parting <= n:
        raise ValueError("parting index outside 0..n_axis")
    f = np.asarray(phi, dtype=np.float64).reshape(nz, ny, nx)
    npax = 2 - axis  # numpy axis of grid axis `axis` in [z][y][x] storage
    g = np.moveaxis(f, npax, -1).copy()  # lines along the last axis
    if parting < n:  # side j >= p: running maximum from j = n - 1 down to p
        g[..., parting:] = np.maximum.accumulate(g[..., parting:][..., ::-1], axis=-1)[..., ::-1]
    if parting > 0:  # side j < p: running maximum from j = 0 up to p - 1
        g[..., :parting] = np.maximum.accumulate(g[..., :parting], axis=-1)
    return np.moveaxis(g, -1, npax).reshape(-1)


def parting_distance(dims, axis, parting):
    """Per element (x fastest), the number of elements between it and the
    parting plane along the casting axis: j - p for j >= p, p - 1 - j for j < p."""
    nx, ny, nz = (int(d) for d in dims)
    n = (nx, ny, nz)[axis]
    if not 0 <= parting <= n:
        raise ValueError("parting index outside 0..n_axis")
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = (i, j, k)[axis]
    return np.where(pos >= parting, pos - parting, parting - 1 - pos).reshape(-1).astype(np.int32)
