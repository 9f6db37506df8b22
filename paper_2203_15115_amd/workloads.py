"""Seeded synthetic inputs for the voxel cantilever solves.

This module only draws and shapes inputs (densities, fixity masks, load
vectors, request streams).  It contains none of the finite element arithmetic,
so both the HIP path and the CPU oracle can be fed from it without sharing any
of the method's code.

Conventions (shared by every consumer of these arrays):

* element ``e = ex + nx*(ey + ny*ez)``, node ``n = i + (nx+1)*(j + (ny+1)*k)``;
* DOF ``3*n + c`` with ``c`` in (x, y, z), i.e. DOFs interleaved per node;
* load arrays have shape ``(nrhs, ndof)`` (row-major, one right-hand side per row).

The cantilever recipe stands in for the paper's part geometries (its figures
are not available): a box domain discretised by unit hexahedral voxels (the
paper discretises its parts by hexahedral elements, Sec. 3.8 step 1), clamped on
the x=0 face, loaded at the far end, with a random solid/void pattern that
plays the role of a topology extracted from a level set (Eq. 3.6).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SOLID = 1.0
VOID = 1.0e-3  # ersatz stiffness scale of void elements


def n_nodes(dims):
    nx, ny, nz = dims
    return (nx + 1) * (ny + 1) * (nz + 1)


def n_elems(dims):
    nx, ny, nz = dims
    return nx * ny * nz


def node_id(dims, i, j, k):
    nx, ny, _ = dims
    return i + (nx + 1) * (j + (ny + 1) * k)


def smooth_field(dims, seed, ell):
    """Smooth Gaussian random field on the element grid, shape (nz, ny, nx).

    White noise from ``default_rng(seed)`` filtered in Fourier space by
    ``exp(-2 pi^2 ell^2 |k|^2)`` (periodic), i.e. a Gaussian kernel of
    standard deviation ``ell`` elements.
    """
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nz, ny, nx))
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    filt = np.exp(-2.0 * math.pi ** 2 * ell ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    f = np.fft.irfftn(np.fft.rfftn(w) * filt, s=(nz, ny, nx))
    return f


def density_from_field(field, void_pct):
    """Per-element scale: VOID where the field is strictly below its
    ``void_pct`` percentile, SOLID elsewhere.  Returned flat in element order."""
    thr = np.percentile(field, void_pct)
    rho = np.where(field < thr, VOID, SOLID)
    return np.ascontiguousarray(rho.reshape(-1), dtype=np.float64)


def clamp_x0(dims):
    """uint8 mask per DOF: 1 on every DOF of the x=0 face."""
    nx, ny, nz = dims
    m = np.zeros((nz + 1, ny + 1, nx + 1, 3), dtype=np.uint8)
    m[:, :, 0, :] = 1
    return m.reshape(-1)


def edge_load(dims, which):
    """Unit total -z force shared equally by the nodes of one x=L edge line.

    ``which`` is 'bottom' (k=0), 'mid' (k=nz//2) or 'top' (k=nz); the edge runs
    along y, so each of its ny+1 nodes carries -1/(ny+1)."""
    nx, ny, nz = dims
    k = {"bottom": 0, "mid": nz // 2, "top": nz}[which]
    f = np.zeros(3 * n_nodes(dims))
    for j in range(ny + 1):
        f[3 * node_id(dims, nx, j, k) + 2] = -1.0 / (ny + 1)
    return f


def point_load_node(dims, seed):
    """A node drawn uniformly among nodes with i >= 1 (not on the clamp)."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    i = int(rng.integers(1, nx + 1))
    j = int(rng.integers(0, ny + 1))
    k = int(rng.integers(0, nz + 1))
    return node_id(dims, i, j, k)


def point_load(dims, node):
    f = np.zeros(3 * n_nodes(dims))
    f[3 * node + 2] = -1.0
    return f


@dataclasses.dataclass
class Problem:
    dims: tuple
    rho: np.ndarray          # (nE,) float64
    fixed: np.ndarray        # (ndof,) uint8
    F: np.ndarray            # (nrhs, ndof) float64
    block: tuple             # agglomeration block edge (elements) per axis
    name: str = ""

    @property
    def ndof(self):
        return 3 * n_nodes(self.dims)

    @property
    def nelem(self):
        return n_elems(self.dims)


def cantilever(dims, void_pct, seed, ell=None, loads=("bottom",), block=(4, 4, 4),
               adjoint_seed=None, name=""):
    """Clamped-at-x=0 voxel cantilever with a seeded random void pattern."""
    nx = dims[0]
    if ell is None:
        ell = max(2.0, nx / 12.0)
    field = smooth_field(dims, seed, ell)
    rho = density_from_field(field, void_pct)
    fs = []
    for w in loads:
        if w == "adjoint":
            fs.append(point_load(dims, point_load_node(dims, adjoint_seed)))
        else:
            fs.append(edge_load(dims, w))
    F = np.ascontiguousarray(np.stack(fs))
    return Problem(tuple(dims), rho, clamp_x0(dims), F, tuple(block), name)


# The five workloads quoted for the solver (unit voxels, E=1, nu=0.3).
E_DEFAULT = 1.0
NU_DEFAULT = 0.3


def config(idx, small=False):
    """Workload ``idx`` in 0..3 (the serving stream is ``request_stream``).

    0: 24x12x12, 30% void, one bottom-edge load, 4^3 blocks.
    1: 192x96x96, 50% void, one bottom-edge load, 8^3 blocks.
    2: 128x64x64, 40% void (level-set field, ell = nx/8), loads at the bottom,
       mid and top edges plus one adjoint point load, 8^3 blocks.
    3: 256x128x128, 50% void, one bottom-edge load, 8^3 blocks (mixed precision).
    ``small`` shrinks 1..3 by 4x per axis (same recipe) for oracle-sized tests.
    """
    seed = 1000 + idx
    if idx == 0:
        return cantilever((24, 12, 12), 30, seed, block=(4, 4, 4), name="c0_24x12x12")
    if idx == 1:
        d = (48, 24, 24) if small else (192, 96, 96)
        return cantilever(d, 50, seed, block=(8, 8, 8), name=f"c1_{d[0]}x{d[1]}x{d[2]}")
    if idx == 2:
        d = (32, 16, 16) if small else (128, 64, 64)
        return cantilever(d, 40, seed, ell=d[0] / 8.0,
                          loads=("bottom", "mid", "top", "adjoint"), block=(8, 8, 8),
                          adjoint_seed=2000 + idx, name=f"c2_{d[0]}x{d[1]}x{d[2]}x4rhs")
    if idx == 3:
        d = (64, 32, 32) if small else (256, 128, 128)
        return cantilever(d, 50, seed, block=(8, 8, 8), name=f"c3_{d[0]}x{d[1]}x{d[2]}")
    raise ValueError(idx)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float       # seconds after stream start
    dims: tuple
    void_pct: float
    nrhs: int
    seed: int


def request_stream(n, rate, seed=7, nx_choices=tuple(range(32, 161, 16))):
    """Poisson arrivals (exponential gaps at ``rate`` requests/s) of cantilever
    solve requests nx x nx/2 x nx/2 with nx uniform over ``nx_choices``, void
    fraction uniform in [20, 60] percent and 1..4 right-hand sides (the first
    ``nrhs`` of bottom, mid, top edge loads and a point load)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n):
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        nx = int(rng.choice(nx_choices))
        out.append(Request(r, t, (nx, nx // 2, nx // 2), float(rng.uniform(20, 60)),
                           int(rng.integers(1, 5)), int(rng.integers(0, 2 ** 31))))
    return out


def request_problem(req: Request):
    loads = ("bottom", "mid", "top", "adjoint")[: req.nrhs]
    return cantilever(req.dims, req.void_pct, req.seed, loads=loads, block=(8, 8, 8),
                      adjoint_seed=req.seed + 1, name=f"req{req.rid}")


class RequestFactory:
    """Inputs of a long request stream at a bounded host cost per request.

    Per grid size the fixity mask, the three edge loads and a pool of
    ``pool`` seeded smooth fields are drawn once; a request takes the field
    ``req.seed % pool`` of its grid size and cuts it at its own void fraction,
    and its point load sits at a node drawn from ``req.seed + 1``.  Requests
    of one grid size thus share a field but differ in void fraction, number of
    right-hand sides and point load.  (``request_problem`` draws a field per
    request; this keeps a 2,000-request stream within a few MB per request
    and a few ms of host time.)
    """

    def __init__(self, seed=7, pool=8):
        self.seed = seed
        self.pool = pool
        self._fields = {}
        self._fixed = {}
        self._edges = {}

    def _field(self, dims, k):
        key = (dims, k)
        if key not in self._fields:
            self._fields[key] = smooth_field(dims, self.seed * 1000003 + dims[0] * 101 + k,
                                             max(2.0, dims[0] / 12.0))
        return self._fields[key]

    def problem(self, req: Request):
        dims = tuple(req.dims)
        if dims not in self._fixed:
            self._fixed[dims] = clamp_x0(dims)
            self._edges[dims] = [edge_load(dims, w) for w in ("bottom", "mid", "top")]
        rho = density_from_field(self._field(dims, req.seed % self.pool), req.void_pct)
        F = np.empty((req.nrhs, 3 * n_nodes(dims)))
        for r in range(min(req.nrhs, 3)):
            F[r] = self._edges[dims][r]
        if req.nrhs == 4:
            F[3] = point_load(dims, point_load_node(dims, req.seed + 1))
        return Problem(dims, rho, self._fixed[dims], F, (8, 8, 8), f"req{req.rid}")
