"""Oracle finite element model: hex8 element matrix, voxel mesh indexing and
global assembly.  TEST INFRASTRUCTURE ONLY (see the package header).

The paper discretises the design domain with hexahedral elements (Sec. 3.8,
step 1) and solves the linear static problem ``K u = f`` (Eq. 1.1).  The
element matrix used for its element sensitivities is ``K^e`` (Eq. 3.5).  Here
the domain is a box of ``nx*ny*nz`` voxels of size ``hx*hy*hz``; element
``e`` has stiffness ``rho_e * Ke`` (``rho_e`` = 1 for solid, a small ersatz
value for void), all elements sharing one ``Ke``.

Two independent constructions of ``Ke`` are provided:

* ``ke_gauss``: the textbook ``sum_g w_g B_g^T D B_g det J`` over a 2x2x2
  Gauss-Legendre rule (exact for the trilinear hexahedron on a box);
* ``ke_exact``: exact rational arithmetic (``fractions.Fraction``) from the
  bilinear form ``lambda div u div v + 2 mu eps(u):eps(v)`` written as
  products of 1-D integrals.  Used only to pin ``ke_gauss``.
"""
from __future__ import annotations

from fractions import Fraction
import itertools

import numpy as np
import scipy.sparse as sp

# Local node order of the hexahedron: bottom face counter-clockwise, then top.
LOCAL = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                  (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)], dtype=np.int64)


def lame(E, nu):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def elasticity_D(E, nu):
    """Isotropic 6x6 constitutive matrix, Voigt order xx, yy, zz, yz, xz, xy
    with engineering shear strains."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def ke_gauss(h=(1.0, 1.0, 1.0), E=1.0, nu=0.3):
    """24x24 FP64 element stiffness by 2x2x2 Gauss quadrature of B^T D B."""
    hx, hy, hz = h
    D = elasticity_D(E, nu)
    g = 1.0 / np.sqrt(3.0)
    sgn = 2 * LOCAL - 1  # node position in the reference cube [-1, 1]^3
    Ke = np.zeros((24, 24))
    detJ = hx * hy * hz / 8.0
    for xi, eta, zeta in itertools.product((-g, g), repeat=3):
        dN = np.zeros((8, 3))  # physical derivatives of each shape function
        for a in range(8):
            sx, sy, sz = sgn[a]
            dN[a, 0] = sx * (1 + sy * eta) * (1 + sz * zeta) / 8.0 * (2.0 / hx)
            dN[a, 1] = sy * (1 + sx * xi) * (1 + sz * zeta) / 8.0 * (2.0 / hy)
            dN[a, 2] = sz * (1 + sx * xi) * (1 + sy * eta) / 8.0 * (2.0 / hz)
        B = np.zeros((6, 24))
        for a in range(8):
            dx, dy, dz = dN[a]
            c = 3 * a
            B[0, c] = dx
            B[1, c + 1] = dy
            B[2, c + 2] = dz
            B[3, c + 1] = dz
            B[3, c + 2] = dy
            B[4, c] = dz
            B[4, c + 2] = dx
            B[5, c] = dy
            B[5, c + 1] = dx
        Ke += B.T @ D @ B * detJ
    return Ke


def ke_exact(h=(1, 1, 1), E=1, nu=Fraction(3, 10)):
    """24x24 element stiffness in exact rationals.

    Ke[(a,i),(b,j)] = lam * G[i][j][a][b] + mu * G[j][i][a][b]
                      + delta_ij * mu * sum_k G[k][k][a][b],
    G[p][q][a][b] = integral of dN_a/dx_p * dN_b/dx_q over the box, each a
    product over the three axes of the 1-D integrals of linear shape functions
    (stiffness S, mass M, mixed C).
    """
    E = Fraction(E)
    nu = Fraction(nu)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    hs = [Fraction(v) for v in h]

    def S(hh):  # int phi_a' phi_b'
        return [[1 / hh, -1 / hh], [-1 / hh, 1 / hh]]

    def M(hh):  # int phi_a phi_b
        return [[hh / 3, hh / 6], [hh / 6, hh / 3]]

    def C(hh):  # int phi_a' phi_b   (phi_0 = 1 - x/h, phi_1 = x/h)
        half = Fraction(1, 2)
        return [[-half, -half], [half, half]]

    def G(p, q, a, b):
        val = Fraction(1)
        for ax in range(3):
            ia, ib = LOCAL[a][ax], LOCAL[b][ax]
            if ax == p and ax == q:
                m = S(hs[ax])[ia][ib]
            elif ax == p:
                m = C(hs[ax])[ia][ib]
            elif ax == q:
                m = C(hs[ax])[ib][ia]
            else:
                m = M(hs[ax])[ia][ib]
            val *= m
        return val

    K = [[Fraction(0)] * 24 for _ in range(24)]
    for a in range(8):
        for b in range(8):
            trace = sum(G(k, k, a, b) for k in range(3))
            for i in range(3):
                for j in range(3):
                    v = lam * G(i, j, a, b) + mu * G(j, i, a, b)
                    if i == j:
                        v += mu * trace
                    K[3 * a + i][3 * b + j] = v
    return K


def rigid_modes_element(h=(1.0, 1.0, 1.0)):
    """24x6 matrix of the six rigid-body motions on the element's nodes."""
    X = LOCAL * np.asarray(h, dtype=float)
    R = np.zeros((24, 6))
    for a in range(8):
        x, y, z = X[a]
        R[3 * a:3 * a + 3, 0:3] = np.eye(3)
        R[3 * a:3 * a + 3, 3] = (0.0, -z, y)
        R[3 * a:3 * a + 3, 4] = (z, 0.0, -x)
        R[3 * a:3 * a + 3, 5] = (-y, x, 0.0)
    return R


# ---------------------------------------------------------------- mesh indexing
def n_nodes(dims):
    nx, ny, nz = dims
    return (nx + 1) * (ny + 1) * (nz + 1)


def connectivity(dims):
    """(nE, 8) global node ids of each element in LOCAL order."""
    nx, ny, nz = dims
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    conn = np.empty((ex.size, 8), dtype=np.int64)
    for a, (dx, dy, dz) in enumerate(LOCAL):
        conn[:, a] = (ex + dx) + (nx + 1) * ((ey + dy) + (ny + 1) * (ez + dz))
    return conn


def dofmap(dims):
    conn = connectivity(dims)
    return (3 * conn[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 24)


def node_coords(dims, h=(1.0, 1.0, 1.0)):
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return np.stack([i.ravel() * h[0], j.ravel() * h[1], k.ravel() * h[2]], axis=1)


def assemble(dims, rho, Ke, chunk=1 << 18):
    """Global stiffness K = sum_e rho_e P_e^T Ke P_e as CSR (duplicates summed)."""
    dm = dofmap(dims)
    ndof = 3 * n_nodes(dims)
    parts = []
    for s in range(0, dm.shape[0], chunk):
        d = dm[s:s + chunk]
        r = np.repeat(d, 24, axis=1).ravel()
        c = np.tile(d, (1, 24)).ravel()
        v = (rho[s:s + chunk, None, None] * Ke[None, :, :]).ravel()
        parts.append(sp.csr_matrix((v, (r, c)), shape=(ndof, ndof)))
    K = parts[0]
    for p in parts[1:]:
        K = K + p
    K.sum_duplicates()
    return K.tocsr()


def apply_ebe(dims, rho, Ke, u):
    """K u element by element (einsum + scatter-add), for meshes too large
    to assemble.  Same definition as ``assemble(...) @ u``."""
    dm = dofmap(dims)
    ue = u[dm]                                   # (nE, 24)
    ye = np.einsum("ij,ej->ei", Ke, ue) * rho[:, None]
    y = np.zeros_like(u)
    np.add.at(y, dm.ravel(), ye.ravel())
    return y


def constrained_operator(K, fixed):
    """The free-free block K_ff and the free-DOF index array."""
    free = np.flatnonzero(np.asarray(fixed) == 0)
    return K[free][:, free].tocsr(), free


def apply_constrained(K, fixed, u):
    """The operator the solver iterates with, on the full DOF vector:
    K_ff on free DOFs (fixed inputs treated as zero), identity on fixed DOFs."""
    fx = np.asarray(fixed) != 0
    uf = np.where(fx, 0.0, u)
    y = K @ uf
    return np.where(fx, u, y)


def apply_at_nodes(dims, rho, Ke, u, nodes, fixed=None):
    """(A u) at the listed nodes only, one node at a time: the sum over the
    (up to 8) elements touching each node of rho_e (Ke u_e) at that node's
    local position; free/fixed handling as in ``apply_constrained``.
    Returns an array (len(nodes), 3)."""
    nx, ny, nz = dims
    fx = None if fixed is None else (np.asarray(fixed) != 0)
    out = np.zeros((len(nodes), 3))
    for q, n in enumerate(nodes):
        i = n % (nx + 1)
        j = (n // (nx + 1)) % (ny + 1)
        k = n // ((nx + 1) * (ny + 1))
        acc = np.zeros(3)
        for a, (dx, dy, dz) in enumerate(LOCAL):
            ex, ey, ez = i - dx, j - dy, k - dz
            if not (0 <= ex < nx and 0 <= ey < ny and 0 <= ez < nz):
                continue
            e = ex + nx * (ey + ny * ez)
            ue = np.empty(24)
            for b, (bx, by, bz) in enumerate(LOCAL):
                m = (ex + bx) + (nx + 1) * ((ey + by) + (ny + 1) * (ez + bz))
                ue[3 * b:3 * b + 3] = u[3 * m:3 * m + 3]
                if fx is not None:
                    ue[3 * b:3 * b + 3] *= ~fx[3 * m:3 * m + 3]
            acc += rho[e] * (Ke[3 * a:3 * a + 3, :] @ ue)
        if fx is not None:
            acc = np.where(fx[3 * n:3 * n + 3], u[3 * n:3 * n + 3], acc)
        out[q] = acc
    return out
