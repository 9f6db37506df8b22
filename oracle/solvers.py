"""Oracle solvers for K_ff u_f = f_f.  TEST INFRASTRUCTURE ONLY.

The method solves the static problem of Eq. 1.1 with an assembly-free deflated
conjugate gradient (Sec. 3.5).  Whatever the solver, the converged result is
the solution of the constrained linear system, so the oracle's reference is
that system solved directly on the assembled matrix (dense Cholesky or
SuperLU).  For sizes a CPU cannot factor, and to check the iteration itself,
the textbook Jacobi-preconditioned CG and the deflated PCG (Saad, Yeung,
Erhel and Guyomarc'h, 2000) are written out on the assembled matrix.

The deflation space W holds the six rigid-body motions of each agglomerated
block of elements.  Node i (per axis) belongs to block min(i // b, nb - 1),
nb = ceil(n_elements / b); the motions are taken about the centre of the
block's node range, in element-unit coordinates divided by the largest block
edge, and are zero on fixed DOFs.
Columns of W that are identically zero are dropped.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


def solve_direct(K, fixed, f):
    """u with K_ff u_f = f_f and u = 0 on fixed DOFs."""
    Kff, free = fem.constrained_operator(K, fixed)
    u = np.zeros(K.shape[0])
    if free.size <= 4000:
        c = sla.cho_factor(Kff.toarray(), lower=True)
        u[free] = sla.cho_solve(c, f[free])
    else:
        lu = spla.splu(Kff.tocsc())
        u[free] = lu.solve(f[free])
    return u


def deflation_basis(dims, fixed, block):
    """Sparse W (ndof x 6*nblocks) and the (I,J,K) index of each block."""
    nn = [d + 1 for d in dims]
    nb = [math.ceil(d / b) for d, b in zip(dims, block)]
    idx = [np.arange(n) for n in nn]
    bid = [np.minimum(ix // b, m - 1) for ix, b, m in zip(idx, block, nb)]
    # centre of each block's node range, per axis
    cen = []
    for ax in range(3):
        lo = np.arange(nb[ax]) * block[ax]
        hi = np.where(np.arange(nb[ax]) == nb[ax] - 1, dims[ax], lo + block[ax] - 1)
        cen.append((lo + hi) / 2.0)
    k, j, i = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    bi, bj, bk = bid[0][i], bid[1][j], bid[2][k]
    blk = bi + nb[0] * (bj + nb[1] * bk)
    sc = float(max(block))  # one scale for all axes keeps the rotations rigid
    x = (i - cen[0][bi]) / sc
    y = (j - cen[1][bj]) / sc
    z = (k - cen[2][bk]) / sc
    nnode = i.size
    one = np.ones(nnode)
    zero = np.zeros(nnode)
    # rows: 3n+c ; columns 6*blk+m
    modes = [  # (ux, uy, uz) of the six motions
        (one, zero, zero), (zero, one, zero), (zero, zero, one),
        (zero, -z, y), (z, zero, -x), (-y, x, zero),
    ]
    rows, cols, vals = [], [], []
    n = np.arange(nnode)
    for m, comp in enumerate(modes):
        for c in range(3):
            v = comp[c]
            nz_ = v != 0
            rows.append(3 * n[nz_] + c)
            cols.append(6 * blk[nz_] + m)
            vals.append(v[nz_])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    keep = np.asarray(fixed)[rows] == 0
    W = sp.csr_matrix((vals[keep], (rows[keep], cols[keep])),
                      shape=(3 * nnode, 6 * nb[0] * nb[1] * nb[2]))
    nzc = np.flatnonzero(np.asarray(abs(W).sum(axis=0)).ravel() > 0)
    return W[:, nzc].tocsr(), nb


def pcg(K, fixed, f, rtol=1e-8, max_iter=100000, x0=None):
    """Jacobi-preconditioned CG on K_ff.  Returns (u, iterations, rel. residual)."""
    Kff, free = fem.constrained_operator(K, fixed)
    b = f[free]
    dinv = 1.0 / Kff.diagonal()
    x = np.zeros_like(b) if x0 is None else x0[free].copy()
    r = b - Kff @ x
    bn = np.linalg.norm(b)
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * bn and it < max_iter:
        q = Kff @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    u = np.zeros(K.shape[0])
    u[free] = x
    return u, it, np.linalg.norm(b - Kff @ x) / bn


def dcg(K, fixed, f, dims, block, rtol=1e-8, max_iter=100000, check=None):
    """Deflated Jacobi-PCG on K_ff (Saad et al. 2000):

    x0 = W E^-1 W^T b, r0 = b - A x0, z = M^-1 r, p0 = z - W E^-1 W^T A z;
    repeat: q = A p, alpha = r.z / p.q, x += alpha p, r -= alpha q,
            z = M^-1 r, beta = r.z_new / r.z_old, mu = E^-1 W^T A z,
            p = beta p + z - W mu,
    with A = K_ff, M = diag(A), E = W^T A W.  ``check(r, W)`` (optional) is
    called on every residual, e.g. to verify that W^T r stays zero.
    Returns (u, iterations, true relative residual).
    """
    Kff, free = fem.constrained_operator(K, fixed)
    Wfull, _ = deflation_basis(dims, fixed, block)
    W = Wfull[free].tocsr()
    AW = (Kff @ W).tocsr()
    E = (W.T @ AW).toarray()
    cf = sla.cho_factor(E, lower=True)

    def coarse(v):
        return sla.cho_solve(cf, v)

    b = f[free]
    dinv = 1.0 / Kff.diagonal()
    bn = np.linalg.norm(b)
    x = W @ coarse(W.T @ b)
    r = b - Kff @ x
    z = dinv * r
    p = z - W @ coarse(AW.T @ z)
    rz = r @ z
    it = 0
    if check is not None:
        check(r, W)
    while np.linalg.norm(r) > rtol * bn and it < max_iter:
        q = Kff @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if check is not None:
            check(r, W)
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = beta * p + z - W @ coarse(AW.T @ z)
        it += 1
    u = np.zeros(K.shape[0])
    u[free] = x
    return u, it, np.linalg.norm(b - Kff @ x) / bn


def coarse_matrix(K, fixed, dims, block):
    """E = W^T K_ff W (dense), with W as in ``deflation_basis`` restricted to
    free DOFs but indexed by ALL 6*nblocks columns (zero columns kept), block
    index = bi + nbx*(bj + nby*bk), mode order (tx, ty, tz, rx, ry, rz)."""
    nn = [d + 1 for d in dims]
    nb = [math.ceil(d / b) for d, b in zip(dims, block)]
    W, _ = _basis_all_columns(dims, fixed, block)
    Kc = K.tocsr().copy()
    fx = np.asarray(fixed) != 0
    # zero fixed rows/cols of K (W is already zero there)
    D = sp.diags((~fx).astype(float))
    Kc = D @ Kc @ D
    return (W.T @ (Kc @ W)).toarray(), nb


def _basis_all_columns(dims, fixed, block):
    nb = [math.ceil(d / b) for d, b in zip(dims, block)]
    W, _ = deflation_basis(dims, np.zeros_like(fixed), block)
    fx = np.asarray(fixed) != 0
    D = sp.diags((~fx).astype(float))
    return (D @ W).tocsr(), nb
