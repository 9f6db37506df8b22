"""Oracle of the linear buckling analysis and its sensitivity (Eq. 3.5, the
buckling constraints of Eq. 3.21 / 3.24-3.25).  TEST INFRASTRUCTURE ONLY.

Linear buckling: for the stress state sigma of the static solution under the
applied loads, the load factor lambda at which (K + lambda K_sigma) phi = 0
has a nontrivial solution; the critical load is lambda times the applied
load.  Readings used here (the paper cites an assembly-free buckling method
without giving it):

* the element geometric stiffness uses the element's centroid stress (the
  stress of stress.element_stress, constant over the element), and the
  ersatz void (elements whose scale is below 1/2) carries none: its scaled
  stress times its ~1/rho_e larger strains would otherwise give spurious
  local modes at load factors near zero in the void, the pseudo-mode effect
  of buckling on ersatz material (prebuckling_stress):
  K_sigma,e[(a,i),(b,j)] = delta_ij sum_pq S_pq int dN_a/dx_p dN_b/dx_q dV,
  S the 3x3 stress tensor; the integrals are products of the 1-D stiffness,
  mass and mixed integrals, as for Ke;
* the smallest positive lambda: the largest positive mu of
  -K_sigma phi = mu K phi on the free DOFs (K is positive definite there),
  lambda = 1 / mu; phi normalised by phi^T K phi = 1;
* the sensitivity field by the element route of Sec. 3.1 (Eq. 3.5, written
  there with the opposite sign convention for K_sigma): with the prebuckling
  stresses held (they scale with rho_e, so K_sigma,e does), the drop of
  lambda when element e loses stiffness, T_P(e) = rho_e d lambda / d rho_e
  = lambda phi_e^T (rho_e Ke + lambda K_sigma,e) phi_e / (phi^T K phi).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, stress


def prebuckling_stress(dims, rho, u, h=(1.0, 1.0, 1.0), E=1.0, nu=0.3):
    """(nE, 6) centroid stresses of the static field u, zero on void elements
    (scale below 1/2)."""
    sig = stress.element_stress(dims, rho, u, h, E, nu)
    sig[np.asarray(rho) < 0.5] = 0.0
    return sig


def grad_tables(h=(1.0, 1.0, 1.0)):
    """G[p][q][a][b] = int dN_a/dx_p dN_b/dx_q over the voxel (LOCAL order)."""
    S1 = lambda hh: np.array([[1.0, -1.0], [-1.0, 1.0]]) / hh   # int phi_a' phi_b'
    M1 = lambda hh: np.array([[2.0, 1.0], [1.0, 2.0]]) * hh / 6  # int phi_a phi_b
    C1 = np.array([[-0.5, -0.5], [0.5, 0.5]])                   # int phi_a' phi_b
    G = np.zeros((3, 3, 8, 8))
    for p in range(3):
        for q in range(3):
            for a in range(8):
                for b in range(8):
                    v = 1.0
                    for ax in range(3):
                        ia, ib = fem.LOCAL[a][ax], fem.LOCAL[b][ax]
                        if ax == p and ax == q:
                            v *= S1(h[ax])[ia, ib]
                        elif ax == p:
                            v *= C1[ia, ib]
                        elif ax == q:
                            v *= C1[ib, ia]
                        else:
                            v *= M1(h[ax])[ia, ib]
                    G[p, q, a, b] = v
    return G


def stress_tensor(sig6):
    sx, sy, sz, tyz, txz, txy = sig6
    return np.array([[sx, txy, txz], [txy, sy, tyz], [txz, tyz, sz]])


def kg_element(S, h=(1.0, 1.0, 1.0), G=None):
    """24x24 geometric stiffness of a voxel under a constant 3x3 stress S."""
    G = grad_tables(h) if G is None else G
    w = np.einsum("pq,pqab->ab", S, G)
    return np.kron(w, np.eye(3))


def kg_gauss(S, h=(1.0, 1.0, 1.0)):
    """The same by 2x2x2 Gauss quadrature of grad(N)^T S grad(N) (exact for it)."""
    g = 1.0 / np.sqrt(3.0)
    sgn = 2 * fem.LOCAL - 1
    detJ = h[0] * h[1] * h[2] / 8.0
    w = np.zeros((8, 8))
    for xi in (-g, g):
        for eta in (-g, g):
            for zeta in (-g, g):
                dN = np.zeros((8, 3))
                for a in range(8):
                    sx, sy, sz = sgn[a]
                    dN[a, 0] = sx * (1 + sy * eta) * (1 + sz * zeta) / 8.0 * (2.0 / h[0])
                    dN[a, 1] = sy * (1 + sx * xi) * (1 + sz * zeta) / 8.0 * (2.0 / h[1])
                    dN[a, 2] = sz * (1 + sx * xi) * (1 + sy * eta) / 8.0 * (2.0 / h[2])
                w += dN @ S @ dN.T * detJ
    return np.kron(w, np.eye(3))


def assemble_kg(dims, sig, h=(1.0, 1.0, 1.0)):
    """Global geometric stiffness from per-element centroid stresses (nE, 6)."""
    G = grad_tables(h)
    dm = fem.dofmap(dims)
    ndof = 3 * fem.n_nodes(dims)
    vals = np.stack([kg_element(stress_tensor(s), h, G) for s in sig])
    r = np.repeat(dm, 24, axis=1).ravel()
    c = np.tile(dm, (1, 24)).ravel()
    K = sp.csr_matrix((vals.ravel(), (r, c)), shape=(ndof, ndof))
    K.sum_duplicates()
    return K


def buckling_modes(K, Kg, fixed, nev=1):
    """The nev smallest positive load factors (ascending) and their modes,
    phi^T K phi = 1, zero on fixed DOFs."""
    Kff, free = fem.constrained_operator(K, fixed)
    Gff, _ = fem.constrained_operator(Kg, fixed)
    if free.size <= 3000:
        mu, V = sla.eigh(-Gff.toarray(), Kff.toarray())
        order = np.argsort(mu)[::-1]
    else:
        mu, V = spla.eigsh(-Gff.tocsc(), k=nev + 2, M=Kff.tocsc(), which="LA")
        order = np.argsort(mu)[::-1]
    mu, V = mu[order[:nev]], V[:, order[:nev]]
    assert np.all(mu > 0), "no positive buckling load factor"
    Phi = np.zeros((nev, K.shape[0]))
    for i in range(nev):
        v = V[:, i] / np.sqrt(V[:, i] @ (Kff @ V[:, i]))
        Phi[i, free] = v
    return 1.0 / mu, Phi


def buckling_sensitivity(dims, rho, Ke, sig, lam, phi, h=(1.0, 1.0, 1.0)):
    """T_P(e) = lambda phi_e^T (rho_e Ke + lambda K_sigma,e) phi_e (phi^T K phi = 1)."""
    G = grad_tables(h)
    dm = fem.dofmap(dims)
    pe = phi[dm]
    ke_term = rho * np.einsum("ei,ij,ej->e", pe, Ke, pe)
    kg_term = np.array([pe[e] @ kg_element(stress_tensor(sig[e]), h, G) @ pe[e] for e in range(len(rho))])
    return lam * (ke_term + lam * kg_term)
