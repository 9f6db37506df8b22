"""Oracle of the modal (eigenvalue) analysis and its sensitivity (Eq. 3.4,
Eq. 3.21's eigenvalue constraint).  TEST INFRASTRUCTURE ONLY.

The paper constrains the lowest eigenvalue lambda of the free vibration
problem K phi = lambda M phi (Eq. 3.21) and uses the topological sensitivity
of Eq. 3.4, sigma:eps - omega^2 rho |u|^2: the strain energy of the mode minus
its kinetic term.  Readings used here:

* M is the consistent mass matrix of the hex8 voxel, M_e = rho_m
  int N^T N dV (per component; the product over the axes of the 1-D mass
  matrices h/6 [[2, 1], [1, 2]]), with unit mass density, and each element's
  mass scaled by the same ersatz factor rho_e as its stiffness (so void
  regions carry no artificial low-frequency modes);
* the constrained problem is K_ff phi = lambda M_ff phi on the free DOFs
  (phi = 0 on fixed DOFs), phi normalised by phi^T M phi = 1;
* the sensitivity field is the element route of Sec. 3.1 applied to Eq. 3.4:
  T_lambda(e) = rho_e phi_e^T (Ke - lambda Me) phi_e, the drop of lambda when
  element e loses its stiffness and mass (d lambda / d rho_e times rho_e, for
  a simple eigenvalue).

The reference eigenpairs come from a dense symmetric-definite eigensolver on
small meshes and from scipy's shift-invert Lanczos (ARPACK) otherwise.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import fem


def me_exact(h=(1, 1, 1)):
    """24x24 consistent mass matrix (unit density) in exact rationals:
    Me[(a,i),(b,j)] = delta_ij prod_axes M1(a_k, b_k), M1 = h/6 [[2, 1], [1, 2]]."""
    hs = [Fraction(v) for v in h]
    M = [[Fraction(0)] * 24 for _ in range(24)]
    for a in range(8):
        for b in range(8):
            v = Fraction(1)
            for ax in range(3):
                v *= hs[ax] * (Fraction(2, 6) if fem.LOCAL[a][ax] == fem.LOCAL[b][ax] else Fraction(1, 6))
            for i in range(3):
                M[3 * a + i][3 * b + i] = v
    return M


def me_gauss(h=(1.0, 1.0, 1.0)):
    """The same matrix by 2x2x2 Gauss quadrature of N^T N (exact for it)."""
    g = 1.0 / np.sqrt(3.0)
    sgn = 2 * fem.LOCAL - 1
    detJ = h[0] * h[1] * h[2] / 8.0
    M = np.zeros((24, 24))
    for xi in (-g, g):
        for eta in (-g, g):
            for zeta in (-g, g):
                N = (1 + sgn[:, 0] * xi) * (1 + sgn[:, 1] * eta) * (1 + sgn[:, 2] * zeta) / 8.0
                Nm = np.zeros((3, 24))
                for a in range(8):
                    Nm[:, 3 * a:3 * a + 3] = N[a] * np.eye(3)
                M += Nm.T @ Nm * detJ
    return M


def lowest_modes(K, M, fixed, nev=1):
    """(eigenvalues ascending, M-normalised eigenvectors as rows) of the
    constrained problem, zero on fixed DOFs."""
    Kff, free = fem.constrained_operator(K, fixed)
    Mff, _ = fem.constrained_operator(M, fixed)
    if free.size <= 3000:
        lam, V = sla.eigh(Kff.toarray(), Mff.toarray(), subset_by_index=[0, nev - 1])
    else:
        lam, V = spla.eigsh(Kff.tocsc(), k=nev, M=Mff.tocsc(), sigma=0.0, which="LM")
        order = np.argsort(lam)
        lam, V = lam[order], V[:, order]
    Phi = np.zeros((nev, K.shape[0]))
    for i in range(nev):
        v = V[:, i] / np.sqrt(V[:, i] @ (Mff @ V[:, i]))
        Phi[i, free] = v
    return lam, Phi


def eigen_sensitivity(dims, rho, Ke, Me, lam, phi):
    """T_lambda(e) = rho_e phi_e^T (Ke - lambda Me) phi_e."""
    dm = fem.dofmap(dims)
    pe = phi[dm]
    return rho * (np.einsum("ei,ij,ej->e", pe, Ke, pe) - lam * np.einsum("ei,ij,ej->e", pe, Me, pe))
