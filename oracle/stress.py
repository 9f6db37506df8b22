"""Oracle of the p-norm von Mises stress constraint (Eq. 3.3, 3.21, 3.23).
TEST INFRASTRUCTURE ONLY.

Readings of the paper used here (it names the quantity, the p-norm of the
von Mises stress, and its topological sensitivity built from the primal
field and an adjoint field, but not the discrete forms):

* element stress at the centroid of the voxel, sigma_e = rho_e D B_c u_e
  (B_c the strain-displacement matrix at the centre; the ersatz scale rho_e
  scales the constitutive matrix as it scales the stiffness);
* von Mises stress vm_e = sqrt(sigma^T V sigma) with V the usual quadratic
  form (sx^2 + sy^2 + sz^2 - sx sy - sy sz - sz sx + 3 (tyz^2 + txz^2 + txy^2));
* the p-norm over every element and every load case,
  sigma_PN = (sum_k sum_e vm_{e,k}^p)^(1/p), p = 8 unless given;
* the adjoint right-hand side of load case k is d sigma_PN / d u_k
  = sigma_PN^(1-p) sum_e vm_e^(p-2) rho_e B_c^T D V sigma_e (scattered to the
  element's DOFs, zero on fixed DOFs), and the adjoint field lambda_k solves
  K lambda_k = that right-hand side;
* the sensitivity field (the element route of Sec. 3.1 applied to Eq. 3.3,
  whose printed trace term mixes the primal and adjoint fields):
  T_sigma(e) = sum_k rho_e lambda_{k,e}^T Ke u_{k,e}, the mutual energy of the
  primal and adjoint fields, i.e. the change of sigma_PN through the
  displacements when element e loses its stiffness.
"""
from __future__ import annotations

import numpy as np

from . import fem, post


def centroid_B(h=(1.0, 1.0, 1.0)):
    """6 x 24 strain-displacement matrix at the voxel centre (Voigt xx, yy,
    zz, yz, xz, xy with engineering shears; local node order of fem.LOCAL)."""
    B = np.zeros((6, 24))
    for a, (dx, dy, dz) in enumerate(fem.LOCAL):
        gx, gy, gz = (2 * dx - 1) / (4.0 * h[0]), (2 * dy - 1) / (4.0 * h[1]), (2 * dz - 1) / (4.0 * h[2])
        c = 3 * a
        B[0, c] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c + 1] = gz
        B[3, c + 2] = gy
        B[4, c] = gz
        B[4, c + 2] = gx
        B[5, c] = gy
        B[5, c + 1] = gx
    return B


def element_stress(dims, rho, u, h=(1.0, 1.0, 1.0), E=1.0, nu=0.3):
    """(nE, 6) centroid stresses rho_e D B_c u_e."""
    ue = u[fem.dofmap(dims)]
    eps = ue @ centroid_B(h).T
    return rho[:, None] * (eps @ fem.elasticity_D(E, nu).T)


def von_mises(sig):
    sx, sy, sz, tyz, txz, txy = sig.T
    return np.sqrt(sx * sx + sy * sy + sz * sz - sx * sy - sy * sz - sz * sx + 3.0 * (tyz * tyz + txz * txz + txy * txy))


def pnorm(U, dims, rho, p=8.0, h=(1.0, 1.0, 1.0), E=1.0, nu=0.3):
    """sigma_PN over every element and every row of U (load cases)."""
    s = sum(float(np.sum(von_mises(element_stress(dims, rho, u, h, E, nu)) ** p)) for u in np.atleast_2d(U))
    return s ** (1.0 / p)


def adjoint_rhs(U, dims, rho, fixed, p=8.0, h=(1.0, 1.0, 1.0), E=1.0, nu=0.3):
    """d sigma_PN / d u_k for every row k of U, zero on fixed DOFs."""
    U = np.atleast_2d(U)
    spn = pnorm(U, dims, rho, p, h, E, nu)
    B = centroid_B(h)
    D = fem.elasticity_D(E, nu)
    dm = fem.dofmap(dims)
    out = np.zeros_like(U)
    for k, u in enumerate(U):
        sig = element_stress(dims, rho, u, h, E, nu)
        vm = von_mises(sig)
        sx, sy, sz, tyz, txz, txy = sig.T
        vsig = np.stack([sx - 0.5 * (sy + sz), sy - 0.5 * (sx + sz), sz - 0.5 * (sx + sy),
                         3.0 * tyz, 3.0 * txz, 3.0 * txy], axis=1)   # V sigma = d(vm^2)/d sigma / 2
        t = (rho * vm ** (p - 2.0))[:, None] * (vsig @ D.T)
        np.add.at(out[k], dm.ravel(), (t @ B).ravel())
        out[k] *= spn ** (1.0 - p)
    out[:, np.asarray(fixed) != 0] = 0.0
    return out


def stress_field(dims, rho, Ke, U, Lam):
    """T_sigma = sum_k rho_e lambda_k,e^T Ke u_k,e (mutual energies)."""
    return sum(post.element_energy(dims, rho, Ke, u, lam) for u, lam in zip(np.atleast_2d(U), np.atleast_2d(Lam)))
