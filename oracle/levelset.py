"""Oracle of the augmented topological level-set loop (Sec. 3.2-3.4, 3.6,
3.8, Fig. 6-7).  TEST INFRASTRUCTURE ONLY.

The loop traces the Pareto curve of minimum volume from the full design
domain downward.  At a target volume fraction v it iterates a fixed point
(Fig. 6): finite element solve over the current topology, topological
sensitivity fields, the augmented topological level-set, and the topology at
v extracted from it.  The constraints g_i <= 0 enter through the augmented
Lagrangian multipliers mu_i and penalties gamma_i (Eq. 3.11-3.12, 3.17-3.18).
Once a topology has converged, v is lowered by dv; when a hard constraint is
violated (or the fixed point does not settle), the loop returns to the last
converged feasible topology and halves dv, and it stops when dv falls below
dv_min (Sec. 3.8 steps 1-9).

Readings of the paper used here (it leaves these open):

* g_i = Q_i / (alpha_i Q_i0) - 1 for a constraint Q_i <= alpha_i Q_i0
  (Eq. 3.21), Q_i0 its value on the full domain; the compliance Q = J is the
  sum of f_k . u_k over the load cases, its field the sum of the element
  strain energies rho_e u_e^T Ke u_e (the element route of Sec. 3.1).
* Augmented level set (Eq. 3.17-3.18, the product in Eq. 3.18 read as
  (mu_i + gamma_i g_i) T_gi): T_L = sum_i w_i T_gi with
  w_i = max(mu_i + gamma_i g_i, 0) and T_gi = T_Qi / (alpha_i Q_i0).  The
  objective's term T_phi (volume) is the same at every point, so it shifts
  the field without reordering it and is left out; if every w_i is 0 the
  constraint fields are taken with weight 1 each.
* Multiplier and penalty updates after every solve k (k = 0 on the full
  domain), from the values before the update: mu <- max(mu + gamma g_k, 0);
  gamma is kept at k = 0 and otherwise updated by Eq. 3.12 as printed, with
  min(g_k, 0) <= varsigma min(g_{k-1}, 0) keeping it and else
  gamma <- max(eta gamma, k^2).
* Step 7's convergence: two successive solves at the same target v whose
  compliances differ by less than conv_tol (1%) of the earlier one; the
  full domain (v = 1) counts as converged; max_fp solves at one target
  without convergence count as a divergence (step 9).
* Step 9: back to the last converged feasible topology (volume v_b), dv
  halved, next target v_b - dv, extracted from that topology's level set;
  termination when dv < dv_min or the next target would be <= 0.
* With the p-norm stress constraint sigma_PN <= alpha_sigma sigma_PN0
  (Eq. 3.23, see stress.py) a second term joins: g_s, its own mu_s and
  gamma_s (same rules, same start values), T_L = w_J T_J / (alpha_J J0) +
  w_s T_sigma / (alpha_sigma sigma_PN0); a violated stress constraint is a
  hard violation like the compliance one.
* With the eigenvalue constraint lambda_1 >= alpha_lambda lambda_10 (Eq. 3.21;
  lambda_1 the lowest eigenvalue of K phi = lambda M phi, see modal.py, void
  elements scaled in mass as in stiffness) a further term joins with
  g_l = 1 - lambda_1 / (alpha_lambda lambda_10), its own mu_l and gamma_l (same
  rules, same start values) and the field T_lambda / (alpha_lambda
  lambda_10), T_lambda(e) = rho_e phi_e^T (Ke - lambda_1 Me) phi_e the drop of
  lambda_1 when element e loses its stiffness and mass (modal.py): like the
  compliance and stress fields, the increase of g when e is removed.  A
  violated eigenvalue constraint is a hard violation; step 7's convergence
  test stays on the compliance.
* With the buckling constraint P >= alpha_P P_0 (Eq. 3.21) a further term
  joins in the same way: P the smallest positive load factor of the stress
  state of load case 0 (buckling.py: the ersatz void carries no stress
  stiffness), g_p = 1 - P / (alpha_P P_0), its own mu_p and gamma_p, the
  field T_P / (alpha_P P_0) with T_P the load-factor field of buckling.py
  (the drop of P when an element loses stiffness, its prebuckling stress
  scaled with it).
* Hard and soft constraints (Sec. 3.6, Eq. 3.20-3.21): a soft constraint
  (the eigenvalue one with lambda_soft, the buckling one with P_soft) keeps its multiplier, penalty and
  level-set term, but its violation neither sends the loop back nor ends it:
  it shapes the topology without bounding the feasible space.
* Topology at v (Eq. 3.6): the ceil(v nE) elements of highest T_L (ties by
  index; with the casting constraint of Sec. 3.7 the projected field, ties by
  the distance to the parting plane, then index); void elements get the
  ersatz scale.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import buckling, fem, modal, post, solvers, stress
from .casting import cast_project, parting_distance

FEA_FIXED_POINT = 0   # a fixed-point solve at the current target
FEA_CONVERGED = 1     # converged: the target is lowered by dv
FEA_VIOLATED = 2      # a hard constraint violated: dv halved, back to the last converged design
FEA_DIVERGED = 3      # max_fp solves without convergence: treated as a violation
FEA_TERMINATED = 4    # dv < dv_min or no volume left: the loop ends after this solve


def al_update(mu, gamma, g_new, g_old, k, varsigma=0.25, eta=10.0):
    """One multiplier / penalty update after solve k (Eq. 3.11, 3.12).

    g_old is None at k = 0.  Both updates use the values before the update."""
    mu_next = max(mu + gamma * g_new, 0.0)
    if g_old is None or min(g_new, 0.0) <= varsigma * min(g_old, 0.0):
        gamma_next = gamma
    else:
        gamma_next = max(eta * gamma, float(k) ** 2)
    return mu_next, gamma_next


def weights(mu, gamma, g):
    """w_i = max(mu_i + gamma_i g_i, 0), all 1 when every w_i is 0 (Eq. 3.18)."""
    w = [max(m + c * x, 0.0) for m, c, x in zip(mu, gamma, g)]
    if all(x == 0.0 for x in w):
        w = [1.0] * len(w)
    return w


def combined_field(fields, coef):
    """sum_i coef_i fields_i, accumulated in the order of the fields."""
    out = coef[0] * fields[0]
    for c, f in zip(coef[1:], fields[1:]):
        out = out + c * f
    return out


@dataclasses.dataclass
class Params:
    alpha_J: float = 3.0       # J <= alpha_J J0 (Eq. 3.22)
    dv0: float = 0.025         # first volume step (Sec. 4.2)
    dv_min: float = 0.025 / 16
    mu0: float = 100.0         # Sec. 3.8 step 1
    gamma0: float = 10.0
    varsigma: float = 0.25     # Eq. 3.12
    eta: float = 10.0
    conv_tol: float = 0.01     # step 7: change in compliance
    max_fp: int = 8
    max_fea: int = 400
    void_scale: float = 1e-3
    cast_axis: int = -1        # casting constraint (Sec. 3.7): axis, or -1 for none
    cast_parting: int = 0
    alpha_sigma: float = 0.0   # sigma_PN <= alpha_sigma sigma_PN0 (Eq. 3.23); <= 0: no stress constraint
    pnorm_p: float = 8.0
    damping: bool = False      # extract from the mean of this level set and the one the topology came from
    alpha_lambda: float = 0.0  # lambda_1 >= alpha_lambda lambda_10 (Eq. 3.21); <= 0: no eigenvalue constraint
    lambda_soft: bool = False  # the eigenvalue constraint as a soft one (Sec. 3.6)
    alpha_P: float = 0.0       # P >= alpha_P P_0 (Eq. 3.21), load case 0; <= 0: no buckling constraint
    P_soft: bool = False       # the buckling constraint as a soft one


@dataclasses.dataclass
class Record:
    fea: int
    event: int
    v: float          # target volume fraction of the analysed topology
    nsolid: int
    J: float
    g: float
    mu: float         # after the update
    gamma: float
    dv: float         # step after this solve's decision
    S: float = 0.0    # stress p-norm (0 without the stress constraint)
    g_s: float = 0.0
    mu_s: float = 0.0
    gamma_s: float = 0.0
    lam: float = 0.0  # lowest eigenvalue (0 without the eigenvalue constraint)
    g_l: float = 0.0
    mu_l: float = 0.0
    gamma_l: float = 0.0
    P: float = 0.0    # smallest buckling load factor (0 without the buckling constraint)
    g_p: float = 0.0
    mu_p: float = 0.0
    gamma_p: float = 0.0


def extract(field, vol, dims, p: Params):
    """Solid mask (uint8) at volume fraction vol from a level-set field."""
    if p.cast_axis >= 0:
        f = cast_project(field, dims, p.cast_axis, p.cast_parting)
        solid, _ = post.threshold(f, vol, parting_distance(dims, p.cast_axis, p.cast_parting))
    else:
        solid, _ = post.threshold(field, vol)
    return solid


def density(solid, p: Params):
    return np.where(solid == 1, 1.0, p.void_scale)


def fea(dims, solid, fixed, F, Ke, p: Params):
    """Displacements of every load case on the topology, by direct solves."""
    K = fem.assemble(dims, density(solid, p), Ke)
    return np.stack([solvers.solve_direct(K, fixed, F[r]) for r in range(F.shape[0])])


def compliance_field(dims, solid, Ke, U, p: Params):
    rho = density(solid, p)
    return sum(post.element_energy(dims, rho, Ke, U[r]) for r in range(U.shape[0]))


def stress_quantities(dims, solid, fixed, Ke, U, p: Params):
    """sigma_PN over the load cases and its sensitivity field (the mutual
    energies of the primal and adjoint fields), by direct adjoint solves."""
    rho = density(solid, p)
    S = stress.pnorm(U, dims, rho, p.pnorm_p)
    B = stress.adjoint_rhs(U, dims, rho, fixed, p.pnorm_p)
    K = fem.assemble(dims, rho, Ke)
    Lam = np.stack([solvers.solve_direct(K, fixed, b) for b in B])
    return S, stress.stress_field(dims, rho, Ke, U, Lam)


def eigen_quantities(dims, solid, fixed, Ke, Me, p: Params):
    """The lowest eigenvalue of the topology and its sensitivity field."""
    rho = density(solid, p)
    K = fem.assemble(dims, rho, Ke)
    M = fem.assemble(dims, rho, Me)
    lam, Phi = modal.lowest_modes(K, M, fixed, 1)
    return float(lam[0]), modal.eigen_sensitivity(dims, rho, Ke, Me, lam[0], Phi[0])


def buckling_quantities(dims, solid, fixed, Ke, U, p: Params):
    """The smallest buckling load factor of load case 0 and its field."""
    rho = density(solid, p)
    sig = buckling.prebuckling_stress(dims, rho, U[0])
    K = fem.assemble(dims, rho, Ke)
    lam, Phi = buckling.buckling_modes(K, buckling.assemble_kg(dims, sig), fixed, 1)
    return float(lam[0]), buckling.buckling_sensitivity(dims, rho, Ke, sig, lam[0], Phi[0])


class Loop:
    """The loop as a state machine: ``first()`` gives the full domain; after
    each solve, ``after_solve(solid, J, field)`` records it and returns the
    next topology to analyse (None at the end).  ``run`` drives it with the
    oracle's direct solves."""

    def __init__(self, dims, p: Params):
        self.dims = tuple(dims)
        self.p = p
        self.n = int(np.prod(dims))
        self.mu, self.gamma = p.mu0, p.gamma0
        self.mu_s, self.gamma_s = p.mu0, p.gamma0
        self.mu_l, self.gamma_l = p.mu0, p.gamma0
        self.L0 = None
        self.gl_prev = None
        self.mu_p, self.gamma_p = p.mu0, p.gamma0
        self.P0 = None
        self.gp_prev = None
        self.dv = p.dv0
        self.k = 0
        self.J0 = None
        self.S0 = None
        self.g_prev = None
        self.gs_prev = None
        self.v = 1.0               # target of the topology being analysed
        self.fp = 0                # solves at the current target
        self.J_prev_same = None    # compliance of the previous solve at this target
        self.best = None           # (solid, v, J, field) of the last converged feasible design
        self.history = []
        self.last_extract = None   # (field, volume fraction) of the last extraction
        self.src = None            # the level set the topology being analysed was extracted from

    def first(self):
        return np.ones(self.n, dtype=np.uint8)

    def after_solve(self, solid, J, field_J, S=None, field_S=None, lam=None, field_lam=None, P=None, field_P=None):
        p = self.p
        k, v = self.k, self.v
        stress = p.alpha_sigma > 0
        eigen = p.alpha_lambda > 0
        buck = p.alpha_P > 0
        if k == 0:
            self.J0 = J
            self.S0 = S
            self.L0 = lam
            self.P0 = P
        g = J / (p.alpha_J * self.J0) - 1.0
        mu, gamma = al_update(self.mu, self.gamma, g, self.g_prev, k, p.varsigma, p.eta)
        self.mu, self.gamma, self.g_prev = mu, gamma, g
        g_s = 0.0
        if stress:
            g_s = S / (p.alpha_sigma * self.S0) - 1.0
            self.mu_s, self.gamma_s = al_update(self.mu_s, self.gamma_s, g_s, self.gs_prev, k, p.varsigma, p.eta)
            self.gs_prev = g_s
        g_l = 0.0
        if eigen:
            g_l = 1.0 - lam / (p.alpha_lambda * self.L0)
            self.mu_l, self.gamma_l = al_update(self.mu_l, self.gamma_l, g_l, self.gl_prev, k, p.varsigma, p.eta)
            self.gl_prev = g_l
        g_p = 0.0
        if buck:
            g_p = 1.0 - P / (p.alpha_P * self.P0)
            self.mu_p, self.gamma_p = al_update(self.mu_p, self.gamma_p, g_p, self.gp_prev, k, p.varsigma, p.eta)
            self.gp_prev = g_p
        self.fp += 1
        if g > 0.0 or g_s > 0.0 or (g_l > 0.0 and not p.lambda_soft) or (g_p > 0.0 and not p.P_soft):
            event = FEA_VIOLATED
        elif k == 0 or self._converged(J):
            event = FEA_CONVERGED
        elif self.fp >= p.max_fp:
            event = FEA_DIVERGED
        else:
            event = FEA_FIXED_POINT
        nxt = None
        if event in (FEA_VIOLATED, FEA_DIVERGED):
            # step 9: back to the last converged feasible design with half the step
            self.dv *= 0.5
            if self.dv < p.dv_min or self.best[1] - self.dv <= 0.0:
                event = FEA_TERMINATED
            else:
                self._target(self.best[1] - self.dv)
                self.last_extract = (self.best[3], self.v)
                self.src = self.best[3]
                nxt = extract(self.best[3], self.v, self.dims, p)
        else:
            # steps 5-6: the augmented level set and the topology extracted from it
            # the active constraints in the order J, stress, eigenvalue, buckling
            mus, gammas, gs, fields, scales = [mu], [gamma], [g], [field_J], [p.alpha_J * self.J0]
            if stress:
                mus.append(self.mu_s), gammas.append(self.gamma_s), gs.append(g_s)
                fields.append(field_S), scales.append(p.alpha_sigma * self.S0)
            if eigen:
                mus.append(self.mu_l), gammas.append(self.gamma_l), gs.append(g_l)
                fields.append(field_lam), scales.append(p.alpha_lambda * self.L0)
            if buck:
                mus.append(self.mu_p), gammas.append(self.gamma_p), gs.append(g_p)
                fields.append(field_P), scales.append(p.alpha_P * self.P0)
            w = weights(mus, gammas, gs)
            field = combined_field(fields, [wi / sc for wi, sc in zip(w, scales)])
            if p.damping and self.src is not None:
                field = 0.5 * (field + self.src)
            if event == FEA_CONVERGED:  # step 8: the next target
                self.best = (solid.copy(), v, J, field)
                if v - self.dv <= 0.0:
                    event = FEA_TERMINATED
                else:
                    self._target(v - self.dv)
                    self.last_extract = (field, self.v)
                    self.src = field
                    nxt = extract(field, self.v, self.dims, p)
            else:
                self.J_prev_same = J
                self.last_extract = (field, v)
                self.src = field
                nxt = extract(field, v, self.dims, p)
        self.history.append(Record(k, event, v, int(solid.sum()), J, g, mu, gamma, self.dv,
                                   S if stress else 0.0, g_s, self.mu_s if stress else 0.0,
                                   self.gamma_s if stress else 0.0, lam if eigen else 0.0, g_l,
                                   self.mu_l if eigen else 0.0, self.gamma_l if eigen else 0.0,
                                   P if buck else 0.0, g_p, self.mu_p if buck else 0.0,
                                   self.gamma_p if buck else 0.0))
        self.k += 1
        if self.k >= p.max_fea:
            nxt = None
        return nxt

    def _converged(self, J):
        return self.J_prev_same is not None and abs(J - self.J_prev_same) < self.p.conv_tol * self.J_prev_same

    def _target(self, v):
        self.v = v
        self.fp = 0
        self.J_prev_same = None

    def run(self, fixed, F, Ke=None):
        """The whole loop with direct solves; returns the last converged
        feasible design (solid, v, J) and the history."""
        Ke = fem.ke_gauss() if Ke is None else Ke
        Me = modal.me_gauss()
        solid = self.first()
        while solid is not None:
            U = fea(self.dims, solid, fixed, F, Ke, self.p)
            J = float(sum(post.compliance(F[r], U[r]) for r in range(F.shape[0])))
            fJ = compliance_field(self.dims, solid, Ke, U, self.p)
            S = fS = lam = fL = P = fP = None
            if self.p.alpha_sigma > 0:
                S, fS = stress_quantities(self.dims, solid, fixed, Ke, U, self.p)
            if self.p.alpha_lambda > 0:
                lam, fL = eigen_quantities(self.dims, solid, fixed, Ke, Me, self.p)
            if self.p.alpha_P > 0:
                P, fP = buckling_quantities(self.dims, solid, fixed, Ke, U, self.p)
            solid = self.after_solve(solid, J, fJ, S, fS, lam, fL, P, fP)
        b = self.best
        return (b[0], b[1], b[2]), self.history
