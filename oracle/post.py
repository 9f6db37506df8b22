"""Oracle post-processing: compliance, element sensitivities, topology
extraction.  TEST INFRASTRUCTURE ONLY.

* Compliance J = f . u (Eq. 1.3-1.4).
* Element strain-energy sensitivity s_e = rho_e u_e^T Ke u_e: the element
  term ``u^T K^e u`` of Eq. 3.5 (the paper's element-sensitivity route of
  Sec. 3.1), scaled by the element's stiffness scale so that
  sum_e s_e = u^T K u = J.  The mutual energy of two fields,
  rho_e u_e^T Ke v_e, is the analogous term pairing a load case with an
  adjoint field (the lambda of Eq. 3.3).
* Topology at volume fraction v: the level set of Eq. 3.6 with its cutting
  value chosen so that ceil(v * nE) elements are solid (Sec. 3.2); elements are
  ranked by decreasing sensitivity, equal values by increasing element index.
  An optional integer tie key ranks equal values first (ascending) and the
  index after it: a field projected by the casting constraint (Sec. 3.7) has
  plateaus of equal values, and cutting them nearer-to-the-parting-plane first
  keeps the extracted topology free of cavities (casting.parting_distance).
  Values compare as numbers, so -0.0 and +0.0 are equal.
"""
from __future__ import annotations

import math

import numpy as np

from . import fem


def compliance(f, u):
    return float(np.dot(f, u))


def element_energy(dims, rho, Ke, u, v=None):
    """rho_e u_e^T Ke v_e for every element (v defaults to u)."""
    dm = fem.dofmap(dims)
    ue = u[dm]
    ve = ue if v is None else v[dm]
    return rho * np.einsum("ei,ij,ej->e", ue, Ke, ve)


def rank_order(s, tie=None):
    """Element indices sorted by (-s, index), or by (-s, tie, index)."""
    idx = np.arange(s.size)
    if tie is None:
        return np.lexsort((idx, -s))
    return np.lexsort((idx, np.asarray(tie, dtype=np.int64), -s))


def threshold(s, vol_frac, tie=None):
    """(solid mask uint8, cut value tau) keeping ceil(vol_frac * n) elements."""
    n = s.size
    keep = min(n, max(0, math.ceil(vol_frac * n)))
    order = rank_order(s, tie)
    solid = np.zeros(n, dtype=np.uint8)
    solid[order[:keep]] = 1
    tau = float(s[order[keep - 1]]) if keep > 0 else float("inf")
    return solid, tau
