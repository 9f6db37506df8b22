"""Pins of the CPU oracle against facts fixed by the mathematics (no GPU).

Each test checks the oracle against something other than itself: an
independent exact-rational construction, a closed form, an invariant, a
textbook special case (the patch test), or brute force on a tiny input.
"""
from fractions import Fraction
import json
import math
import os

import numpy as np
import scipy.linalg as sla
import pytest

from oracle import fem, solvers, post
from paper_2203_15115_amd import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    """A hand-worked fixture under tests/golden (each states what it pins)."""
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


# ----------------------------------------------------------------- element matrix
@pytest.mark.parametrize("h", [(1, 1, 1), (1, 2, Fraction(1, 2)), (3, 1, 2)])
def test_ke_gauss_equals_exact_rationals(h):
    Kg = fem.ke_gauss(tuple(float(v) for v in h), 1.0, 0.3)
    Kx = np.array([[float(v) for v in row] for row in fem.ke_exact(h, 1, Fraction(3, 10))])
    assert np.max(np.abs(Kg - Kx)) <= 4e-16 * np.max(np.abs(Kx)) * 24


def test_ke_unit_cube_closed_forms():
    # Unit cube, E=1, nu=3/10: lambda=15/26, mu=5/13.  Every diagonal entry is
    # (lambda+2mu)/9 + 2*mu/9 = (lambda+4mu)/9 = 55/234 and the trace is 24x that.
    g = golden("ke_unit_cube.json")
    K = fem.ke_exact()
    lam, mu = lame(Fraction(1), Fraction(3, 10))
    assert (lam, mu) == tuple(Fraction(v) for v in g["lame"])
    for i in range(24):
        assert K[i][i] == (lam + 4 * mu) / 9 == Fraction(g["diagonal"])
    assert sum(K[i][i] for i in range(24)) == Fraction(g["trace"])
    for i in range(24):
        for j in range(24):
            assert K[i][j] == K[j][i]


def test_ke_box_diagonal_closed_form():
    # Diagonal for displacement component i: (lam+2mu) int (dN/dx_i)^2
    # + mu sum_{k != i} int (dN/dx_k)^2, with int (dN/dx)^2 = hy hz / (9 hx).
    h = (1.0, 2.0, 0.5)
    lam, mu = lame(1.0, 0.3)
    g = [h[1] * h[2] / (9 * h[0]), h[0] * h[2] / (9 * h[1]), h[0] * h[1] / (9 * h[2])]
    K = fem.ke_gauss(h, 1.0, 0.3)
    for a in range(8):
        for i in range(3):
            want = (lam + 2 * mu) * g[i] + mu * (sum(g) - g[i])
            assert abs(K[3 * a + i, 3 * a + i] - want) < 1e-15


def test_ke_rigid_null_space_and_rank():
    for h in [(1.0, 1.0, 1.0), (1.0, 2.0, 0.5)]:
        K = fem.ke_gauss(h, 1.0, 0.3)
        R = fem.rigid_modes_element(h)
        assert np.max(np.abs(K @ R)) < 1e-14
        ev = np.linalg.eigvalsh(K)
        assert np.sum(ev < 1e-12) == 6 and np.all(ev > -1e-13)


def test_ke_unit_cube_spectrum():
    # Eigenvalues of the unit-cube matrix (E=1, nu=3/10), derived from the
    # rational matrix: 0 (x6), 5/78 (x2), 55/468 (x3), 5/26 (x3), 10/39 (x1),
    # 5/13 (x8), 5/4 (x1).  They sum to the trace 220/39.
    g = golden("ke_unit_cube.json")
    spec = [Fraction(v) for v, m in g["spectrum"] for _ in range(m)]
    assert len(spec) == 24 and sum(spec) == Fraction(g["trace"])
    ev = np.sort(np.linalg.eigvalsh(fem.ke_gauss()))
    assert np.allclose(ev, np.sort([float(v) for v in spec]), atol=1e-14)


def test_ke_uniform_strain_energy():
    # A linear displacement u = eps x has the uniform strain eps, so its
    # energy is exactly V * (lam tr(eps)^2 + 2 mu eps:eps) for any symmetric eps.
    rng = np.random.default_rng(0)
    for h in [(1.0, 1.0, 1.0), (2.0, 0.5, 1.5)]:
        K = fem.ke_gauss(h, 2.5, 0.27)
        lam, mu = lame(2.5, 0.27)
        X = fem.LOCAL * np.asarray(h)
        for _ in range(5):
            A = rng.standard_normal((3, 3))
            eps = (A + A.T) / 2
            u = (X @ eps.T).ravel()   # antisymmetric part would be a rotation
            want = np.prod(h) * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
            assert abs(u @ K @ u - want) < 1e-12 * abs(want)


# ----------------------------------------------------------------- assembly
def _rand_rho(dims, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random(wl.n_elems(dims)) < 0.3, 1e-3, 1.0) * rng.uniform(0.5, 2.0, wl.n_elems(dims))


def test_assembly_rigid_modes_and_jacobi_closed_form():
    dims = (5, 3, 4)
    rho = _rand_rho(dims, 1)
    K = fem.assemble(dims, rho, fem.ke_gauss())
    X = fem.node_coords(dims)
    x, y, z = X.T
    o, zz = np.ones_like(x), np.zeros_like(x)
    for m in [(o, zz, zz), (zz, o, zz), (zz, zz, o), (zz, -z, y), (z, zz, -x), (-y, x, zz)]:
        r = np.stack(m, axis=1).ravel()
        assert np.max(np.abs(K @ r)) < 1e-12
    # diag(K)_(n,c) = 55/234 * sum of rho over the elements touching n
    conn = fem.connectivity(dims)
    rs = np.zeros(wl.n_nodes(dims))
    np.add.at(rs, conn.ravel(), np.repeat(rho, 8))
    assert np.allclose(K.diagonal(), np.repeat(rs, 3) * 55 / 234, rtol=1e-14, atol=0)
    assert abs(K - K.T).max() < 1e-15


def test_assembly_linear_field():
    dims = (4, 5, 3)
    rng = np.random.default_rng(2)
    lam, mu = lame(1.0, 0.3)
    A = rng.standard_normal((3, 3))
    eps = (A + A.T) / 2
    X = fem.node_coords(dims)
    u = (X @ eps.T).ravel()
    # uniform density: uniform stress is in equilibrium at interior nodes
    K1 = fem.assemble(dims, np.ones(wl.n_elems(dims)), fem.ke_gauss())
    y = (K1 @ u).reshape(-1, 3)
    nx, ny, nz = dims
    for k in range(1, nz):
        for j in range(1, ny):
            for i in range(1, nx):
                assert np.max(np.abs(y[wl.node_id(dims, i, j, k)])) < 1e-12
    # any density: energy of a uniform strain is sum_e rho_e V eps:C:eps
    rho = _rand_rho(dims, 3)
    K = fem.assemble(dims, rho, fem.ke_gauss())
    want = rho.sum() * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    assert abs(u @ K @ u - want) < 1e-11 * want


def test_ebe_apply_equals_assembled():
    dims = (6, 4, 3)
    rho = _rand_rho(dims, 4)
    Ke = fem.ke_gauss()
    K = fem.assemble(dims, rho, Ke)
    u = np.random.default_rng(5).standard_normal(3 * wl.n_nodes(dims))
    assert np.allclose(fem.apply_ebe(dims, rho, Ke, u), K @ u, rtol=0, atol=1e-13)


# ----------------------------------------------------------------- solve
def test_patch_test_uniaxial_stress():
    # Rollers on x=0 (ux), y=0 (uy), z=0 (uz); traction sigma on x=Lx lumped
    # consistently (sigma*hy*hz/4 per node per face quad).  The exact solution is
    # linear: ux = sigma x/E, uy = -nu sigma y/E, uz = -nu sigma z/E.
    dims = (4, 3, 2)
    h = (1.5, 1.0, 2.0)
    E, nu, sig = 3.0, 0.3, 0.7
    nx, ny, nz = dims
    K = fem.assemble(dims, np.ones(wl.n_elems(dims)), fem.ke_gauss(h, E, nu))
    X = fem.node_coords(dims, h)
    fixed = np.zeros(3 * wl.n_nodes(dims), dtype=np.uint8)
    fixed[3 * np.flatnonzero(X[:, 0] == 0) + 0] = 1
    fixed[3 * np.flatnonzero(X[:, 1] == 0) + 1] = 1
    fixed[3 * np.flatnonzero(X[:, 2] == 0) + 2] = 1
    f = np.zeros(3 * wl.n_nodes(dims))
    for k in range(nz):
        for j in range(ny):
            for (dj, dk) in [(0, 0), (1, 0), (0, 1), (1, 1)]:
                f[3 * wl.node_id(dims, nx, j + dj, k + dk)] += sig * h[1] * h[2] / 4
    u = solvers.solve_direct(K, fixed, f).reshape(-1, 3)
    want = np.stack([sig * X[:, 0] / E, -nu * sig * X[:, 1] / E, -nu * sig * X[:, 2] / E], axis=1)
    assert np.max(np.abs(u - want)) < 1e-12
    vol = np.prod([d * hh for d, hh in zip(dims, h)])
    assert abs(post.compliance(f, u.ravel()) - sig ** 2 * vol / E) < 1e-12


def _tiny_problem(dims, seed, block):
    rho = _rand_rho(dims, seed)
    fixed = wl.clamp_x0(dims)
    f = wl.edge_load(dims, "bottom") + 0.3 * wl.point_load(dims, wl.node_id(dims, dims[0] // 2 + 1, 1, dims[2]))
    return rho, fixed, f


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 1), (3, 2, 2), (6, 3, 3)])
def test_direct_equals_dense_bruteforce(dims):
    rho, fixed, f = _tiny_problem(dims, 7, (2, 2, 2))
    K = fem.assemble(dims, rho, fem.ke_gauss())
    u = solvers.solve_direct(K, fixed, f)
    free = np.flatnonzero(fixed == 0)
    ub = np.linalg.solve(K.toarray()[np.ix_(free, free)], f[free])
    assert np.allclose(u[free], ub, rtol=1e-10, atol=0)
    assert np.all(u[fixed == 1] == 0)


@pytest.mark.parametrize("dims,block", [((8, 4, 4), (2, 2, 2)), ((12, 6, 6), (4, 4, 4)),
                                        ((9, 5, 4), (4, 4, 4)), ((24, 12, 12), (4, 4, 4))])
def test_cg_and_dcg_equal_direct(dims, block):
    rho, fixed, f = _tiny_problem(dims, 11, block)
    K = fem.assemble(dims, rho, fem.ke_gauss())
    ud = solvers.solve_direct(K, fixed, f)
    uc, itc, rc = solvers.pcg(K, fixed, f, rtol=1e-12)
    seen = []

    def chk(r, W):
        seen.append(np.max(np.abs(W.T @ r)) / np.max(np.abs(f)))

    ux, itx, rx = solvers.dcg(K, fixed, f, dims, block, rtol=1e-12, check=chk)
    nrm = np.linalg.norm(ud)
    assert np.linalg.norm(uc - ud) / nrm < 1e-8
    assert np.linalg.norm(ux - ud) / nrm < 1e-8
    assert rc < 1e-11 and rx < 1e-11
    assert max(seen) < 1e-9          # W^T r = 0 is an invariant of the deflated iteration
    assert itx < itc


def test_dcg_config0_workload():
    p = wl.config(0)
    K = fem.assemble(p.dims, p.rho, fem.ke_gauss())
    ud = solvers.solve_direct(K, p.fixed, p.F[0])
    ux, it, rr = solvers.dcg(K, p.fixed, p.F[0], p.dims, p.block, rtol=1e-8)
    assert rr <= 1e-8
    assert np.linalg.norm(ux - ud) / np.linalg.norm(ud) < 1e-3


def test_linearity_and_mirror_symmetry():
    dims = (6, 4, 3)
    nx, ny, nz = dims
    rng = np.random.default_rng(3)
    r = np.where(rng.random((nz, ny, nx)) < 0.3, 1e-3, 1.0)
    r = 0.5 * (r + r[:, ::-1, :])          # symmetric about the mid y-plane
    rho = r.ravel()
    K = fem.assemble(dims, rho, fem.ke_gauss())
    fixed = wl.clamp_x0(dims)
    f = wl.edge_load(dims, "top")           # uniform along y: symmetric
    u = solvers.solve_direct(K, fixed, f).reshape(nz + 1, ny + 1, nx + 1, 3)
    assert np.max(np.abs(u[:, :, :, 1] + u[:, ::-1, :, 1])) < 1e-12 * np.max(np.abs(u))
    assert np.max(np.abs(u[:, :, :, 2] - u[:, ::-1, :, 2])) < 1e-12 * np.max(np.abs(u))
    u2 = solvers.solve_direct(K, fixed, -2.5 * f).reshape(u.shape)
    assert np.max(np.abs(u2 + 2.5 * u)) < 1e-12 * np.max(np.abs(u2))


# ----------------------------------------------------------------- post-processing
def test_energy_identity_and_reciprocity():
    dims = (8, 4, 4)
    rho, fixed, _ = _tiny_problem(dims, 13, (4, 4, 4))
    Ke = fem.ke_gauss()
    K = fem.assemble(dims, rho, Ke)
    f1 = wl.edge_load(dims, "bottom")
    f2 = wl.point_load(dims, wl.node_id(dims, 5, 2, 3))
    u1 = solvers.solve_direct(K, fixed, f1)
    u2 = solvers.solve_direct(K, fixed, f2)
    s1 = post.element_energy(dims, rho, Ke, u1)
    s12 = post.element_energy(dims, rho, Ke, u1, u2)
    assert abs(s1.sum() - post.compliance(f1, u1)) < 1e-12 * abs(s1.sum())
    # Maxwell-Betti: f1.u2 = f2.u1 = sum of the mutual energies
    assert abs(post.compliance(f1, u2) - post.compliance(f2, u1)) < 1e-12 * abs(post.compliance(f2, u1))
    assert abs(s12.sum() - post.compliance(f2, u1)) < 1e-12 * abs(s12.sum())
    assert np.all(s1 >= 0)


@pytest.mark.parametrize("n,vf", [(1, 0.5), (7, 0.5), (50, 0.3), (50, 1.0), (50, 0.0), (333, 0.475)])
def test_threshold_bruteforce(n, vf):
    rng = np.random.default_rng(n)
    s = rng.integers(0, 6, n).astype(float) * 0.25      # many ties
    solid, tau = post.threshold(s, vf)
    ranked = sorted(range(n), key=lambda e: (-s[e], e))
    keep = math.ceil(vf * n)
    want = np.zeros(n, dtype=np.uint8)
    want[ranked[:keep]] = 1
    assert np.array_equal(solid, want)
    if keep:
        assert tau == s[ranked[keep - 1]]
        assert np.all(s[solid == 1] >= tau) and np.all(s[solid == 0] <= tau)


@pytest.mark.parametrize("n,vf", [(7, 0.5), (50, 0.3), (333, 0.475)])
def test_threshold_tie_key_bruteforce(n, vf):
    # a secondary key ranks equal values (ascending) before the index
    rng = np.random.default_rng(n + 1)
    s = rng.integers(0, 4, n).astype(float) * 0.5
    tie = rng.integers(0, 5, n)
    solid, tau = post.threshold(s, vf, tie)
    ranked = sorted(range(n), key=lambda e: (-s[e], tie[e], e))
    assert list(post.rank_order(s, tie)) == ranked
    keep = math.ceil(vf * n)
    want = np.zeros(n, dtype=np.uint8)
    want[ranked[:keep]] = 1
    assert np.array_equal(solid, want)
    assert tau == s[ranked[keep - 1]]


def test_signed_zeros_rank_as_equal_values():
    # -0.0 and +0.0 are the same number: ranked by index among themselves
    s = np.array([0.0, -0.0, 1.0, -0.0, 0.0, -1.0])
    assert list(post.rank_order(s)) == [2, 0, 1, 3, 4, 5]
    solid, tau = post.threshold(s, 0.5)
    assert list(solid) == [1, 1, 1, 0, 0, 0] and tau == 0.0


def test_coarse_matrix_structure():
    dims = (8, 4, 4)
    block = (4, 2, 2)
    rho = _rand_rho(dims, 17)
    K = fem.assemble(dims, rho, fem.ke_gauss())
    # unconstrained, one block: rigid modes have zero energy
    E1, _ = solvers.coarse_matrix(K, np.zeros(K.shape[0], np.uint8), dims, (8, 4, 4))
    assert np.max(np.abs(E1)) < 1e-12
    E, nb = solvers.coarse_matrix(K, wl.clamp_x0(dims), dims, block)
    assert nb == [2, 2, 2]
    assert np.allclose(E, E.T, atol=1e-14)
    assert np.linalg.eigvalsh(E).min() > 0       # clamped: positive definite


# ------------------------------------------------------------- casting (Sec. 3.7)
def test_casting_projection_worked_line():
    # a line of 8 elements, worked by hand for a parting plane inside it and
    # for one-sided castings, laid along each axis in turn
    from oracle.casting import cast_project
    g = golden("casting_worked_line.json")
    phi = g["phi"]
    for case in g["cases"]:
        for axis, dims in ((0, (8, 1, 1)), (1, (1, 8, 1)), (2, (1, 1, 8))):
            assert list(cast_project(phi, dims, axis, case["parting"])) == case["want"], (case, axis)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_casting_projection_is_the_least_monotone_majorant(axis):
    # characterisation independent of the running-maximum formula: along every
    # line the result (i) is >= phi, (ii) does not increase away from the
    # parting plane on either side, and (iii) equals phi at some element between
    # it and the far end of its side -- so every field with (i) and (ii) is >= it
    from oracle.casting import cast_project
    rng = np.random.default_rng(40 + axis)
    dims = (5, 4, 6)
    n = dims[axis]
    for p in range(n + 1):
        phi = rng.integers(0, 7, size=int(np.prod(dims))).astype(float)  # ties on purpose
        g = cast_project(phi, dims, axis, p)
        f3 = np.moveaxis(phi.reshape(dims[::-1]), 2 - axis, -1).reshape(-1, n)
        g3 = np.moveaxis(g.reshape(dims[::-1]), 2 - axis, -1).reshape(-1, n)
        assert np.all(g3 >= f3)
        for fl, gl in zip(f3, g3):
            for j in range(n):
                if j >= p:
                    if j + 1 < n:
                        assert gl[j] >= gl[j + 1]
                    assert gl[j] in set(fl[j:])
                else:
                    if j >= 1:
                        assert gl[j] >= gl[j - 1]
                    assert gl[j] in set(fl[:j + 1])
        assert np.array_equal(cast_project(g, dims, axis, p), g)  # idempotent


def test_parting_distance_worked_line():
    # 8 elements, plane before element 3: 2 1 0 | 0 1 2 3 4
    from oracle.casting import parting_distance
    assert list(parting_distance((8, 1, 1), 0, 3)) == [2, 1, 0, 0, 1, 2, 3, 4]
    assert list(parting_distance((1, 1, 8), 2, 0)) == list(range(8))
    assert list(parting_distance((1, 8, 1), 1, 8)) == list(range(7, -1, -1))
    with pytest.raises(ValueError):
        parting_distance((4, 1, 1), 0, 5)


def test_casting_plateau_cut_nearer_the_plane_first():
    # all equal values on a line with the plane in the middle: a cut keeping 4
    # of 8 elements keeps the 4 nearest the plane (2 on each side), not the 4
    # lowest indices (which would leave voids between the plane and solid)
    from oracle.casting import cast_project, parting_distance
    phi = np.full(8, 2.0)
    g = cast_project(phi, (8, 1, 1), 0, 4)
    solid, _ = post.threshold(g, 0.5, parting_distance((8, 1, 1), 0, 4))
    assert list(solid) == [0, 0, 1, 1, 1, 1, 0, 0]
    solid_idx, _ = post.threshold(g, 0.5)
    assert list(solid_idx) == [1, 1, 1, 1, 0, 0, 0, 0]


def _has_cavity(solid, dims, axis, parting):
    # along a line, a void between the plane and a solid element on either side
    n = dims[axis]
    lines = np.moveaxis(solid.reshape(dims[::-1]), 2 - axis, -1).reshape(-1, n)
    for ln in lines:
        hi = ln[parting:]
        if hi.any() and not hi[:np.nonzero(hi)[0].max() + 1].all():
            return True
        lo = ln[:parting][::-1]
        if lo.any() and not lo[:np.nonzero(lo)[0].max() + 1].all():
            return True
    return False


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_casting_topology_has_no_cavity(axis):
    # the thresholded topology of a cast-projected field, ties cut by the
    # distance to the plane, has no cavity for any parting plane; the
    # index-only cut does leave cavities when the plane is inside the grid
    from oracle.casting import cast_project, parting_distance
    dims = (12, 10, 14)
    n = dims[axis]
    rng = np.random.default_rng(70 + axis)
    idx_cavities = 0
    for p in (0, 1, n // 2, n - 1, n):
        for seed in range(4):
            phi = rng.standard_normal(int(np.prod(dims)))
            phi[rng.random(phi.size) < 0.3] = 0.0
            g = cast_project(phi, dims, axis, p)
            solid, _ = post.threshold(g, 0.4, parting_distance(dims, axis, p))
            assert not _has_cavity(solid, dims, axis, p), (p, seed)
            idx_cavities += _has_cavity(post.threshold(g, 0.4)[0], dims, axis, p)
    assert idx_cavities > 0


# ------------------------------------------------------------- constrained operator
def _dense_operator(apply, n):
    """Matrix of a linear map given only as a function, column by column."""
    A = np.zeros((n, n))
    e = np.zeros(n)
    for i in range(n):
        e[i] = 1.0
        A[:, i] = apply(e)
        e[i] = 0.0
    return A


def test_apply_constrained_is_the_extended_free_block():
    # the operator the solver iterates with: K_ff on free DOFs (fixed inputs
    # count as zero), the identity on fixed DOFs.  Pinned against the dense
    # assembled matrix, and by the properties a wrong masking would break:
    # symmetry, identity rows AND columns on fixed DOFs, A u = f for the direct
    # solution, positive definiteness with a clamped face
    dims = (4, 3, 2)
    rho = _rand_rho(dims, 21)
    K = fem.assemble(dims, rho, fem.ke_gauss())
    n = K.shape[0]
    rng = np.random.default_rng(22)
    fixed = (rng.random(n) < 0.2).astype(np.uint8)
    A = _dense_operator(lambda u: fem.apply_constrained(K, fixed, u), n)
    assert np.max(np.abs(A - A.T)) <= 1e-15 * np.max(np.abs(A))
    fx = np.flatnonzero(fixed)
    fr = np.flatnonzero(fixed == 0)
    assert np.array_equal(A[fx][:, fx], np.eye(fx.size))
    assert not A[fx][:, fr].any() and not A[fr][:, fx].any()
    Kd = K.toarray()
    assert np.max(np.abs(A[np.ix_(fr, fr)] - Kd[np.ix_(fr, fr)])) <= 1e-15 * np.max(np.abs(Kd))
    # the direct solution satisfies A u = f (f is zero on fixed DOFs, u too)
    fixed_c = wl.clamp_x0(dims)
    f = wl.edge_load(dims, "bottom") + 0.5 * wl.point_load(dims, wl.node_id(dims, 2, 1, 2))
    u = solvers.solve_direct(K, fixed_c, f)
    assert np.max(np.abs(fem.apply_constrained(K, fixed_c, u) - f)) <= 1e-12 * np.max(np.abs(f))
    Ac = _dense_operator(lambda v: fem.apply_constrained(K, fixed_c, v), n)
    assert np.linalg.eigvalsh(Ac).min() > 0


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (1.0, 2.0, 0.5)])
def test_apply_at_nodes_equals_assembled_operator_everywhere(h):
    # the per-node oracle of the full-size apply, at EVERY node of a ragged mesh
    # with scattered fixed DOFs, against the assembled constrained operator
    dims = (5, 3, 4)
    rho = _rand_rho(dims, 23)
    Ke = fem.ke_gauss(h, 1.0, 0.3)
    K = fem.assemble(dims, rho, Ke)
    n = K.shape[0]
    rng = np.random.default_rng(24)
    fixed = (rng.random(n) < 0.15).astype(np.uint8)
    u = rng.standard_normal(n)
    nodes = np.arange(wl.n_nodes(dims))
    got = fem.apply_at_nodes(dims, rho, Ke, u, nodes, fixed)
    want = fem.apply_constrained(K, fixed, u).reshape(-1, 3)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # unconstrained: no response to a rigid motion at any node
    X = fem.node_coords(dims, h)
    x, y, z = X.T
    rot = np.stack([0.3 + 0.7 * y - 0.2 * z, -0.1 - 0.7 * x + 0.5 * z, 0.25 + 0.2 * x - 0.5 * y], axis=1)
    got0 = fem.apply_at_nodes(dims, rho, Ke, rot.ravel(), nodes)
    assert np.max(np.abs(got0)) <= 1e-13 * np.max(np.abs(Ke)) * np.max(np.abs(rot))


def test_coarse_matrix_order_from_hand_built_motions():
    # E(6I+a, 6J+b) = w_Ia^T K_ff w_Jb with every column built here from the
    # physics of a rigid motion (translation e_a, rotation e_a x (x - c) about
    # the centre c of the block's node range, coordinates in element units over
    # the largest block edge), zero on fixed DOFs, block I = bi + nbx (bj + nby bk):
    # pins the block and mode order the GPU coarse matrix is compared in
    dims, block = (8, 4, 4), (4, 4, 4)          # two blocks along x
    rho = _rand_rho(dims, 25)
    K = fem.assemble(dims, rho, fem.ke_gauss())
    fixed = wl.clamp_x0(dims)
    E, nb = solvers.coarse_matrix(K, fixed, dims, block)
    assert nb == [2, 1, 1] and E.shape == (12, 12)
    nx, ny, nz = dims
    centres = {0: (1.5, 2.0, 2.0), 1: (6.0, 2.0, 2.0)}   # node ranges 0..3 and 4..8 along x, 0..4 in y, z
    cols = []
    for I in range(2):
        c = np.array(centres[I])
        for a in range(6):
            w = np.zeros(3 * wl.n_nodes(dims))
            for k in range(nz + 1):
                for j in range(ny + 1):
                    for i in range(nx + 1):
                        if min(i // 4, 1) != I:
                            continue
                        if a < 3:
                            d = np.eye(3)[a]
                        else:
                            d = np.cross(np.eye(3)[a - 3], (np.array([i, j, k]) - c) / 4.0)
                        nid = wl.node_id(dims, i, j, k)
                        w[3 * nid:3 * nid + 3] = d
            w[fixed == 1] = 0.0
            cols.append(w)
    W = np.stack(cols, axis=1)
    Kd = K.toarray()
    keep = (fixed == 0).astype(float)
    Eref = W.T @ (Kd * keep[:, None] * keep[None, :]) @ W
    assert np.max(np.abs(E - Eref)) <= 1e-13 * np.max(np.abs(Eref))
    # block 1 (no fixed DOF) is coupled to block 0 only through the shared elements:
    # its rigid motions cost energy only there, so E(1, 1) is not zero but far
    # smaller than the clamped block's
    assert np.trace(E[6:, 6:]) < np.trace(E[:6, :6])


# ------------------------------------------------------------- level-set loop (Sec. 3.3-3.4, 3.8)
def test_al_update_hand_checked_sequence():
    # mu <- max(mu + gamma g, 0); gamma kept when min(g_k, 0) <= 0.25 min(g_{k-1}, 0),
    # else max(10 gamma, k^2) (Eq. 3.11-3.12 as printed), both from the old values;
    # the sequence from mu = 100, gamma = 10 is worked by hand in the fixture
    from oracle.levelset import al_update
    g = golden("al_update_sequence.json")
    mu, gamma, prev = float(g["mu0"]), float(g["gamma0"]), None
    for st in g["steps"]:
        gk = float(Fraction(st["g"]))
        mu, gamma = al_update(mu, gamma, gk, prev, st["k"])
        prev = gk
        want_mu = float(Fraction(st["mu"]))
        assert abs(mu - want_mu) <= 1e-12 * max(1.0, want_mu) and gamma == st["gamma"], (st, mu, gamma)
    # the k^2 branch: a small penalty late in the run
    L = g["late_step"]
    got = al_update(float(L["mu"]), float(L["gamma"]), float(Fraction(L["g"])), float(Fraction(L["g_prev"])), L["k"])
    assert got == (float(Fraction(L["want_mu"])), float(L["want_gamma"]))


def test_augmented_weights():
    from oracle.levelset import combined_field, weights
    assert weights([100.0, 3.0], [10.0, 10.0], [-0.5, -0.5]) == [95.0, 0.0]
    assert weights([0.0], [10.0], [-0.2]) == [1.0]  # no active weight: the field itself
    f = [np.array([1.0, 2.0]), np.array([10.0, -1.0])]
    assert list(combined_field(f, [2.0, 0.5])) == [7.0, 3.5]


def _loop_run(dims, p, F_which=("bottom",)):
    from oracle import levelset as ls
    fixed = wl.clamp_x0(dims)
    F = np.stack([wl.edge_load(dims, w) for w in F_which])
    loop = ls.Loop(dims, p)
    return loop.run(fixed, F)


def test_levelset_loop_invariants():
    # Pareto tracing under J <= 3 J0 on a 12x6x6 cantilever (direct solves)
    from oracle import levelset as ls
    dims = (12, 6, 6)
    n = int(np.prod(dims))
    p = ls.Params(alpha_J=3.0)
    (best, v_best, J_best), h = _loop_run(dims, p)
    J0 = h[0].J
    assert h[0].v == 1.0 and h[0].nsolid == n and h[0].event == ls.FEA_CONVERGED
    assert abs(h[0].g - (1 / 3 - 1)) < 1e-15
    assert h[-1].event == ls.FEA_TERMINATED and h[-1].dv < p.dv_min
    conv = [r for r in h if r.event == ls.FEA_CONVERGED]
    assert all(r.g <= 0 for r in conv)                                  # converged designs are feasible
    assert all(a.v > b.v for a, b in zip(conv, conv[1:]))                # the Pareto trace descends
    assert conv[-1].v == v_best and conv[-1].J == J_best and J_best <= 3 * J0
    assert int(best.sum()) == conv[-1].nsolid
    for r in h[1:]:
        assert r.nsolid == math.ceil(r.v * n - 1e-9), r                  # topology at its target volume
    for a, b in zip(h, h[1:]):
        assert b.dv <= a.dv                                              # the step only shrinks ...
        if b.event in (ls.FEA_VIOLATED, ls.FEA_DIVERGED, ls.FEA_TERMINATED) and b.dv < a.dv:
            assert b.dv == a.dv / 2                                      # ... by halving
        if b.event == ls.FEA_VIOLATED:
            assert b.g > 0
        if a.event == ls.FEA_FIXED_POINT and a.v == b.v and b.event != ls.FEA_VIOLATED:
            # step 7: converged iff the compliance moved by less than 1%
            assert (b.event == ls.FEA_CONVERGED) == (abs(b.J - a.J) < 0.01 * a.J)
    assert any(r.event == ls.FEA_VIOLATED for r in h)                    # the hard constraint bound the run


def test_levelset_loop_with_casting_has_no_cavity():
    # every topology the loop analyses under the casting constraint (parting
    # plane in the middle of z) is free of cavities along z
    from oracle import levelset as ls
    dims = (12, 6, 6)
    p = ls.Params(alpha_J=2.0, cast_axis=2, cast_parting=3)
    fixed = wl.clamp_x0(dims)
    F = wl.edge_load(dims, "bottom")[None]
    loop = ls.Loop(dims, p)
    seen = []
    orig = loop.after_solve

    def spy(solid, J, field, *rest):
        seen.append(solid.copy())
        return orig(solid, J, field, *rest)
    loop.after_solve = spy
    (best, v, J), h = loop.run(fixed, F)
    assert len(seen) == len(h) > 5 and J <= 2 * h[0].J
    for s in seen:
        assert not _has_cavity(s, dims, 2, 3)


# ------------------------------------------------------------- p-norm stress (Eq. 3.3, 3.23)
def test_von_mises_special_cases_and_invariance():
    from oracle.stress import von_mises
    assert von_mises(np.array([[3.0, 0, 0, 0, 0, 0]]))[0] == 3.0               # uniaxial
    assert abs(von_mises(np.array([[0, 0, 0, 0, 0, 2.0]]))[0] - 2 * np.sqrt(3)) < 1e-15  # pure shear
    assert von_mises(np.array([[5.0, 5.0, 5.0, 0, 0, 0]]))[0] == 0.0           # hydrostatic
    # invariant under rotations of the stress tensor
    rng = np.random.default_rng(3)
    for _ in range(5):
        S = rng.standard_normal((3, 3))
        S = S + S.T
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        R = Q @ S @ Q.T
        v = lambda T: np.array([[T[0, 0], T[1, 1], T[2, 2], T[1, 2], T[0, 2], T[0, 1]]])
        assert abs(von_mises(v(S))[0] - von_mises(v(R))[0]) < 1e-12 * von_mises(v(S))[0]
        # and equal to sqrt(3/2 |dev S|^2)
        dev = S - np.trace(S) / 3 * np.eye(3)
        assert abs(von_mises(v(S))[0] - np.sqrt(1.5 * np.sum(dev * dev))) < 1e-12 * von_mises(v(S))[0]


def test_element_stress_of_a_linear_field():
    # trilinear elements reproduce a linear displacement u = A x exactly: the
    # centroid stress is lambda tr(eps) I + 2 mu eps with eps = sym(A), times rho
    from oracle.stress import element_stress
    dims, h, E, nu = (3, 2, 2), (1.0, 2.0, 0.5), 2.0, 0.27
    A = np.random.default_rng(4).standard_normal((3, 3))
    X = fem.node_coords(dims, h)
    u = (X @ A.T).reshape(-1)
    rho = np.random.default_rng(5).uniform(0.5, 2.0, wl.n_elems(dims))
    sig = element_stress(dims, rho, u, h, E, nu)
    lam, mu = fem.lame(E, nu)
    eps = 0.5 * (A + A.T)
    S = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
    want = np.array([S[0, 0], S[1, 1], S[2, 2], S[1, 2], S[0, 2], S[0, 1]])
    assert np.allclose(sig, rho[:, None] * want[None, :], rtol=1e-13, atol=1e-13)


def _stress_problem(dims=(6, 3, 3)):
    rng = np.random.default_rng(8)
    rho = np.where(rng.random(wl.n_elems(dims)) < 0.3, 1e-3, 1.0)
    fixed = wl.clamp_x0(dims)
    F = np.stack([wl.edge_load(dims, "bottom"), wl.point_load(dims, wl.node_id(dims, dims[0], 1, dims[2]))])
    K = fem.assemble(dims, rho, fem.ke_gauss())
    U = np.stack([solvers.solve_direct(K, fixed, f) for f in F])
    return dims, rho, fixed, F, K, U


def test_adjoint_rhs_is_the_gradient_of_the_pnorm():
    # central differences of sigma_PN along random directions of each load
    # case's displacements (p = 8): the adjoint right-hand side is the gradient
    from oracle.stress import adjoint_rhs, pnorm
    dims, rho, fixed, F, K, U = _stress_problem()
    B = adjoint_rhs(U, dims, rho, fixed, p=8.0)
    rng = np.random.default_rng(9)
    for k in range(2):
        for _ in range(3):
            d = rng.standard_normal(U.shape[1]) * (fixed == 0)
            eps = 1e-6 * np.linalg.norm(U[k]) / np.linalg.norm(d)
            Up, Um = U.copy(), U.copy()
            Up[k] += eps * d
            Um[k] -= eps * d
            fd = (pnorm(Up, dims, rho) - pnorm(Um, dims, rho)) / (2 * eps)
            assert abs(fd - B[k] @ d) <= 1e-6 * abs(fd), (k, fd, B[k] @ d)
    assert np.all(B[:, fixed == 1] == 0)


def test_stress_field_is_the_displacement_route_sensitivity():
    # T_sigma(e) = sum_k rho_e lambda_k,e^T Ke u_k,e equals the derivative of
    # sigma_PN (stresses evaluated with the old densities) through the
    # displacements when element e's stiffness scale shrinks by a factor (1 - d)
    from oracle.stress import adjoint_rhs, pnorm, stress_field
    dims, rho, fixed, F, K, U = _stress_problem()
    Ke = fem.ke_gauss()
    B = adjoint_rhs(U, dims, rho, fixed)
    Lam = np.stack([solvers.solve_direct(K, fixed, b) for b in B])
    T = stress_field(dims, rho, Ke, U, Lam)
    for e in (0, 7, 25, 53):
        vals = []
        for d in (1e-5, -1e-5):
            r2 = rho.copy()
            r2[e] *= 1 - d
            K2 = fem.assemble(dims, r2, Ke)
            U2 = np.stack([solvers.solve_direct(K2, fixed, f) for f in F])
            vals.append(pnorm(U2, dims, rho))
        fd = (vals[0] - vals[1]) / 2e-5
        assert abs(fd - T[e]) <= 1e-5 * np.max(np.abs(T)), (e, fd, T[e])


def test_levelset_loop_with_stress_invariants():
    # J <= 100 J0 (inactive) and sigma_PN <= 1.5 sigma_PN0 with damping on a
    # 12x6x6 cantilever: every converged design satisfies both constraints,
    # the stress constraint is the one that binds, and the fixed points settle
    from oracle import levelset as ls
    dims = (12, 6, 6)
    p = ls.Params(alpha_J=100.0, alpha_sigma=1.5, dv_min=0.025 / 4, damping=True)
    (best, v, J), h = _loop_run(dims, p)
    S0 = h[0].S
    conv = [r for r in h if r.event == ls.FEA_CONVERGED]
    assert all(r.g <= 0 and r.g_s <= 0 and r.S <= 1.5 * S0 for r in conv)
    assert any(r.event == ls.FEA_VIOLATED and r.g_s > 0 and r.g <= 0 for r in h)
    assert conv[-1].S > 1.3 * S0 and conv[-1].v < 0.6
    assert not any(r.event == ls.FEA_DIVERGED for r in h)
    assert abs(h[0].g_s - (1 / 1.5 - 1)) < 1e-15


def _mid_span_load(dims):
    # unit -z force shared by the bottom nodes of the line x = nx/2 (along y)
    nx, ny, nz = dims
    f = np.zeros(3 * wl.n_nodes(dims))
    for j in range(ny + 1):
        f[3 * wl.node_id(dims, nx // 2, j, 0) + 2] = -1.0 / (ny + 1)
    return f


def test_levelset_loop_with_eigen_invariants():
    # J <= 3 J0 and lambda_1 >= lambda_10 with damping on a 12x6x4 cantilever
    # (unequal cross-section: the lowest eigenvalue stays simple, lambda_2 >=
    # 1.22 lambda_1 along the run) loaded at mid-span: the first volume steps take mass-dominated material
    # (T_lambda < 0, near the free end), so lambda_1 rises; later the
    # eigenvalue bound is the one that stops a step; every converged design
    # satisfies both constraints; mu_l / gamma_l follow Eq. 3.11-3.12
    from oracle import levelset as ls
    dims = (12, 6, 4)
    p = ls.Params(alpha_J=3.0, alpha_lambda=1.0, damping=True, dv_min=0.025 / 4)
    loop = ls.Loop(dims, p)
    (best, v, J), h = loop.run(wl.clamp_x0(dims), _mid_span_load(dims)[None])
    L0 = h[0].lam
    assert L0 > 0 and h[0].g_l == 0.0
    conv = [r for r in h if r.event == ls.FEA_CONVERGED]
    assert all(r.g <= 0 and r.g_l <= 0 and r.lam >= L0 for r in conv)
    assert conv[1].lam > conv[0].lam and conv[2].lam > conv[1].lam      # the field's sign
    assert any(r.event == ls.FEA_VIOLATED and r.g_l > 0 and r.g <= 0 for r in h)  # the eigenvalue bound binds
    mu, gamma, g_old = p.mu0, p.gamma0, None
    for k, r in enumerate(h):
        mu, gamma = ls.al_update(mu, gamma, r.g_l, g_old, k, p.varsigma, p.eta)
        g_old = r.g_l
        assert abs(mu - r.mu_l) <= 1e-12 * max(1.0, mu) and gamma == r.gamma_l, k
    assert conv[-1].v < 0.85 and h[-1].event == ls.FEA_TERMINATED
    # the same bound as a soft constraint (Sec. 3.6): it still shapes the
    # topology (the first steps are those of the hard run) but never stops a
    # step (only the compliance bound does), so the run goes deeper
    ps = ls.Params(alpha_J=3.0, alpha_lambda=1.0, lambda_soft=True, damping=True, dv_min=0.025 / 4)
    (best_s, v_s, J_s), hs = ls.Loop(dims, ps).run(wl.clamp_x0(dims), _mid_span_load(dims)[None])
    assert not any(r.event == ls.FEA_VIOLATED and r.g <= 0 for r in hs)
    assert any(r.g_l > 0 and r.g <= 0 and r.event != ls.FEA_VIOLATED for r in hs)
    conv_s = [r for r in hs if r.event == ls.FEA_CONVERGED]
    assert [r.nsolid for r in conv_s[:4]] == [r.nsolid for r in conv[:4]]
    assert conv_s[-1].v < conv[-1].v


def test_levelset_loop_with_buckling_invariants():
    # J <= 3 J0 and P >= 0.8 P0 with damping on an axially compressed 12x6x4
    # cantilever (plus a mid-edge load): every removal lowers the load
    # factor; the first volume step takes elements of small T_P (a field of
    # the wrong sign would take the critical ones and lose far more); the
    # buckling bound stops a step; mu_p / gamma_p follow Eq. 3.11-3.12; as a
    # soft bound it is exceeded without a step back and the run goes deeper
    from oracle import levelset as ls
    dims = (12, 6, 4)
    F = wl.edge_load(dims, "mid")
    for j in range(dims[1] + 1):
        for k in range(dims[2] + 1):
            F[3 * wl.node_id(dims, dims[0], j, k)] -= 1.0 / ((dims[1] + 1) * (dims[2] + 1))
    runs = {}
    for soft in (False, True):
        p = ls.Params(alpha_J=3.0, alpha_P=0.8, P_soft=soft, damping=True, dv_min=0.025 / 4)
        runs[soft] = (p, ls.Loop(dims, p).run(wl.clamp_x0(dims), F[None])[1])
    p, h = runs[False]
    P0 = h[0].P
    assert P0 > 0 and abs(h[0].g_p - (1 - 1 / 0.8)) < 1e-15
    conv = [r for r in h if r.event == ls.FEA_CONVERGED]
    assert all(r.g <= 0 and r.g_p <= 0 and r.P >= 0.8 * P0 for r in conv)
    assert 0.9 * P0 < conv[1].P < P0
    assert any(r.event == ls.FEA_VIOLATED and r.g_p > 0 and r.g <= 0 for r in h)
    mu, gamma, g_old = p.mu0, p.gamma0, None
    for k, r in enumerate(h):
        mu, gamma = ls.al_update(mu, gamma, r.g_p, g_old, k, p.varsigma, p.eta)
        g_old = r.g_p
        assert abs(mu - r.mu_p) <= 1e-12 * max(1.0, mu) and gamma == r.gamma_p, k
    ps, hs = runs[True]
    assert not any(r.event == ls.FEA_VIOLATED and r.g <= 0 for r in hs)
    assert any(r.g_p > 0 and r.g <= 0 and r.event != ls.FEA_VIOLATED for r in hs)
    conv_s = [r for r in hs if r.event == ls.FEA_CONVERGED]
    assert conv_s[-1].v < conv[-1].v


# ------------------------------------------------------------- modal analysis (Eq. 3.4, 3.21)
def test_mass_matrix_exact_and_quadrature():
    from oracle.modal import me_exact, me_gauss
    for h in ((1, 1, 1), (1, 2, Fraction(1, 2))):
        Mx = np.array([[float(v) for v in row] for row in me_exact(h)])
        assert np.max(np.abs(me_gauss(tuple(float(x) for x in h)) - Mx)) <= 1e-15 * np.max(Mx)
        vol = float(h[0] * h[1] * h[2])
        # one component of a unit translation carries the element's mass
        t = np.zeros(24)
        t[0::3] = 1.0
        assert abs(t @ Mx @ t - vol) <= 1e-15 * vol
    # per-component spectrum of the unit cube: products of the 1-D values 1/2, 1/6
    M = np.array([[float(v) for v in row] for row in me_exact((1, 1, 1))])
    ev = np.sort(np.linalg.eigvalsh(M[0::3, 0::3]))
    want = np.sort([1 / 8] + [1 / 24] * 3 + [1 / 72] * 3 + [1 / 216])
    assert np.allclose(ev, want, rtol=1e-14)


def test_single_element_modes_and_scaling():
    # a free element: six zero-energy modes, the rest positive; with the voxel
    # edges scaled by s the eigenvalues scale by 1/s^2 (K ~ s, M ~ s^3)
    from oracle.modal import me_gauss
    lam1 = sla.eigh(fem.ke_gauss(), me_gauss(), eigvals_only=True)
    assert np.sum(np.abs(lam1) < 1e-12) == 6 and np.all(lam1[6:] > 1e-3)
    lam2 = sla.eigh(fem.ke_gauss((2.0, 2.0, 2.0)), me_gauss((2.0, 2.0, 2.0)), eigvals_only=True)
    assert np.allclose(lam2[6:], lam1[6:] / 4, rtol=1e-12)


def _modal_problem(dims, seed=50):
    from oracle.modal import me_gauss
    rho = np.where(np.random.default_rng(seed).random(wl.n_elems(dims)) < 0.3, 1e-3, 1.0)
    fixed = wl.clamp_x0(dims)
    K = fem.assemble(dims, rho, fem.ke_gauss())
    M = fem.assemble(dims, rho, me_gauss())
    return rho, fixed, K, M


def test_lowest_modes_dense_and_lanczos_agree():
    from oracle.modal import lowest_modes
    dims = (12, 6, 6)  # 3,822 free DOFs: the shift-invert Lanczos branch
    rho, fixed, K, M = _modal_problem(dims)
    lam, Phi = lowest_modes(K, M, fixed, nev=3)
    Kff, free = fem.constrained_operator(K, fixed)
    Mff, _ = fem.constrained_operator(M, fixed)
    lam_d = sla.eigh(Kff.toarray(), Mff.toarray(), eigvals_only=True, subset_by_index=[0, 2])
    assert np.allclose(lam, lam_d, rtol=1e-10)
    for i in range(3):
        p = Phi[i]
        assert abs(p @ (M @ p) - 1) < 1e-12 and np.all(p[fixed == 1] == 0)
        res = Kff @ p[free] - lam[i] * (Mff @ p[free])
        assert np.linalg.norm(res) <= 1e-8 * lam[i] * np.linalg.norm(Mff @ p[free])
    assert abs(Phi[0] @ (M @ Phi[1])) < 1e-10


def test_eigen_sensitivity_is_the_derivative():
    # T_lambda(e) = rho_e phi^T (Ke - lambda Me) phi equals the drop of the
    # lowest eigenvalue when element e's stiffness and mass shrink by (1 - d)
    from oracle.modal import eigen_sensitivity, lowest_modes, me_gauss
    dims = (6, 4, 2)  # unequal cross-section: bending in y and z well apart
    rho, fixed, K, M = _modal_problem(dims, 51)
    lam, Phi = lowest_modes(K, M, fixed, 2)
    assert lam[1] > 1.05 * lam[0]  # a simple eigenvalue
    Ke, Me = fem.ke_gauss(), me_gauss()
    T = eigen_sensitivity(dims, rho, Ke, Me, lam[0], Phi[0])
    for e in (0, 9, 31, 47):
        vals = []
        for d in (1e-5, -1e-5):
            r2 = rho.copy()
            r2[e] *= 1 - d
            l2, _ = lowest_modes(fem.assemble(dims, r2, Ke), fem.assemble(dims, r2, Me), fixed, 1)
            vals.append(l2[0])
        fd = (vals[1] - vals[0]) / 2e-5
        assert abs(fd - T[e]) <= 1e-6 * np.max(np.abs(T)), (e, fd, T[e])


# ------------------------------------------------------------- linear buckling (Eq. 3.5)
def test_geometric_stiffness_quadrature_and_closed_forms():
    from oracle.buckling import kg_element, kg_gauss
    rng = np.random.default_rng(80)
    h = (1.0, 2.0, 0.5)
    S = rng.standard_normal((3, 3))
    S = S + S.T
    Kg = kg_element(S, h)
    assert np.max(np.abs(Kg - kg_gauss(S, h))) <= 1e-14 * np.max(np.abs(Kg))
    assert np.allclose(Kg, Kg.T, atol=1e-15)
    X = fem.LOCAL * np.asarray(h)
    for c in range(3):  # translations carry no geometric energy
        t = np.zeros(24)
        t[c::3] = 1.0
        assert np.max(np.abs(Kg @ t)) <= 1e-13 * np.max(np.abs(Kg))
    # u_y = theta x + phi y: int S_pq du_y/dx_p du_y/dx_q = (S_xx th^2 + 2 S_xy th ph + S_yy ph^2) V
    th, ph = 0.7, -0.3
    u = np.zeros(24)
    u[1::3] = th * X[:, 0] + ph * X[:, 1]
    V = h[0] * h[1] * h[2]
    want = (S[0, 0] * th * th + 2 * S[0, 1] * th * ph + S[1, 1] * ph * ph) * V
    assert abs(u @ Kg @ u - want) <= 1e-13 * abs(want)


def _buckling_problem(dims):
    from oracle import stress
    from oracle.buckling import prebuckling_stress
    rng = np.random.default_rng(81)
    rho = np.where(rng.random(wl.n_elems(dims)) < 0.2, 1e-3, 1.0)
    fixed = wl.clamp_x0(dims)
    f = wl.edge_load(dims, "mid")
    # an axial compression of the x = L face plus the transverse edge load
    for j in range(dims[1] + 1):
        for k in range(dims[2] + 1):
            f[3 * wl.node_id(dims, dims[0], j, k)] -= 1.0 / ((dims[1] + 1) * (dims[2] + 1))
    K = fem.assemble(dims, rho, fem.ke_gauss())
    u = solvers.solve_direct(K, fixed, f)
    sig = prebuckling_stress(dims, rho, u)
    assert np.all(sig[rho < 0.5] == 0) and np.all(sig[rho >= 0.5] == stress.element_stress(dims, rho, u)[rho >= 0.5])
    return rho, fixed, f, K, u, sig


def test_buckling_modes_dense_and_lanczos_agree():
    from oracle.buckling import assemble_kg, buckling_modes
    dims = (12, 6, 6)
    rho, fixed, f, K, u, sig = _buckling_problem(dims)
    Kg = assemble_kg(dims, sig)
    lam, Phi = buckling_modes(K, Kg, fixed, 2)   # Lanczos branch (3,822 free DOFs)
    Kff, free = fem.constrained_operator(K, fixed)
    Gff, _ = fem.constrained_operator(Kg, fixed)
    mu = sla.eigh(-Gff.toarray(), Kff.toarray(), eigvals_only=True)
    want = np.sort(1.0 / mu[mu > 0])[:2]
    assert np.allclose(lam, want, rtol=1e-9)
    for i in range(2):
        p = Phi[i][free]
        assert abs(p @ (Kff @ p) - 1) < 1e-12
        r = Kff @ p + lam[i] * (Gff @ p)
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(Kff @ p)


def test_buckling_sensitivity_is_the_derivative():
    # with the prebuckling stresses held (scaled with rho_e), T_P(e) is the
    # drop of the smallest load factor when element e's scale shrinks by (1 - d)
    from oracle.buckling import assemble_kg, buckling_modes, buckling_sensitivity
    dims = (6, 3, 3)
    rho, fixed, f, K, u, sig = _buckling_problem(dims)
    Ke = fem.ke_gauss()
    lam, Phi = buckling_modes(K, assemble_kg(dims, sig), fixed, 2)
    assert lam[1] > 1.05 * lam[0]
    T = buckling_sensitivity(dims, rho, Ke, sig, lam[0], Phi[0])
    for e in (0, 7, 30, 53):
        vals = []
        for d in (1e-5, -1e-5):
            r2 = rho.copy()
            r2[e] *= 1 - d
            s2 = sig * (r2 / rho)[:, None]
            l2, _ = buckling_modes(fem.assemble(dims, r2, Ke), assemble_kg(dims, s2), fixed, 1)
            vals.append(l2[0])
        fd = (vals[1] - vals[0]) / 2e-5
        assert abs(fd - T[e]) <= 1e-6 * np.max(np.abs(T)), (e, fd, T[e])
