"""CPU check of the two-ended super-block order used by the coarse factor.

The library orders the banded coarse matrix E (half bandwidth w <= P) in K
super-blocks of P unknowns: chain A (super-blocks 0..m-1, unchanged), chain B
(super-blocks K-1..m+1, in reverse order and with their unknowns reversed) and
the middle super-block m (reversed) last, m = (K-1)/2.  This test restates that
order and the windowed block Cholesky and triangular solves the library
performs on it (the coupling windows: first w rows / last w columns for the
chain couplings, last w rows / last w columns for the middle's coupling X to
chain A's end), in plain numpy, and checks the result against a dense solve
of the same symmetric positive definite banded system.  It pins the algebra
of the order; the GPU tests pin the library's kernels against the oracle.
"""
import numpy as np
import pytest


def twist_position(q, P, K, m):
    j, r = divmod(q, P)
    if j < m:
        return q
    if j == m:
        return (K - 1) * P + (P - 1 - r)
    return (m + K - 1 - j) * P + (P - 1 - r)


def windowed_solve(E, g, P, w):
    n = E.shape[0]
    K = -(-n // P)
    m = (K - 1) // 2
    npad, o = K * P, P - w
    perm = [twist_position(q, P, K, m) for q in range(n)]
    assert sorted(perm) == sorted(set(perm)) and max(perm) < npad
    Ep = np.eye(npad)
    Ep[np.ix_(perm, perm)] = E
    blk = lambda a, b: Ep[a * P:(a + 1) * P, b * P:(b + 1) * P].copy()
    # the only couplings below the diagonal, and their windows
    for kr in range(K):
        for kc in range(kr):
            chain = kr == kc + 1 and kc != m - 1
            middle_x = kr == K - 1 and kc == m - 1
            Bk = blk(kr, kc)
            if chain:
                assert not Bk[w:, :].any() and not Bk[:, :o].any()
            elif middle_x:
                assert not Bk[:o, :].any() and not Bk[:, :o].any()
            else:
                assert not Bk.any()
    D = [blk(k, k) for k in range(K)]
    B = [blk(k + 1, k) if k + 1 < K else None for k in range(K)]
    if m >= 1:
        B[m - 1] = blk(K - 1, m - 1)
    Li = [None] * K
    T = [np.zeros((P, P)) for _ in range(K)]
    U = [np.zeros((P, P)) for _ in range(K)]
    Cx = None
    for k in range(K):
        Dk = D[k]
        pred, mid_x = k > 0 and k != m, k == K - 1 and m >= 1
        if pred:
            Dk[:w, :w] -= B[k - 1][:w, o:] @ B[k - 1][:w, o:].T
        if mid_x:
            Dk[o:, o:] -= Cx @ Cx.T
        Li[k] = np.linalg.inv(np.linalg.cholesky(Dk))
        if pred:
            T[k][:, o:] = Li[k][:, :w] @ B[k - 1][:w, o:]
        if mid_x:
            T[m][:, o:] = Li[k][:, o:] @ Cx
        if k == m - 1:
            Cx = B[m - 1][o:, o:] @ Li[k][o:, o:].T
            U[k][:, o:] = Li[k][o:, :].T @ Cx.T
        elif k < K - 1:
            B[k][:w, o:] = B[k][:w, o:] @ Li[k][o:, o:].T
            U[k][:, :w] = Li[k][o:, :].T @ B[k][:w, o:].T
    gp = np.zeros(npad)
    gp[perm] = g
    x = [Li[k] @ gp[k * P:(k + 1) * P] for k in range(K)]
    la, lb = max(m - 1, 0), max(K - 2 - m, 0)
    for q in range(1, max(la, lb) + 1):  # the paired chain steps
        for pos in ([q] if q <= la else []) + ([m + q] if q <= lb else []):
            x[pos] = x[pos] - T[pos][:, o:] @ x[pos - 1][o:]
    if K >= 2:
        x[K - 1] = x[K - 1] - T[K - 1][:, o:] @ x[K - 2][o:]
    if m >= 1:
        x[K - 1] = x[K - 1] - T[m][:, o:] @ x[m - 1][o:]
    mu = [Li[k].T @ x[k] for k in range(K)]
    if K >= 2:
        mu[K - 2] = mu[K - 2] - U[K - 2][:, :w] @ mu[K - 1][:w]
    if m >= 1:
        mu[m - 1] = mu[m - 1] - U[m - 1][:, o:] @ mu[K - 1][o:]
    for q in range(1, max(la, lb) + 1):
        for pos in ([m - 1 - q] if q <= la else []) + ([K - 2 - q] if q <= lb else []):
            mu[pos] = mu[pos] - U[pos][:, :w] @ mu[pos + 1][:w]
    return np.concatenate(mu)[perm], K


# includes w = P (the coupling windows then cover whole super-blocks)
@pytest.mark.parametrize("n,w,P", [(40, 8, 48), (100, 20, 48), (130, 30, 32), (200, 30, 32), (324, 60, 64),
                                   (500, 40, 48), (768, 60, 64), (256, 32, 32), (300, 48, 48)])
def test_two_ended_block_cholesky_solves(n, w, P):
    rng = np.random.default_rng(n + w + P)
    E = np.zeros((n, n))
    for i in range(n):
        for j in range(max(0, i - w), i + 1):
            E[i, j] = E[j, i] = rng.standard_normal()
    E += (2 * w + 2) * 3.0 * np.eye(n)  # diagonally dominant: SPD
    g = rng.standard_normal(n)
    got, K = windowed_solve(E, g, P, w)
    want = np.linalg.solve(E, g)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want), K
