"""Pins of the oracle's eigenbasis and eigen-block operators (Sections 3.1,
3.2): the block operators of the Newton-like truncations are written out in
``oracle.newton.block_operator``; here they are tied to the exact Newton
matrix of the stage equations, which is built from A alone."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import newton as nw
from oracle import problems as pb
from oracle import tableau as tb
from paper_2101_01776_amd import inputs


def _lam(blocks, s):
    L = np.zeros((s, s))
    for first, width, eta, beta in blocks:
        L[first, first] = eta
        if width == 2:
            L[first, first + 1] = beta
            L[first + 1, first] = -beta
            L[first + 1, first + 1] = eta
    return L


@pytest.mark.parametrize("family,s", [(f, s) for f in ("gauss", "radau") for s in (1, 2, 3, 4, 5)]
                         + [("lobatto", 3), ("lobatto", 4), ("lobatto", 5)])
def test_real_eigenbasis(family, s):
    """A0^{-1} T = T Lambda, the eigenvalues are those of A0^{-1}, and the
    normalization holds: unit columns (|a|^2 + |b|^2 = 1 for a pair), a
    orthogonal to b with |a| >= |b|, largest entry positive; the d weights of
    every transformed row sum to 1 over the stages and those of two different
    rows to 0 (T^{-1} T = I)."""
    A, _, _ = tb.tableau(family, s)
    T, blocks = tb.real_eigenbasis(A)
    Ainv = np.linalg.inv(A)
    assert np.abs(Ainv @ T - T @ _lam(blocks, s)).max() <= 1e-13 * np.abs(Ainv).max()
    want = tb.inverse_eigs(A)
    assert [(e, b) for _, _, e, b in blocks] == pytest.approx(want, rel=1e-12, abs=1e-12)
    for first, width, _, _ in blocks:
        a = T[:, first]
        if width == 1:
            assert abs(a @ a - 1) < 1e-14
        else:
            bb = T[:, first + 1]
            assert abs(a @ a + bb @ bb - 1) < 1e-14 and abs(a @ bb) < 1e-14 and a @ a >= bb @ bb
        assert a[np.argmax(np.abs(a))] > 0
    d = tb.d_weights(T)
    np.testing.assert_allclose(d.sum(axis=2), np.eye(s), atol=1e-12)


def _transformed_newton(problem, A, c, u, t, dt, K, T, blocks):
    """(T^{-1} (x) I) J (T Lambda (x) I) for the exact Newton matrix J of the
    stage equations (block (i, j) = delta_ij M - dt a_ij L(U_i))."""
    s = len(c)
    S, Ub, Vb = nw._newton_matrix(problem, A, c, u, t, dt, K)
    assert Ub is None
    J = S.toarray()
    N = problem.size
    Tl = T @ _lam(blocks, s)
    return np.kron(np.linalg.inv(T), np.eye(N)) @ J @ np.kron(Tl, np.eye(N))


def _case(kind):
    if kind == "burgers":
        prob = pb.Burgers1D(16, 0.01)
        u = inputs.burgers_u0(16, 3)
        return prob, u, 1e-2
    prob = pb.NonlinearDiffusion2D(6)
    u = inputs.nldiff_random_u0(6, 11).ravel()
    return prob, u, 5e-3


@pytest.mark.parametrize("kind", ["burgers", "nldiff"])
@pytest.mark.parametrize("family,s", [("gauss", 2), ("gauss", 3), ("radau", 3), ("gauss", 5)])
def test_block_operators_against_exact_newton(kind, family, s):
    """Newton-like (3) in the eigenbasis is the diagonal block of the
    transformed exact Newton matrix (for 2-stage methods: exact Newton, as
    the paper notes); (2) is that block without the L-terms that couple the
    two rows of a pair; (1) and (0) lump each row's stage weights.  On a
    U-independent operator every truncation is the same (the weights of a
    row sum to 1).  (For Gauss-2 the eigenbasis weights happen to be one-hot
    with no coupling between the two rows, so there (1) = (2) = (3) = exact
    Newton.)"""
    prob, u, dt = _case(kind)
    A, _, c = tb.tableau(family, s)
    T, blocks = tb.real_eigenbasis(A)
    rng = np.random.default_rng(5)
    K = 0.3 * rng.standard_normal((s, prob.size))
    Jt = _transformed_newton(prob, A, c, u, 0.1, dt, K, T, blocks)
    N = prob.size
    M = np.diag(prob.mass)
    scale = np.abs(Jt).max()
    for blk in blocks:
        first, width, eta, beta = blk
        sl = slice(first * N, (first + width) * N)
        D3 = nw.block_operator(prob, A, c, u, 0.1, dt, K, T, blk, 3).toarray()
        np.testing.assert_allclose(D3, Jt[sl, sl], atol=1e-13 * scale)
        D2 = nw.block_operator(prob, A, c, u, 0.1, dt, K, T, blk, 2).toarray()
        want2 = Jt[sl, sl].copy()
        if width == 2:
            want2[:N, N:] = beta * M
            want2[N:, :N] = -beta * M
        np.testing.assert_allclose(D2, want2, atol=1e-13 * scale)
    if s == 2:
        # one pair block: Newton-like (3) is the whole transformed Jacobian
        np.testing.assert_allclose(nw.block_operator(prob, A, c, u, 0.1, dt, K, T, blocks[0], 3).toarray(), Jt,
                                   atol=1e-13 * scale)
    lin = pb.NonlinearDiffusion2D(6, kappa_quadratic=False)
    ul = inputs.nldiff_random_u0(6, 11).ravel()
    Kl = 0.3 * rng.standard_normal((s, lin.size))
    for blk in blocks:
        ops = [nw.block_operator(lin, A, c, ul, 0.1, dt, Kl, T, blk, v).toarray() for v in range(3)]
        for o in ops[1:]:
            np.testing.assert_allclose(o, ops[0], atol=1e-12 * np.abs(ops[0]).max())


@pytest.mark.parametrize("family,s,row", [("gauss", 3, 0), ("gauss", 5, 0), ("lobatto", 3, 0)])
def test_lumped_stage_tie_break(family, s, row):
    """Newton-like (1) lumps a row to its largest stage weight.  On the real
    eigenvalue's row of Gauss-3, Gauss-5 and Lobatto IIIC-3 the two largest
    weights are the mirror pair d_rr,k = d_rr,s-1-k (equal to rounding), so
    the convention -- the lowest stage index among weights within a relative
    1e-12 of the largest -- picks stage 0; rows with a clear maximum keep
    their argmax."""
    A, _, _ = tb.tableau(family, s)
    T, _ = tb.real_eigenbasis(A)
    d = tb.d_weights(T)
    w = np.abs(d[row, row, :])
    k = int(np.argmax(w))
    assert abs(w[k] - w[s - 1 - k]) <= 1e-14 * w[k] and k != s - 1 - k
    assert nw.lumped_stage(d[row, row, :]) == min(k, s - 1 - k) == 0
    for r in range(s):
        if r == row:
            continue
        wr = np.sort(np.abs(d[r, r, :]))
        assert wr[-1] - wr[-2] > 1e-3
        assert nw.lumped_stage(d[r, r, :]) == int(np.argmax(np.abs(d[r, r, :])))
