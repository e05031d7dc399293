"""Pins of the oracle's tableaux and small s x s quantities against facts the
paper and textbook theory fix (closed forms, order conditions, Pade
approximants, Table 1, the worked example of equation (Gauss4Radau3_example))."""
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import tableau as tb

FAMILIES = ("gauss", "radau", "lobatto")
CASES = [(f, s) for f in FAMILIES for s in (1, 2, 3, 4, 5) if not (f == "lobatto" and s == 1)]


def test_closed_forms_one_and_two_stages():
    # Gauss s=1: implicit midpoint; Radau IIA s=1: backward Euler
    A, b, c = tb.tableau("gauss", 1)
    assert np.allclose(A, [[0.5]], atol=1e-16) and np.allclose(b, [1.0]) and np.allclose(c, [0.5])
    A, b, c = tb.tableau("radau", 1)
    assert np.allclose(A, [[1.0]], atol=1e-16) and np.allclose(b, [1.0]) and np.allclose(c, [1.0])
    # Gauss s=2: c = 1/2 -+ sqrt(3)/6
    r3 = math.sqrt(3.0)
    A, b, c = tb.tableau("gauss", 2)
    assert np.allclose(c, [0.5 - r3 / 6, 0.5 + r3 / 6], atol=1e-15, rtol=0)
    assert np.allclose(A, [[0.25, 0.25 - r3 / 6], [0.25 + r3 / 6, 0.25]], atol=1e-15, rtol=0)
    assert np.allclose(b, [0.5, 0.5], atol=1e-15, rtol=0)
    # Radau IIA s=2: c = (1/3, 1)
    A, b, c = tb.tableau("radau", 2)
    assert np.allclose(c, [1 / 3, 1.0], atol=1e-15, rtol=0)
    assert np.allclose(A, [[5 / 12, -1 / 12], [0.75, 0.25]], atol=1e-15, rtol=0)
    assert np.allclose(b, [0.75, 0.25], atol=1e-15, rtol=0)
    # Lobatto IIIC s=2 and s=3 (the textbook tables)
    A, b, c = tb.tableau("lobatto", 2)
    assert np.allclose(c, [0.0, 1.0], atol=0) and np.allclose(b, [0.5, 0.5], atol=1e-16, rtol=0)
    assert np.allclose(A, [[0.5, -0.5], [0.5, 0.5]], atol=1e-16, rtol=0)
    A, b, c = tb.tableau("lobatto", 3)
    assert np.allclose(c, [0.0, 0.5, 1.0], atol=1e-16, rtol=0)
    assert np.allclose(b, [1 / 6, 2 / 3, 1 / 6], atol=1e-16, rtol=0)
    assert np.allclose(A, [[1 / 6, -1 / 3, 1 / 6], [1 / 6, 5 / 12, -1 / 12], [1 / 6, 2 / 3, 1 / 6]],
                       atol=1e-16, rtol=0)


@pytest.mark.parametrize("family,s", CASES)
def test_order_conditions(family, s):
    """B(p): sum_i b_i c_i^{k-1} = 1/k for k <= p (p = 2s Gauss, 2s-1 Radau
    IIA, 2s-2 Lobatto IIIC), failing at k = p+1; C(q): sum_j a_ij c_j^{k-1} =
    c_i^k / k for k <= q (q = s collocation, s-1 Lobatto IIIC, whose C(s)
    fails); Lobatto IIIC also has a_i1 = b_1 and a_sj = b_j."""
    A, b, c = tb.tableau(family, s)
    p = {"gauss": 2 * s, "radau": 2 * s - 1, "lobatto": 2 * s - 2}[family]
    for k in range(1, p + 1):
        assert abs(b @ c ** (k - 1) - 1.0 / k) < 2e-15
    assert abs(b @ c ** p - 1.0 / (p + 1)) > 1e-6
    q = s - 1 if family == "lobatto" else s
    for k in range(1, q + 1):
        assert np.max(np.abs(A @ c ** (k - 1) - c ** k / k)) < 2e-15
    if family == "lobatto":
        assert np.max(np.abs(A @ c ** (s - 1) - c ** s / s)) > 1e-6
        assert np.max(np.abs(A[:, 0] - b[0])) < 2e-16
    if family in ("radau", "lobatto"):
        assert np.max(np.abs(A[-1] - b)) < 2e-16   # stiffly accurate


@pytest.mark.parametrize("family,s", CASES)
def test_stability_function_is_pade(family, s):
    """R(z) = Pade (s,s) of e^z for Gauss, (s-1,s) for Radau IIA, (s-2,s) for
    Lobatto IIIC."""
    A, b, c = tb.tableau(family, s)
    k = {"gauss": s, "radau": s - 1, "lobatto": s - 2}[family]
    for z in (-0.3, -2.0, -50.0, 3j, -1 + 2j, 0.4, -1e3):
        R = tb.stability_function(A, b, z)
        P = tb.pade_exp(k, s, z)
        assert abs(R - P) <= 1e-13 * max(1.0, abs(P)), (z, R, P)


@pytest.mark.parametrize("family,s", CASES)
def test_assumption1_positive_real_part(family, s):
    """Assumption 1 (Section 2.2): eigenvalues of A0 have positive real part."""
    A, _, _ = tb.tableau(family, s)
    assert np.all(np.linalg.eigvals(A).real > 0)


def test_table1_condition_bounds():
    """Table 1: kappa(P_gamma*) bound per eigenvalue (pair) of A0^{-1}.
    The printed s=4 entries sit up to 0.007 above the recomputed ones, so the
    tolerance is 0.011 there and half a unit of the last digit elsewhere."""
    for row in read_golden("table1_kappa.txt"):
        fam, s = row[0], int(row[1])
        printed = [float(v) for v in row[2:]]
        A, _, _ = tb.tableau(fam, s)
        eigs = tb.inverse_eigs(A)
        got = [tb.kappa_bound(e, bt) if bt > 0 else 1.0 for e, bt in eigs]
        assert len(got) == len(printed)
        tol = 0.011 if s == 4 else 0.0051
        for g, p in zip(got, printed):
            assert abs(g - p) <= tol, (fam, s, got, printed)


def test_gamma_star_closed_forms():
    """gamma_* = eta + beta^2/eta (equation (gamma*)).  Two-stage closed forms:
    Gauss A0^{-1} has eigenvalues 3 +- i sqrt(3) (gamma_* = 4); Radau IIA
    2 +- i sqrt(2) (gamma_* = 3)."""
    for fam, eta, beta, gs in (("gauss", 3.0, math.sqrt(3.0), 4.0),
                               ("radau", 2.0, math.sqrt(2.0), 3.0)):
        A, _, _ = tb.tableau(fam, 2)
        (e, bt), = tb.inverse_eigs(A)
        assert abs(e - eta) < 1e-13 and abs(bt - beta) < 1e-13
        assert abs(tb.gamma_star(e, bt) - gs) < 1e-13


def test_worked_example_d_weights():
    """Equation (Gauss4Radau3_example): d-weights of the real Schur basis."""
    for row in read_golden("worked_example_d.txt"):
        fam, s, k, l = row[0], int(row[1]), int(row[2]) - 1, int(row[3]) - 1
        want = np.array([float(v) for v in row[4:]])
        A, _, _ = tb.tableau(fam, s)
        Q, R = tb.real_schur_standard(np.linalg.inv(A))
        assert np.allclose(Q @ R @ Q.T, np.linalg.inv(A), atol=1e-13)
        d = tb.d_weights(Q)
        assert np.max(np.abs(d[k, l] - want)) <= 5e-4, (fam, k, l, d[k, l], want)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_d_weights_sum_to_kronecker_delta(seed):
    """sum_i (d_{k,l})_i = delta_{kl} for any invertible similarity T."""
    rng = np.random.default_rng(seed)
    T = rng.standard_normal((5, 5)) + 3 * np.eye(5)
    d = tb.d_weights(T)
    assert np.max(np.abs(d.sum(axis=2) - np.eye(5))) < 1e-13


def _butcher_conditions(A, b, c):
    """Residuals of the order conditions, grouped by order (rooted trees up
    to order 5)."""
    return {
        1: [b.sum() - 1],
        2: [b @ c - 1 / 2],
        3: [b @ c ** 2 - 1 / 3, b @ A @ c - 1 / 6],
        4: [b @ c ** 3 - 1 / 4, (b * c) @ A @ c - 1 / 8, b @ A @ c ** 2 - 1 / 12, b @ A @ A @ c - 1 / 24],
        5: [b @ c ** 4 - 1 / 5, (b * c ** 2) @ A @ c - 1 / 10, (b * c) @ A @ c ** 2 - 1 / 15,
            (b * c) @ A @ A @ c - 1 / 30, b @ (A @ c) ** 2 - 1 / 20, b @ A @ c ** 3 - 1 / 20,
            b @ A @ (c * (A @ c)) - 1 / 40, b @ A @ A @ c ** 2 - 1 / 60, b @ A @ A @ A @ c - 1 / 120],
    }


@pytest.mark.parametrize("s,p", [(1, 1), (2, 2), (3, 3), (5, 4)])
def test_sdirk_published_methods(s, p):
    """SDIRK comparison methods: singly diagonally implicit (lower triangular,
    constant diagonal), stiffly accurate, all order conditions (rooted trees)
    up to order p and not all of order p+1, L-stable (|R(iy)| <= 1, R -> 0)."""
    A, b, c = tb.tableau("sdirk", s)
    assert np.allclose(np.triu(A, 1), 0.0) and np.allclose(np.diag(A), A[0, 0])
    assert np.max(np.abs(A[-1] - b)) < 1e-16 and np.max(np.abs(A.sum(axis=1) - c)) < 4e-15
    cond = _butcher_conditions(A, b, c)
    for q in range(1, p + 1):
        assert max(abs(x) for x in cond[q]) < 3e-15, (q, cond[q])
    assert max(abs(x) for x in cond[p + 1]) > 1e-4
    for y in (0.1, 1.0, 10.0, 1e3):
        assert abs(tb.stability_function(A, b, 1j * y)) <= 1 + 1e-14
    assert abs(tb.stability_function(A, b, -1e9)) < 1e-6
    if s == 3:   # gamma is the root of x^3 - 3x^2 + 3x/2 - 1/6 in (1/3, 1/2)
        g = A[0, 0]
        assert 1 / 3 < g < 1 / 2 and abs(g ** 3 - 3 * g ** 2 + 1.5 * g - 1 / 6) < 1e-15
