"""Pins of the oracle's tableaux and small s x s quantities against facts the
paper and textbook theory fix (closed forms, order conditions, Pade
approximants, Table 1, the worked example of equation (Gauss4Radau3_example))."""
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import tableau as tb

FAMILIES = ("gauss", "radau")


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


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_order_conditions(family, s):
    """B(p): sum_i b_i c_i^{k-1} = 1/k for k <= p (p = 2s Gauss, 2s-1 Radau IIA),
    failing at k = p+1; C(s): sum_j a_ij c_j^{k-1} = c_i^k / k for k <= s."""
    A, b, c = tb.tableau(family, s)
    p = 2 * s if family == "gauss" else 2 * s - 1
    for k in range(1, p + 1):
        assert abs(b @ c ** (k - 1) - 1.0 / k) < 2e-15
    assert abs(b @ c ** p - 1.0 / (p + 1)) > 1e-6
    for k in range(1, s + 1):
        assert np.max(np.abs(A @ c ** (k - 1) - c ** k / k)) < 2e-15
    if family == "radau":
        assert np.max(np.abs(A[-1] - b)) < 2e-16   # stiffly accurate


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_stability_function_is_pade(family, s):
    """R(z) = Pade (s,s) of e^z for Gauss, (s-1,s) for Radau IIA."""
    A, b, c = tb.tableau(family, s)
    k = s if family == "gauss" else s - 1
    for z in (-0.3, -2.0, -50.0, 3j, -1 + 2j, 0.4, -1e3):
        R = tb.stability_function(A, b, z)
        P = tb.pade_exp(k, s, z)
        assert abs(R - P) <= 1e-13 * max(1.0, abs(P)), (z, R, P)


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
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
