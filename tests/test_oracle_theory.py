"""Dense checks of the preconditioning theory the GPU path relies on
(Section 4): the condition bounds of Corollary 1, the Remark on symmetric
definite / skew-symmetric operators and Theorem 2, and the two-iteration
property of GMRES with the exact block lower-triangular preconditioner
(equation (Lprec))."""
import numpy as np
import pytest

from oracle import tableau as tb


def _lap1d(n, scale):
    L = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    L[0, -1] = L[-1, 0] = 1.0
    return scale * L


def _adv1d(n, scale):
    D = np.eye(n, k=1) - np.eye(n, k=-1)
    D[0, -1], D[-1, 0] = -1.0, 1.0
    return scale * D


def _pairs():
    out = []
    for fam in ("gauss", "radau"):
        for s in (2, 3, 4, 5):
            A, _, _ = tb.tableau(fam, s)
            out += [(fam, s, e, b) for e, b in tb.inverse_eigs(A) if b > 0]
    return out


def _kappa_pgamma(L1, L2, eta, beta, gamma):
    """Two-norm condition number of the right-preconditioned Schur complement
    P_gamma = [eta I - L2 + beta^2 (eta I - L1)^{-1}] (gamma I - L2)^{-1}."""
    n = L1.shape[0]
    I = np.eye(n)
    S = eta * I - L2 + beta ** 2 * np.linalg.inv(eta * I - L1)
    P = S @ np.linalg.inv(gamma * I - L2)
    return np.linalg.cond(P)


@pytest.mark.parametrize("fam,s,eta,beta", _pairs())
def test_corollary1_and_remark_bounds(fam, s, eta, beta):
    gs = tb.gamma_star(eta, beta)
    for scale in (0.1, 10.0, 1e4):
        L = _lap1d(24, scale)                 # symmetric negative semi-definite
        k = _kappa_pgamma(L, L, eta, beta, gs)
        assert k <= 0.5 * (1 + np.sqrt(1 + beta ** 2 / eta ** 2)) + 1e-9
        assert k <= tb.kappa_bound(eta, beta) + 1e-9
        L = _adv1d(24, scale)                 # skew-symmetric
        assert _kappa_pgamma(L, L, eta, beta, gs) <= tb.kappa_bound(eta, beta) + 1e-9


@pytest.mark.parametrize("fam,s,eta,beta", _pairs()[:4])
def test_theorem2_bound(fam, s, eta, beta):
    """L1 != L2 with <L1 w, L2 w> >= 0: kappa <= 2 + beta^2/eta^2."""
    rng = np.random.default_rng(0)
    gs = tb.gamma_star(eta, beta)
    for _ in range(5):
        L1 = _lap1d(20, 30.0)
        d = np.diag(rng.uniform(0.5, 2.0, 20))
        L2 = d @ L1 @ d                       # SNSD, same null space
        w = rng.standard_normal((20, 50))
        assert np.all(np.einsum("ij,ij->j", L1 @ w, L2 @ w) >= -1e-9)
        assert _kappa_pgamma(L1, L2, eta, beta, gs) <= 2 + beta ** 2 / eta ** 2 + 1e-9


def _gmres_iterations(Aop, Pinv, b, tol=1e-12, maxit=20):
    """Right-preconditioned GMRES; returns iterations to reach tol."""
    n = b.size
    V = np.zeros((n, maxit + 1))
    H = np.zeros((maxit + 1, maxit))
    beta0 = np.linalg.norm(b)
    V[:, 0] = b / beta0
    for j in range(maxit):
        w = Aop @ (Pinv @ V[:, j])
        for i in range(j + 1):
            H[i, j] = V[:, i] @ w
            w -= H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        e1 = np.zeros(j + 2)
        e1[0] = beta0
        y, *_ = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)
        if np.linalg.norm(H[: j + 2, : j + 1] @ y - e1) <= tol * beta0:
            return j + 1
        if H[j + 1, j] < 1e-300:
            return j + 1
        V[:, j + 1] = w / H[j + 1, j]
    return maxit


@pytest.mark.parametrize("fam,s,eta,beta", _pairs()[:3])
def test_exact_triangular_preconditioner_two_iterations(fam, s, eta, beta):
    """With exact diagonal inverses and the exact Schur complement, GMRES on
    the 2x2 block system converges in two iterations (Section 4)."""
    n = 16
    I = np.eye(n)
    L1 = _lap1d(n, 50.0) + _adv1d(n, 3.0)
    L2 = _lap1d(n, 40.0) + _adv1d(n, 2.0)
    phi = beta
    Ablk = np.block([[eta * I - L1, phi * I], [-beta ** 2 / phi * I, eta * I - L2]])
    S = eta * I - L2 + beta ** 2 * np.linalg.inv(eta * I - L1)
    Lp = np.block([[eta * I - L1, 0 * I], [-beta ** 2 / phi * I, S]])
    b = np.random.default_rng(1).standard_normal(2 * n)
    assert _gmres_iterations(Ablk, np.linalg.inv(Lp), b) <= 2
