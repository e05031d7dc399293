"""Runge-Kutta tableaux and the small s x s quantities of the paper (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

* Gauss and Radau IIA are the collocation methods named in Section 2.2
  (Assumption 1 holds for both).  Their nodes c are the roots of the shifted
  Legendre polynomial P_s(2x-1) (Gauss) and of P_s(2x-1) - P_{s-1}(2x-1)
  (Radau IIA, which puts c_s = 1); the collocation conditions give
  a_ij = int_0^{c_i} l_j and b_j = int_0^1 l_j for the Lagrange basis l_j on c.
  Roots and integrals are computed with mpmath at 60 digits and rounded to
  float64 once, at the end.
* Lobatto IIIC (named with Gauss and Radau IIA in Section 2.2 and Table 1)
  has the Lobatto nodes c_1 = 0, c_s = 1 and the interior roots of the
  derivative of P_{s-1}(2x-1), the Lobatto quadrature weights b_j =
  int_0^1 l_j, and the A with first column a_i1 = b_1 that satisfies the
  simplifying conditions C(s-1): sum_j a_ij c_j^{k-1} = c_i^k / k,
  k = 1..s-1 (Chipman's construction); order 2s-2, stability function the
  (s-2, s) Pade approximant.  s >= 2.
* SDIRK (singly diagonally implicit, the paper's comparison class): the
  paper prints no tableau, so the published L-stable methods are used:
  s = 1 backward Euler; s = 2 Alexander's two-stage order-2 method
  (gamma = 1 - 1/sqrt 2); s = 3 Alexander's three-stage order-3 method
  (gamma the root of x^3 - 3x^2 + 3x/2 - 1/6 in (1/3, 1/2)); s = 5 the
  five-stage order-4 method of Hairer and Wanner (gamma = 1/4).  All are
  stiffly accurate (b = last row of A).
* ``inverse_eigs`` gives the eigenvalues eta +- i beta of A0^{-1}
  (Section 3), ``gamma_star`` equation (gamma*), ``kappa_bound`` equation
  (kappa_gamma*_L1=L2) as tabulated in Table 1, and ``d_weights`` the vectors
  d_{k,l} of equation (Q0approx) for any similarity transform.
* ``real_schur_standard`` is the real Schur form A0^{-1} = Q0 R0 Q0^T with
  each 2x2 diagonal block standardized to equal diagonal entries (the form
  the worked example of equation (Gauss4Radau3_example) uses).
* ``real_eigenbasis`` is the real eigenbasis A0^{-1} = T Lambda T^{-1}
  (Section 3.1 with phi = beta): one column per real eigenvalue and the pair
  (Re v, Im v) per conjugate pair, normalized so that the transformed blocks
  and their d weights are unique (see the function).
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np
import scipy.linalg as sla

_DPS = 60


def _shifted_legendre(n: int) -> list:
    """Coefficients (ascending powers of x) of P_n(2x - 1), exact integers.

    P_n(2x-1) = sum_k (-1)^(n+k) C(n,k) C(n+k,k) x^k (Rodrigues' formula on
    [0, 1]).
    """
    return [mp.mpf((-1) ** (n + k) * math.comb(n, k) * math.comb(n + k, k))
            for k in range(n + 1)]


def _poly_roots_real(coeffs_ascending: list) -> list:
    """All roots of a polynomial known to have only real roots, ascending."""
    with mp.workdps(_DPS):
        roots = mp.polyroots(list(reversed(coeffs_ascending)), maxsteps=400,
                             extraprec=4 * _DPS)
        out = sorted(mp.re(r) for r in roots)
    return out


def nodes(family: str, s: int) -> list:
    """Collocation nodes c_1 < ... < c_s as mpmath numbers (Section 2.2)."""
    if s < 1:
        raise ValueError("s must be >= 1")
    with mp.workdps(_DPS):
        ps = _shifted_legendre(s)
        if family == "gauss":
            poly = ps
        elif family == "radau":
            if s == 1:
                return [mp.mpf(1)]
            pm = _shifted_legendre(s - 1) + [mp.mpf(0)]
            poly = [a - b for a, b in zip(ps, pm)]
        elif family == "lobatto":
            if s < 2:
                raise ValueError("Lobatto IIIC needs s >= 2")
            if s == 2:
                return [mp.mpf(0), mp.mpf(1)]
            q = _shifted_legendre(s - 1)
            dq = [k * q[k] for k in range(1, len(q))]       # d/dx P_{s-1}(2x-1)
            return [mp.mpf(0)] + _poly_roots_real(dq) + [mp.mpf(1)]
        else:
            raise ValueError(f"unknown family {family!r}")
        roots = _poly_roots_real(poly)
        if family == "radau":
            roots[-1] = mp.mpf(1)   # exact root of P_s - P_{s-1} at x = 1
        return roots


def _lagrange_coeffs(c: list, j: int) -> list:
    """Ascending coefficients of the Lagrange basis polynomial l_j on nodes c."""
    poly = [mp.mpf(1)]
    denom = mp.mpf(1)
    for m, cm in enumerate(c):
        if m == j:
            continue
        # multiply by (x - c_m)
        new = [mp.mpf(0)] * (len(poly) + 1)
        for p, a in enumerate(poly):
            new[p] -= a * cm
            new[p + 1] += a
        poly = new
        denom *= (c[j] - cm)
    return [a / denom for a in poly]


def _integral_0_to(poly: list, x) -> mp.mpf:
    return sum(a * x ** (p + 1) / (p + 1) for p, a in enumerate(poly))


def tableau_mp(family: str, s: int):
    """(A, b, c) as nested lists of mpmath numbers at 60 digits."""
    with mp.workdps(_DPS):
        c = nodes(family, s)
        basis = [_lagrange_coeffs(c, j) for j in range(s)]
        b = [_integral_0_to(basis[j], mp.mpf(1)) for j in range(s)]
        if family == "lobatto":
            # a_i1 = b_1; the remaining s-1 entries of row i from C(s-1):
            # sum_{j>=2} a_ij c_j^{k-1} = c_i^k / k - b_1 [k = 1], k = 1..s-1
            V = mp.matrix(s - 1, s - 1)
            for k in range(1, s):
                for j in range(1, s):
                    V[k - 1, j - 1] = c[j] ** (k - 1)
            A = []
            for i in range(s):
                rhs = mp.matrix([c[i] ** k / k - (b[0] if k == 1 else 0) for k in range(1, s)])
                x = mp.lu_solve(V, rhs)
                A.append([b[0]] + [x[j] for j in range(s - 1)])
        else:
            A = [[_integral_0_to(basis[j], c[i]) for j in range(s)] for i in range(s)]
    return A, b, c


def _sdirk_mp(s: int):
    """SDIRK tableaux of the published methods listed in the module notes."""
    with mp.workdps(_DPS):
        F = mp.mpf
        if s == 1:
            A = [[F(1)]]
        elif s == 2:
            g = 1 - 1 / mp.sqrt(2)
            A = [[g, F(0)], [1 - g, g]]
        elif s == 3:
            g = mp.findroot(lambda x: x ** 3 - 3 * x ** 2 + F(3) / 2 * x - F(1) / 6, F("0.4358665"))
            t2 = (1 + g) / 2
            b1 = -(6 * g ** 2 - 16 * g + 1) / 4
            b2 = (6 * g ** 2 - 20 * g + 5) / 4
            A = [[g, F(0), F(0)], [t2 - g, g, F(0)], [b1, b2, g]]
        elif s == 5:
            q = mp.mpf
            A = [[q(1) / 4, 0, 0, 0, 0],
                 [q(1) / 2, q(1) / 4, 0, 0, 0],
                 [q(17) / 50, -q(1) / 25, q(1) / 4, 0, 0],
                 [q(371) / 1360, -q(137) / 2720, q(15) / 544, q(1) / 4, 0],
                 [q(25) / 24, -q(49) / 48, q(125) / 16, -q(85) / 12, q(1) / 4]]
            A = [[mp.mpf(v) for v in row] for row in A]
        else:
            raise ValueError("SDIRK methods are provided for s in {1, 2, 3, 5}")
        b = list(A[-1])
        c = [sum(row) for row in A]
    return A, b, c


def tableau(family: str, s: int):
    """Butcher tableau (A0, b0, c0) of the s-stage Gauss, Radau IIA or
    Lobatto IIIC method, rounded to float64 from the extended-precision
    construction."""
    A, b, c = _sdirk_mp(s) if family == "sdirk" else tableau_mp(family, s)
    return (np.array([[float(v) for v in row] for row in A]),
            np.array([float(v) for v in b]),
            np.array([float(v) for v in c]))


def stability_function(A: np.ndarray, b: np.ndarray, z: complex) -> complex:
    """R(z) = 1 + z b^T (I - z A)^{-1} 1 (value of one step on u' = lambda u)."""
    s = len(b)
    one = np.ones(s, dtype=complex)
    return 1.0 + z * (b.astype(complex) @ np.linalg.solve(np.eye(s) - z * A, one))


def pade_exp(k: int, j: int, z: complex) -> complex:
    """(k, j) Pade approximant of exp(z): numerator degree k, denominator j
    (closed form of the Pade table of the exponential)."""
    num = sum(math.factorial(k + j - i) * math.factorial(k)
              / (math.factorial(k + j) * math.factorial(i) * math.factorial(k - i)) * z ** i
              for i in range(k + 1))
    den = sum(math.factorial(k + j - i) * math.factorial(j)
              / (math.factorial(k + j) * math.factorial(i) * math.factorial(j - i)) * (-z) ** i
              for i in range(j + 1))
    return num / den


def inverse_eigs(A: np.ndarray):
    """Eigen-structure of A0^{-1} (Section 3): list of (eta, beta) with one
    entry per real eigenvalue (beta = 0) and one per conjugate pair (beta > 0),
    sorted as the paper's Table 1 columns: real first, then pairs by
    decreasing beta."""
    lam = np.linalg.eigvals(np.linalg.inv(A))
    real = sorted(float(l.real) for l in lam if abs(l.imag) < 1e-12)
    pairs = sorted(((float(l.real), float(l.imag)) for l in lam if l.imag > 1e-12),
                   key=lambda p: -p[1])
    return [(e, 0.0) for e in real] + pairs


def gamma_star(eta: float, beta: float) -> float:
    """Equation (gamma*): gamma_* = eta + beta^2 / eta."""
    return eta + beta * beta / eta


def kappa_bound(eta: float, beta: float) -> float:
    """Equation (kappa_gamma*_L1=L2): kappa(P_gamma*) <= 1 + beta^2/(2 eta^2)."""
    return 1.0 + beta * beta / (2.0 * eta * eta)


def d_weights(T: np.ndarray) -> np.ndarray:
    """d[k, l, i] = (T^{-1})_{k i} T_{i l}: the weight of stage operator L_i in
    block (k, l) of (T^{-1} (x) I) diag(L_i) (T (x) I), equation (Q0approx)
    (there with T = Q0, T^{-1} = Q0^T)."""
    Ti = np.linalg.inv(T)
    return np.einsum("ki,il->kli", Ti, T)


def real_schur_standard(Ainv: np.ndarray):
    """Real Schur form Ainv = Q0 R0 Q0^T with every 2x2 diagonal block rotated
    to equal diagonal entries (LAPACK's standardized form)."""
    R, Q = sla.schur(Ainv, output="real")
    s = R.shape[0]
    i = 0
    while i < s:
        if i + 1 < s and abs(R[i + 1, i]) > 1e-14:
            a, b_, c_, d = R[i, i], R[i, i + 1], R[i + 1, i], R[i + 1, i + 1]
            # rotation G making the block's diagonal equal: tan(2t) = (d-a)/(b+c)
            t = 0.5 * math.atan2(d - a, b_ + c_)
            G = np.eye(s)
            G[i, i], G[i, i + 1], G[i + 1, i], G[i + 1, i + 1] = (
                math.cos(t), -math.sin(t), math.sin(t), math.cos(t))
            R = G.T @ R @ G
            Q = Q @ G
            if abs(R[i, i + 1]) > abs(R[i + 1, i]):
                # a quarter turn swaps the off-diagonal magnitudes; keep the
                # smaller one above the diagonal (phi in [[eta, phi],
                # [-beta^2/phi, eta]] with |phi| <= beta)
                G = np.eye(s)
                G[i, i], G[i, i + 1], G[i + 1, i], G[i + 1, i + 1] = 0.0, -1.0, 1.0, 0.0
                R = G.T @ R @ G
                Q = Q @ G
            i += 2
        else:
            i += 1
    return Q, R


def real_eigenbasis(A: np.ndarray):
    """Real eigenbasis of A0^{-1}: A0^{-1} = T Lambda T^{-1}, Lambda block
    diagonal with eta for a real eigenvalue and [[eta, beta], [-beta, eta]]
    for a pair eta +- i beta (beta > 0): if A0^{-1} v = (eta + i beta) v with
    v = a + i b, then A0^{-1} [a b] = [a b] [[eta, beta], [-beta, eta]].
    Blocks: real eigenvalues first (ascending), then pairs by decreasing beta.
    Normalization: unit vectors; for a pair the phase of v that makes a
    orthogonal to b with |a| >= |b| (it maximizes |a|^2 - |b|^2); the entry of
    largest magnitude of a (of v, for a real eigenvalue) positive.  Returns
    (T, blocks) with blocks a list of (first_row, width, eta, beta)."""
    s = A.shape[0]
    lam, V = np.linalg.eig(np.linalg.inv(A))
    reals = sorted((float(lam[k].real), k) for k in range(s) if abs(lam[k].imag) < 1e-12)
    ups = sorted(((float(lam[k].imag), k) for k in range(s) if lam[k].imag > 1e-12), reverse=True)
    T = np.zeros((s, s))
    blocks = []
    row = 0
    for eta, k in reals:
        v = np.real(V[:, k])
        v = v / np.linalg.norm(v)
        if v[np.argmax(np.abs(v))] < 0:
            v = -v
        T[:, row] = v
        blocks.append((row, 1, eta, 0.0))
        row += 1
    for beta, k in ups:
        v = V[:, k] / np.linalg.norm(V[:, k])
        a, b = v.real, v.imag
        th = 0.5 * math.atan2(-2.0 * float(a @ b), float(a @ a - b @ b))
        v = v * np.exp(1j * th)
        if v.real[np.argmax(np.abs(v.real))] < 0:
            v = -v
        T[:, row], T[:, row + 1] = v.real, v.imag
        blocks.append((row, 2, float(lam[k].real), beta))
        row += 2
    return T, blocks
