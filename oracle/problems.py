"""Semi-discrete operators N_h(u, t) and their exact Jacobians (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Each problem is written in the form M u' = N(u, t) of equation (problem)
(Section 1.1) with a diagonal mass matrix M (1 on differential rows, 0 on
algebraic rows, Section 6 equation (dae)).  A problem exposes

* ``mass``            -- the diagonal of M (float64 vector),
* ``rhs(u, t)``       -- N(u, t),
* ``jac(u, t)``       -- the exact Jacobian dN/du as ``(S, U, V)`` with
  dN/du = S + U V^T, S a SciPy sparse matrix and U, V dense low-rank factors
  (``None`` when there is no low-rank part).

The discretizations are the plain finite-difference definitions on a
periodic grid of spacing h = L / n with nodes x_i = i h:

* ``Burgers1D``: N(u)_i = -(u_{i+1}^2 - u_{i-1}^2)/(4h)
  + nu (u_{i+1} - 2u_i + u_{i-1}) / h^2.
* ``NonlinearDiffusion2D``: N(u) = h^{-2} sum_faces kappa_f (u_nb - u_c) + f,
  kappa(u) = 1 + u^2, kappa_f = (kappa(u_c) + kappa(u_nb)) / 2; forcing f from
  the manufactured solution u* = sin(2 pi x) sin(2 pi y) cos t, either of the
  PDE (``forcing="continuous"``) or of the semi-discrete system
  (``forcing="discrete"``, f = du*/dt - N_h(u*)), or none.
* ``VorticityStreamfunction2D``: state (omega, psi);
  omega rows: J_A(psi, omega) + nu Lap_h omega with J_A Arakawa's 9-point
  Jacobian; psi rows (algebraic, index 1): Lap_h psi + omega - mean(omega)
  - mean(psi), whose zero set is -Lap_h psi = omega - mean(omega) together
  with the gauge mean(psi) = 0 (the rows of Lap_h psi + omega - mean(omega)
  sum to zero, so summing the rows forces mean(psi) = 0).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

TWO_PI = 2.0 * np.pi


def _periodic_shift_matrix(n: int, shift: int) -> sp.csr_matrix:
    """P with (P x)_i = x_{(i + shift) mod n}."""
    rows = np.arange(n)
    cols = (rows + shift) % n
    return sp.csr_matrix((np.ones(n), (rows, cols)), shape=(n, n))


# --------------------------------------------------------------------------
# 1-D viscous Burgers
# --------------------------------------------------------------------------
class Burgers1D:
    """u_t + (u^2/2)_x = nu u_xx, periodic on [0, length)."""

    def __init__(self, n: int, nu: float, length: float = 1.0):
        self.n = n
        self.nu = nu
        self.h = length / n
        self.size = n
        self.mass = np.ones(n)
        self._Ep = _periodic_shift_matrix(n, +1)
        self._Em = _periodic_shift_matrix(n, -1)

    def rhs(self, u, t=0.0):
        h, nu = self.h, self.nu
        up, um = np.roll(u, -1), np.roll(u, 1)
        return -(up * up - um * um) / (4.0 * h) + nu * (up - 2.0 * u + um) / (h * h)

    def jac(self, u, t=0.0):
        """L(U) x = -(U_{i+1} x_{i+1} - U_{i-1} x_{i-1})/(2h) + nu D2 x."""
        h, nu, n = self.h, self.nu, self.n
        adv = -(self._Ep @ sp.diags(u) - self._Em @ sp.diags(u)) / (2.0 * h)
        dif = nu * (self._Ep - 2.0 * sp.identity(n) + self._Em) / (h * h)
        return (adv + dif).tocsr(), None, None


# --------------------------------------------------------------------------
# 2-D nonlinear diffusion u_t = div((1 + u^2) grad u) + f
# --------------------------------------------------------------------------
def mms_solution(x, y, t):
    """u*(x, y, t) = sin(2 pi x) sin(2 pi y) cos t."""
    return np.sin(TWO_PI * x) * np.sin(TWO_PI * y) * np.cos(t)


def mms_continuous_forcing(x, y, t):
    """f = u*_t - div((1 + u*^2) grad u*) for u* = S cos t, S = sin2pix sin2piy.

    div((1+u^2) grad u) = (1 + u^2) Lap u + 2 u |grad u|^2 with
    Lap u* = -8 pi^2 u*, |grad u*|^2 = 4 pi^2 G cos^2 t,
    G = cos^2(2pix) sin^2(2piy) + sin^2(2pix) cos^2(2piy).
    """
    sx, cx = np.sin(TWO_PI * x), np.cos(TWO_PI * x)
    sy, cy = np.sin(TWO_PI * y), np.cos(TWO_PI * y)
    S = sx * sy
    G = cx * cx * sy * sy + sx * sx * cy * cy
    ct, st = np.cos(t), np.sin(t)
    u = S * ct
    lap = -8.0 * np.pi ** 2 * u
    grad2 = 4.0 * np.pi ** 2 * G * ct * ct
    div_term = (1.0 + u * u) * lap + 2.0 * u * grad2
    return -S * st - div_term


class NonlinearDiffusion2D:
    """Periodic [0, length)^2, n x n nodes, arrays indexed [j (y), i (x)]."""

    def __init__(self, n: int, forcing: str = "continuous", length: float = 1.0,
                 kappa_quadratic: bool = True):
        if forcing not in ("continuous", "discrete", "none"):
            raise ValueError(forcing)
        self.n = n
        self.h = length / n
        self.size = n * n
        self.mass = np.ones(n * n)
        self.forcing = forcing
        # kappa_quadratic=False freezes kappa = 1: the linear constant-
        # coefficient variant used by the Fourier-symbol test
        self.kq = 1.0 if kappa_quadratic else 0.0
        g = np.arange(n) * self.h
        self.X, self.Y = np.meshgrid(g, g)          # X[j, i] = x_i, Y[j, i] = y_j
        self._shifts = []
        for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            self._shifts.append(self._shift_matrix(dj, di))

    def _shift_matrix(self, dj: int, di: int) -> sp.csr_matrix:
        n = self.n
        j, i = np.divmod(np.arange(n * n), n)
        cols = ((j + dj) % n) * n + (i + di) % n
        return sp.csr_matrix((np.ones(n * n), (np.arange(n * n), cols)), shape=(n * n, n * n))

    def kappa(self, u):
        return 1.0 + self.kq * u * u

    def flux_operator(self, u2d):
        """h^{-2} sum over the 4 faces of kappa_f (u_nb - u_c), on a 2-D array."""
        h2 = self.h * self.h
        kc = self.kappa(u2d)
        out = np.zeros_like(u2d)
        for axis, step in ((1, -1), (1, 1), (0, -1), (0, 1)):
            unb = np.roll(u2d, step, axis=axis)
            kf = 0.5 * (kc + self.kappa(unb))
            out += kf * (unb - u2d)
        return out / h2

    def forcing_term(self, t):
        if self.forcing == "none":
            return np.zeros((self.n, self.n))
        if self.forcing == "continuous":
            return mms_continuous_forcing(self.X, self.Y, t)
        # semi-discrete manufactured solution: f_h = du*/dt - N_h(u*)
        S = np.sin(TWO_PI * self.X) * np.sin(TWO_PI * self.Y)
        return -S * np.sin(t) - self.flux_operator(S * np.cos(t))

    def rhs(self, u, t=0.0):
        u2 = u.reshape(self.n, self.n)
        return (self.flux_operator(u2) + self.forcing_term(t)).ravel()

    def jac(self, u, t=0.0):
        """L(U) x = h^{-2} sum_f [kappa_f (x_nb - x_c)
                                 + (kappa'(U_c) x_c + kappa'(U_nb) x_nb)(U_nb - U_c)/2]."""
        h2 = self.h * self.h
        U = u.ravel()
        kc = self.kappa(U)
        dk = 2.0 * self.kq * U                      # kappa'(U)
        L = sp.csr_matrix((self.size, self.size))
        for P in self._shifts:
            Unb = P @ U
            kf = 0.5 * (kc + self.kappa(Unb))
            dU = Unb - U
            # coefficient of x_c and of x_nb in this face's term
            diag_c = -kf + 0.5 * dk * dU
            coef_nb = kf + 0.5 * (P @ dk) * dU
            L = L + sp.diags(diag_c) + sp.diags(coef_nb) @ P
        return (L / h2).tocsr(), None, None


# --------------------------------------------------------------------------
# 2-D vorticity-streamfunction (index-1 DAE)
# --------------------------------------------------------------------------
def arakawa(psi, om, h):
    """Arakawa's energy- and enstrophy-conserving Jacobian J(psi, omega)
    ~ psi_x omega_y - psi_y omega_x, as the mean of the three second-order
    forms J++, J+x, Jx+; arrays indexed [j (y), i (x)]."""
    def s(a, dj, di):
        # value at (j + dj, i + di), periodic
        return np.roll(np.roll(a, -dj, axis=0), -di, axis=1)
    p, w = psi, om
    jpp = ((s(p, 0, 1) - s(p, 0, -1)) * (s(w, 1, 0) - s(w, -1, 0))
           - (s(p, 1, 0) - s(p, -1, 0)) * (s(w, 0, 1) - s(w, 0, -1)))
    jpx = (s(p, 0, 1) * (s(w, 1, 1) - s(w, -1, 1))
           - s(p, 0, -1) * (s(w, 1, -1) - s(w, -1, -1))
           - s(p, 1, 0) * (s(w, 1, 1) - s(w, 1, -1))
           + s(p, -1, 0) * (s(w, -1, 1) - s(w, -1, -1)))
    jxp = (s(w, 1, 0) * (s(p, 1, 1) - s(p, 1, -1))
           - s(w, -1, 0) * (s(p, -1, 1) - s(p, -1, -1))
           - s(w, 0, 1) * (s(p, 1, 1) - s(p, -1, 1))
           + s(w, 0, -1) * (s(p, 1, -1) - s(p, -1, -1)))
    return (jpp + jpx + jxp) / (12.0 * h * h)


def laplacian(a, h):
    """5-point periodic Laplacian."""
    return (np.roll(a, 1, 0) + np.roll(a, -1, 0) + np.roll(a, 1, 1)
            + np.roll(a, -1, 1) - 4.0 * a) / (h * h)


class VorticityStreamfunction2D:
    """State u = (omega, psi) stacked, each n x n, periodic [0, length)^2."""

    def __init__(self, n: int, nu: float, length: float = 1.0):
        self.n = n
        self.nu = nu
        self.h = length / n
        self.nn = n * n
        self.size = 2 * n * n
        self.mass = np.concatenate([np.ones(n * n), np.zeros(n * n)])

    def split(self, u):
        n = self.n
        return u[: self.nn].reshape(n, n), u[self.nn:].reshape(n, n)

    def rhs(self, u, t=0.0):
        om, psi = self.split(u)
        h = self.h
        dom = arakawa(psi, om, h) + self.nu * laplacian(om, h)
        con = laplacian(psi, h) + om - om.mean() - psi.mean()
        return np.concatenate([dom.ravel(), con.ravel()])

    def _lin_matrix(self, fn):
        """Sparse matrix of the linear map x -> fn(x) on n x n arrays, built
        column by column from unit vectors placed on an m x m colouring with
        m the smallest divisor of n that is at least 3 (the stencils reach
        one cell, so probed points of one colour are at least three cells
        apart also across the periodic wrap): m^2 applications recover every
        column.  Without such a divisor below n, column by column."""
        n, nn = self.n, self.nn
        m = next((d for d in range(3, n) if n % d == 0), n)
        if m == n:
            return self._lin_matrix_dense(fn)
        rows, cols, vals = [], [], []
        jj, ii = np.divmod(np.arange(nn), n)
        for cj in range(m):
            for ci in range(m):
                mask = ((jj % m) == cj) & ((ii % m) == ci)
                e = mask.astype(float).reshape(n, n)
                col = fn(e).ravel()
                nz = np.nonzero(col)[0]
                # each nonzero row r comes from the unique probed point within
                # one cell of it: offset d in {-1, 0, 1} with r + d = colour (mod m)
                rj, ri = np.divmod(nz, n)
                dj = (cj - rj) % m
                di = (ci - ri) % m
                dj[dj == m - 1] = -1
                di[di == m - 1] = -1
                assert np.all(np.abs(dj) <= 1) and np.all(np.abs(di) <= 1)
                src = ((rj + dj) % n) * n + (ri + di) % n
                rows.append(nz)
                cols.append(src)
                vals.append(col[nz])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(nn, nn))

    def _lin_matrix_dense(self, fn):
        n, nn = self.n, self.nn
        M = np.zeros((nn, nn))
        for c in range(nn):
            e = np.zeros(nn)
            e[c] = 1.0
            M[:, c] = fn(e.reshape(n, n)).ravel()
        return sp.csr_matrix(M)

    def jac(self, u, t=0.0):
        """dN/du = S + U V^T: S holds J_A(psi, .), J_A(., omega), nu Lap, Lap
        and the identity; the rank-2 part holds the two mean terms."""
        om, psi = self.split(u)
        h, nn = self.h, self.nn
        A_ww = self._lin_matrix(lambda x: arakawa(psi, x, h) + self.nu * laplacian(x, h))
        A_wp = self._lin_matrix(lambda x: arakawa(x, om, h))
        A_pp = self._lin_matrix(lambda x: laplacian(x, h))
        S = sp.bmat([[A_ww, A_wp], [sp.identity(nn), A_pp]]).tocsr()
        ones_rows = np.concatenate([np.zeros(nn), np.ones(nn)])
        Ulow = np.stack([ones_rows, ones_rows], axis=1)
        Vlow = np.stack([np.concatenate([np.full(nn, -1.0 / nn), np.zeros(nn)]),
                         np.concatenate([np.zeros(nn), np.full(nn, -1.0 / nn)])], axis=1)
        return S, Ulow, Vlow

    def gauge_pins(self):
        """(row, column) entries that make S nonsingular: S alone is singular
        along the constant-psi direction, which the rank-1 mean(psi) term
        removes.  The Newton solver adds these entries to S and subtracts them
        again in the low-rank part, so the Jacobian it solves is unchanged."""
        return [(self.nn, self.nn)]
