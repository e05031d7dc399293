"""One implicit Runge-Kutta step by full Newton with a direct sparse solve.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

This is the plain definition the paper's method converges to (Section 3.2:
its Newton-like iterations are preconditioned nonlinear Richardson iterations
whose fixed point is the solution of the stage equations):

* stage equations, equation (stages) / (dae_stage):
  R_i(K) = M k_i - N(u_n + dt sum_j a_ij k_j, t_n + c_i dt) = 0;
* Newton matrix, equation (k0): block (i, j) = delta_ij M - dt a_ij L(U_i),
  with L(U_i) the exact Jacobian of N at the i-th stage value;
* each Newton correction solved with SciPy's SuperLU (ordering
  MMD_AT_PLUS_A) and, where the Jacobian carries a dense low-rank part
  (the mean terms of the DAE constraint), the Sherman-Morrison-Woodbury
  identity around the sparse LU;
* iteration until the correction reaches rounding level (||dK|| <= 4 eps ||K||)
  or stops decreasing, so the result is the stage solution to roundoff;
* update, equation (update): u_{n+1} = u_n + dt sum_i b_i k_i.

The initial guess is the same for every stage, k_i = M^+ N(u_n, t_n) on the
differential rows and 0 on algebraic rows (the paper leaves it open).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

EPS = np.finfo(np.float64).eps


@dataclasses.dataclass
class StepInfo:
    newton_its: int
    corrections: list
    residual_norms: list


def stage_values(A, u_n, dt, K):
    """U_i = u_n + dt sum_j a_ij k_j for every stage i (K has shape (s, N))."""
    return u_n[None, :] + dt * (A @ K)


def stage_residual(problem, A, c, u_n, t_n, dt, K):
    """R_i = M k_i - N(U_i, t_n + c_i dt), equation (stages)."""
    U = stage_values(A, u_n, dt, K)
    return np.stack([problem.mass * K[i] - problem.rhs(U[i], t_n + c[i] * dt)
                     for i in range(len(c))])


def _newton_matrix(problem, A, c, u_n, t_n, dt, K):
    """Sparse part S and low-rank factors (Ub, Vb) of the Newton matrix,
    J = S + Ub Vb^T, block (i, j) = delta_ij M - dt a_ij L(U_i)."""
    s = len(c)
    N = problem.size
    U = stage_values(A, u_n, dt, K)
    blocks = [[None] * s for _ in range(s)]
    Ucols, Vcols = [], []
    Mdiag = sp.diags(problem.mass)
    pins = problem.gauge_pins() if hasattr(problem, "gauge_pins") else []
    for i in range(s):
        Si, Ui, Vi = problem.jac(U[i], t_n + c[i] * dt)
        for j in range(s):
            blk = -dt * A[i, j] * Si
            if i == j:
                blk = blk + Mdiag
            blocks[i][j] = blk
        if Ui is not None:
            r = Ui.shape[1]
            for q in range(r):
                ucol = np.zeros(s * N)
                ucol[i * N:(i + 1) * N] = Ui[:, q]
                vcol = np.zeros(s * N)
                for j in range(s):
                    vcol[j * N:(j + 1) * N] = -dt * A[i, j] * Vi[:, q]
                Ucols.append(ucol)
                Vcols.append(vcol)
    S = sp.bmat(blocks, format="lil")
    for i in range(s):
        for (r, col) in pins:
            # add a unit entry to S and remove it again through the low-rank part
            S[i * N + r, i * N + col] += 1.0
            ucol = np.zeros(s * N)
            ucol[i * N + r] = -1.0
            vcol = np.zeros(s * N)
            vcol[i * N + col] = 1.0
            Ucols.append(ucol)
            Vcols.append(vcol)
    Ub = np.stack(Ucols, axis=1) if Ucols else None
    Vb = np.stack(Vcols, axis=1) if Vcols else None
    return S.tocsc(), Ub, Vb


def solve_sparse_lowrank(S, Ub, Vb, rhs):
    """x = (S + Ub Vb^T)^{-1} rhs by SuperLU on S and the Woodbury identity."""
    lu = spla.splu(S, permc_spec="MMD_AT_PLUS_A")
    x = lu.solve(rhs)
    if Ub is None:
        return x
    SU = lu.solve(Ub)
    small = np.eye(Ub.shape[1]) + Vb.T @ SU
    return x - SU @ np.linalg.solve(small, Vb.T @ x)


def initial_stages(problem, A, c, u_n, t_n, dt):
    """Starting stage vectors K^0.  Algorithm 1 leaves them open; of the two
    natural candidates -- K = 0 (every stage value U_i at u_n, the usual stiff
    start) and the explicit k_i = M^{-1} N(u_n, t_n) on differential rows, 0
    on algebraic rows (good for smooth, non-stiff motion) -- take the one with
    the smaller stage residual of equation (stages), zero on ties."""
    s = len(c)
    zero = np.zeros((s, problem.size))
    explicit = np.stack([problem.rhs(u_n, t_n) * problem.mass] * s)
    r_zero = np.linalg.norm(stage_residual(problem, A, c, u_n, t_n, dt, zero))
    r_expl = np.linalg.norm(stage_residual(problem, A, c, u_n, t_n, dt, explicit))
    return explicit if r_expl < r_zero else zero


def irk_stages(problem, A, c, u_n, t_n, dt, max_iter=60, K0=None):
    """Stage vectors K (shape (s, N)) solving equation (stages) to roundoff."""
    s = len(c)
    K = initial_stages(problem, A, c, u_n, t_n, dt) if K0 is None else K0.copy()
    corr, res = [], []
    prev = np.inf
    for it in range(1, max_iter + 1):
        R = stage_residual(problem, A, c, u_n, t_n, dt, K)
        res.append(float(np.linalg.norm(R)))
        S, Ub, Vb = _newton_matrix(problem, A, c, u_n, t_n, dt, K)
        dK = solve_sparse_lowrank(S, Ub, Vb, -R.ravel()).reshape(K.shape)
        K = K + dK
        nd = float(np.linalg.norm(dK))
        corr.append(nd)
        if nd <= 4.0 * EPS * float(np.linalg.norm(K)) or (it >= 3 and nd >= prev):
            return K, StepInfo(it, corr, res)
        prev = nd
    raise RuntimeError(f"oracle Newton did not converge in {max_iter} iterations: {corr}")


def irk_step(problem, A, b, c, u_n, t_n, dt, max_iter=60):
    """u_{n+1} = u_n + dt sum_i b_i k_i with K from ``irk_stages``."""
    K, info = irk_stages(problem, A, c, u_n, t_n, dt, max_iter=max_iter)
    return u_n + dt * (b @ K), K, info
