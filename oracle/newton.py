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

The initial guess is the best (smallest residual) of K = 0, the explicit
k_i = M^+ N(u_n, t_n) on differential rows and 0 on algebraic rows, and on a
continued step the previous stages extrapolated (the paper leaves it open).

``block_operator`` writes out the Krylov operator of one eigen-block under
each Newton-like truncation of Section 3.2 (the definition those iterations
are built from; used to pin the GPU's block operators).
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


def extrapolated_stages(c, K_prev, dt_prev, dt):
    """Previous step's stage vectors carried along their interpolating
    polynomial: k_j^prev sits at the previous step's node c_j (in units of
    dt_prev), the new stage i at 1 + c_i dt / dt_prev, so
    k_i = sum_j l_j(1 + c_i dt/dt_prev) k_j^prev with l_j the Lagrange basis
    on the nodes c.  For collocation methods the k_j are the derivative of the
    collocation polynomial at the nodes, and this is its continuation."""
    c = np.asarray(c, dtype=np.float64)
    s = len(c)
    W = np.ones((s, s))
    for i in range(s):
        x = 1.0 + c[i] * dt / dt_prev
        for j in range(s):
            for m in range(s):
                if m != j:
                    W[i, j] *= (x - c[m]) / (c[j] - c[m])
    return W @ K_prev


def initial_stages(problem, A, c, u_n, t_n, dt, prev=None):
    """Starting stage vectors K^0.  Algorithm 1 leaves them open.  Candidates,
    in this order: K = 0 (every stage value U_i at u_n, the usual stiff
    start); the explicit k_i = M^{-1} N(u_n, t_n) on differential rows, 0 on
    algebraic rows (good for smooth, non-stiff motion); and, when the step
    continues a previous one (``prev`` = (K_prev, dt_prev)), the previous
    stage vectors extrapolated (``extrapolated_stages``).  The one with the
    smallest stage residual of equation (stages) is taken, the earlier one on
    ties.  Returns (K0, index of the candidate)."""
    s = len(c)
    cands = [np.zeros((s, problem.size)), np.stack([problem.rhs(u_n, t_n) * problem.mass] * s)]
    if prev is not None:
        cands.append(extrapolated_stages(c, prev[0], prev[1], dt))
    res = [np.linalg.norm(stage_residual(problem, A, c, u_n, t_n, dt, K)) for K in cands]
    best = 0
    for k in range(1, len(cands)):
        if res[k] < res[best]:
            best = k
    return cands[best], best


def irk_stages(problem, A, c, u_n, t_n, dt, max_iter=60, K0=None, prev=None):
    """Stage vectors K (shape (s, N)) solving equation (stages) to roundoff.
    ``prev`` = (K_prev, dt_prev) of the step this one continues, if any."""
    s = len(c)
    K = initial_stages(problem, A, c, u_n, t_n, dt, prev)[0] if K0 is None else K0.copy()
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


def irk_step(problem, A, b, c, u_n, t_n, dt, max_iter=60, prev=None):
    """u_{n+1} = u_n + dt sum_i b_i k_i with K from ``irk_stages``."""
    K, info = irk_stages(problem, A, c, u_n, t_n, dt, max_iter=max_iter, prev=prev)
    return u_n + dt * (b @ K), K, info


def lumped_stage(dr):
    """Stage Newton-like (1) lumps a row with diagonal weights ``dr`` to: the
    largest |d_rr,k|, and among weights within a relative 1e-12 of the
    largest the lowest index k.  (The real eigenvalue's row of Gauss with odd
    s and of 3-stage Lobatto IIIC has its two largest weights equal,
    d_rr,k = d_rr,s-1-k; a plain argmax would decide those by rounding.)"""
    w = np.abs(np.asarray(dr, dtype=np.float64))
    big = float(w.max())
    for k in range(len(w)):
        if w[k] >= big * (1.0 - 1e-12):
            return k
    return int(np.argmax(w))


def block_operator(problem, A, c, u_n, t_n, dt, K, T, block, variant):
    """Krylov operator D_b of one eigen-block (equation (diag_blocks)) as a
    sparse matrix on the block's transformed components.  With the stage
    Jacobians L_k = L(U_k) and d weights d_{r,q,k} = (T^{-1})_{r k} T_{k q}
    (equation (Q0approx) for the similarity T), row a of the block (transformed
    row r_a = first + a) is
      Lambda_{ab} M - dt sum_k W_{a b k} L_k
    with the truncations of Section 3.2 written in the eigenbasis:
      0: W_{aak} = [k = s-1] (every row linearized at the last stage),
      1: W_{aak} = [k = lumped_stage(d_{r_a r_a})] (lumped to the largest
         weight, the lowest stage index among ties),
      2: W_{aak} = d_{r_a r_a k} (the diagonal weights, not lumped),
      3: W_{abk} = d_{r_a r_b k} for both rows of the block (the truncation to
         the block sparsity of R0; in the eigenbasis R0 is block diagonal).
    ``block`` = (first_row, width, eta, beta); ODE operators only (M = I or
    the problem's mass, no low-rank Jacobian part)."""
    first, width, eta, beta = block
    s = len(c)
    U = stage_values(A, u_n, dt, K)
    L = []
    for k in range(s):
        S, Ul, _ = problem.jac(U[k], t_n + c[k] * dt)
        assert Ul is None
        L.append(S)
    Ti = np.linalg.inv(T)
    W = np.zeros((width, width, s))
    for a in range(width):
        r = first + a
        dr = Ti[r, :] * T[:, r]
        if variant == 0:
            W[a, a, s - 1] = 1.0
        elif variant == 1:
            W[a, a, lumped_stage(dr)] = 1.0
        elif variant == 2:
            W[a, a, :] = dr
        else:
            for b2 in range(width):
                W[a, b2, :] = Ti[r, :] * T[:, first + b2]
    Lam = np.array([[eta]]) if width == 1 else np.array([[eta, beta], [-beta, eta]])
    M = sp.diags(problem.mass)
    blocks = [[Lam[a, b2] * M - dt * sum(W[a, b2, k] * L[k] for k in range(s)) for b2 in range(width)]
              for a in range(width)]
    return sp.bmat(blocks, format="csr")
