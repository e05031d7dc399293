"""Pins of the oracle's spatial operators: exact Jacobians against finite
differences of N, truncation error against the PDE (second order), the
Arakawa Jacobian's conservation laws, and the manufactured forcing against a
symbolic derivation."""
import numpy as np
import pytest
import sympy

from oracle import problems as pb
from paper_2101_01776_amd import inputs


def _fd_check(problem, u, t=0.3, seed=0, eps=1e-6):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(problem.size)
    S, U, V = problem.jac(u, t)
    Jx = S @ x + (U @ (V.T @ x) if U is not None else 0.0)
    fd = (problem.rhs(u + eps * x, t) - problem.rhs(u - eps * x, t)) / (2 * eps)
    return np.linalg.norm(Jx - fd) / np.linalg.norm(fd)


def test_burgers_jacobian_fd():
    p = pb.Burgers1D(64, 0.01)
    assert _fd_check(p, inputs.burgers_u0(64, 3)) < 1e-8


@pytest.mark.parametrize("forcing", ["continuous", "discrete", "none"])
def test_nldiff_jacobian_fd(forcing):
    p = pb.NonlinearDiffusion2D(12, forcing=forcing)
    u = inputs.nldiff_random_u0(12, 5).ravel()
    assert _fd_check(p, u) < 1e-8


def test_vsf_jacobian_fd():
    p = pb.VorticityStreamfunction2D(12, 1e-3)
    st = inputs.vsf_state0(12, 1, 6).ravel()
    st[144:] += 0.01 * np.random.default_rng(0).standard_normal(144)   # off the constraint
    assert _fd_check(p, st) < 1e-8


@pytest.mark.parametrize("n", [8, 10, 14, 16])
def test_vsf_jacobian_fd_coloured(n):
    """Grids whose side is not a multiple of 3 (colourings of period 4, 5,
    7 and 4) against finite differences too."""
    p = pb.VorticityStreamfunction2D(n, 1e-3)
    st = inputs.vsf_state0(n, 2, 4).ravel()
    st[n * n:] += 0.01 * np.random.default_rng(1).standard_normal(n * n)
    assert _fd_check(p, st) < 1e-8


@pytest.mark.parametrize("n", [8, 9, 10, 7])
def test_vsf_coloured_assembly_equals_column_by_column(n):
    """The coloured assembly of each linear block equals the matrix built
    one unit vector at a time (n = 7 has no divisor in [3, n): column by
    column itself)."""
    p = pb.VorticityStreamfunction2D(n, 1e-3)
    om, psi = p.split(inputs.vsf_state0(n, 3, 4).ravel())
    for fn in (lambda x: pb.arakawa(psi, x, p.h) + p.nu * pb.laplacian(x, p.h),
               lambda x: pb.arakawa(x, om, p.h), lambda x: pb.laplacian(x, p.h)):
        a = p._lin_matrix(fn).toarray()
        b = p._lin_matrix_dense(fn).toarray()
        assert np.array_equal(a, b)


def test_burgers_truncation_second_order():
    """N_h(u) vs -(u^2/2)_x + nu u_xx for u = sin(2 pi x) + 0.5 cos(4 pi x)."""
    errs = []
    for n in (32, 64, 128):
        x = np.arange(n) / n
        u = np.sin(2 * np.pi * x) + 0.5 * np.cos(4 * np.pi * x)
        ux = 2 * np.pi * np.cos(2 * np.pi * x) - 2 * np.pi * np.sin(4 * np.pi * x)
        uxx = -4 * np.pi ** 2 * np.sin(2 * np.pi * x) - 8 * np.pi ** 2 * np.cos(4 * np.pi * x)
        exact = -u * ux + 0.01 * uxx
        errs.append(np.max(np.abs(pb.Burgers1D(n, 0.01).rhs(u) - exact)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.1), rates


def test_nldiff_truncation_second_order():
    """N_h(u) (no forcing) vs div((1 + u^2) grad u) for a smooth periodic u."""
    errs = []
    for n in (32, 64, 128):
        p = pb.NonlinearDiffusion2D(n, forcing="none")
        X, Y = p.X, p.Y
        u = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + 0.3 * np.sin(4 * np.pi * Y)
        ux = 2 * np.pi * np.cos(2 * np.pi * X) * np.cos(2 * np.pi * Y)
        uy = -2 * np.pi * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) + 1.2 * np.pi * np.cos(4 * np.pi * Y)
        lap = -8 * np.pi ** 2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) - 4.8 * np.pi ** 2 * np.sin(4 * np.pi * Y)
        exact = (1 + u * u) * lap + 2 * u * (ux * ux + uy * uy)
        errs.append(np.max(np.abs(p.rhs(u.ravel()).reshape(n, n) - exact)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.15), rates


def test_mms_forcing_matches_symbolic():
    """The continuous forcing equals u*_t - div((1+u*^2) grad u*), derived by sympy."""
    x, y, t = sympy.symbols("x y t")
    u = sympy.sin(2 * sympy.pi * x) * sympy.sin(2 * sympy.pi * y) * sympy.cos(t)
    k = 1 + u ** 2
    f = sympy.diff(u, t) - (sympy.diff(k * sympy.diff(u, x), x) + sympy.diff(k * sympy.diff(u, y), y))
    fn = sympy.lambdify((x, y, t), f, "numpy")
    rng = np.random.default_rng(0)
    X, Y, T = rng.uniform(0, 1, 50), rng.uniform(0, 1, 50), rng.uniform(0, 3, 50)
    assert np.max(np.abs(pb.mms_continuous_forcing(X, Y, T) - fn(X, Y, T))) < 1e-11


def test_nldiff_continuous_mms_converges_in_space():
    """With the continuous forcing, u* solves the PDE, so the residual of the
    semi-discrete system on u* is the O(h^2) truncation error."""
    errs = []
    for n in (16, 32, 64):
        p = pb.NonlinearDiffusion2D(n, forcing="continuous")
        t = 0.7
        us = pb.mms_solution(p.X, p.Y, t)
        dudt = -np.sin(2 * np.pi * p.X) * np.sin(2 * np.pi * p.Y) * np.sin(t)
        errs.append(np.max(np.abs(dudt.ravel() - p.rhs(us.ravel(), t))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.15), rates


def test_arakawa_consistency_and_conservation():
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        g = np.arange(n) * h
        X, Y = np.meshgrid(g, g)
        psi = np.sin(2 * np.pi * X) * np.sin(4 * np.pi * Y)
        om = np.cos(2 * np.pi * X + 0.3) * np.sin(2 * np.pi * Y)
        px = 2 * np.pi * np.cos(2 * np.pi * X) * np.sin(4 * np.pi * Y)
        py = 4 * np.pi * np.sin(2 * np.pi * X) * np.cos(4 * np.pi * Y)
        ox = -2 * np.pi * np.sin(2 * np.pi * X + 0.3) * np.sin(2 * np.pi * Y)
        oy = 2 * np.pi * np.cos(2 * np.pi * X + 0.3) * np.cos(2 * np.pi * Y)
        J = pb.arakawa(psi, om, h)
        errs.append(np.max(np.abs(J - (px * oy - py * ox))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.15), rates
    rng = np.random.default_rng(1)
    psi = rng.standard_normal((24, 24))
    om = rng.standard_normal((24, 24))
    J = pb.arakawa(psi, om, 1 / 24)
    scale = np.sum(np.abs(J * om))
    assert abs(J.sum()) < 1e-12 * scale            # vorticity (mean)
    assert abs((om * J).sum()) < 1e-12 * scale     # enstrophy
    assert abs((psi * J).sum()) < 1e-12 * np.sum(np.abs(J * psi))   # energy


def test_vsf_constraint_zero_set():
    """The algebraic rows vanish exactly for the consistent (omega, psi)."""
    p = pb.VorticityStreamfunction2D(32, 1e-3)
    st = inputs.vsf_state0(32, 2, 10)
    r = p.rhs(st.ravel())[32 * 32:]
    assert np.max(np.abs(r)) < 1e-9 * np.abs(st[0]).max()
    assert abs(st[1].mean()) < 1e-14
