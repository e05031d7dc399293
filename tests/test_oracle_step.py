"""Pins of the oracle's Newton / sparse-LU step against results fixed by the
mathematics: the stability function on linear problems (scalar and per
Fourier mode), an independent nonlinear solver (MINPACK), the order of
accuracy against an independent explicit reference, conservation of quadratic
invariants by Gauss methods, and the exact reduction of the index-1 DAE."""
import numpy as np
import pytest
import scipy.integrate as si
import scipy.optimize as so
import scipy.sparse as sp

from oracle import newton as nw
from oracle import problems as pb
from oracle import tableau as tb
from paper_2101_01776_amd import inputs

FAMS = ([("gauss", s) for s in (1, 2, 3, 4, 5)] + [("radau", s) for s in (1, 2, 3, 4, 5)] +
        [("lobatto", s) for s in (2, 3, 4, 5)] + [("sdirk", s) for s in (1, 2, 3, 5)])


class _Diagonal:
    """u' = diag(lam) u (a stack of Dahlquist test equations)."""

    def __init__(self, lam):
        self.lam = np.asarray(lam, dtype=float)
        self.size = len(self.lam)
        self.mass = np.ones(self.size)

    def rhs(self, u, t=0.0):
        return self.lam * u

    def jac(self, u, t=0.0):
        return sp.diags(self.lam).tocsr(), None, None


@pytest.mark.parametrize("family,s", FAMS)
def test_scalar_step_is_stability_function(family, s):
    A, b, c = tb.tableau(family, s)
    lam = np.array([-0.5, -7.0, -3000.0, 0.7])
    u0 = np.array([1.0, -2.0, 0.5, 3.0])
    dt = 0.1
    u1, _, _ = nw.irk_step(_Diagonal(lam), A, b, c, u0, 0.0, dt)
    want = np.array([tb.stability_function(A, b, dt * l).real for l in lam]) * u0
    # relative to the value, plus a rounding allowance on the input scale for
    # the strongly damped stiff mode (L-stable methods: R(-300) ~ 1e-5)
    assert np.all(np.abs(u1 - want) <= 1e-13 * np.abs(want) + 4e-15 * np.abs(u0))


@pytest.mark.parametrize("family,s", [("gauss", 3), ("radau", 3), ("gauss", 5)])
def test_linear_diffusion_fourier_symbol(family, s):
    """Frozen-coefficient (kappa = 1) periodic diffusion: each Fourier mode is
    multiplied by R(dt lambda_k), lambda_k = -(4/h^2)(sin^2(pi kx/n) + sin^2(pi ky/n))."""
    n = 16
    A, b, c = tb.tableau(family, s)
    p = pb.NonlinearDiffusion2D(n, forcing="none", kappa_quadratic=False)
    u0 = inputs.nldiff_random_u0(n, 7)
    dt = 5e-3
    u1, _, _ = nw.irk_step(p, A, b, c, u0.ravel(), 0.0, dt)
    k = np.arange(n)
    s1 = (4.0 * n * n) * np.sin(np.pi * k / n) ** 2
    lam = -(s1[:, None] + s1[None, :])
    R = np.vectorize(lambda z: tb.stability_function(A, b, z).real)(dt * lam)
    want = np.real(np.fft.ifft2(R * np.fft.fft2(u0)))
    assert np.linalg.norm(u1 - want.ravel()) / np.linalg.norm(want) < 1e-12


@pytest.mark.parametrize("family,s", [("gauss", 2), ("gauss", 3), ("radau", 2), ("radau", 3)])
def test_matches_minpack_root(family, s):
    """Stage solution equals MINPACK's hybrid root of the same residual."""
    A, b, c = tb.tableau(family, s)
    for prob, u0, dt in ((pb.Burgers1D(32, 0.01), inputs.burgers_u0(32, 1), 1e-2),
                         (pb.NonlinearDiffusion2D(8), inputs.nldiff_u0(8).ravel(), 5e-3)):
        K, _ = nw.irk_stages(prob, A, c, u0, 0.2, dt)
        K0, _ = nw.initial_stages(prob, A, c, u0, 0.2, dt)
        sol = so.root(lambda z: nw.stage_residual(prob, A, c, u0, 0.2, dt, z.reshape(K.shape)).ravel(),
                      K0.ravel(), method="hybr", options={"xtol": 1e-15, "maxfev": 200000})
        Kr = sol.x.reshape(K.shape)
        assert np.linalg.norm(K - Kr) / np.linalg.norm(K) < 1e-11


@pytest.mark.parametrize("family,s", [("gauss", 1), ("gauss", 2), ("gauss", 3),
                                      ("radau", 1), ("radau", 2), ("radau", 3),
                                      ("lobatto", 2), ("lobatto", 3), ("lobatto", 4),
                                      ("sdirk", 2), ("sdirk", 3), ("sdirk", 5)])
def test_order_of_accuracy(family, s):
    """Observed order 2s (Gauss) / 2s-1 (Radau IIA) / 2s-2 (Lobatto IIIC) /
    2, 3, 4 (the SDIRK methods with 2, 3, 5 stages) on 1-D Burgers (n=32),
    against an explicit DOP853 reference at rtol 1e-13."""
    n, nu, T = 32, 0.01, 0.4
    prob = pb.Burgers1D(n, nu)
    u0 = 0.5 * inputs.burgers_u0(n, 4)
    ref = si.solve_ivp(lambda t, u: prob.rhs(u, t), (0, T), u0, method="DOP853",
                       rtol=1e-13, atol=1e-15).y[:, -1]
    A, b, c = tb.tableau(family, s)
    p = {"gauss": 2 * s, "radau": 2 * s - 1, "lobatto": 2 * s - 2, "sdirk": {2: 2, 3: 3, 5: 4}.get(s)}[family]
    dts = [0.1, 0.05, 0.025] if p >= 5 else [0.05, 0.025, 0.0125]
    errs = []
    for dt in dts:
        u = u0.copy()
        for m in range(int(round(T / dt))):
            u, _, _ = nw.irk_step(prob, A, b, c, u, m * dt, dt)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert min(errs) > 1e-12, errs          # still above the solver floor
    assert abs(rates[-1] - p) < 0.3, (errs, rates)


def test_gauss_conserves_quadratic_invariants_vsf():
    """With nu = 0, the Arakawa semi-discretization conserves enstrophy
    sum(omega^2) and energy sum(psi omega); Gauss methods conserve quadratic
    invariants, Radau IIA dissipates them."""
    n = 12
    prob = pb.VorticityStreamfunction2D(n, 0.0)
    st0 = inputs.vsf_state0(n, 3, 6).ravel()
    nn = n * n
    ens = lambda u: np.sum(u[:nn] ** 2)
    energy = lambda u: np.sum(u[:nn] * u[nn:])
    for fam, s in (("gauss", 2), ("gauss", 3)):
        A, b, c = tb.tableau(fam, s)
        u1, _, _ = nw.irk_step(prob, A, b, c, st0, 0.0, 5e-2)
        assert abs(ens(u1) - ens(st0)) / ens(st0) < 1e-12
        assert abs(energy(u1) - energy(st0)) / energy(st0) < 1e-12
    A, b, c = tb.tableau("radau", 2)
    u1, _, _ = nw.irk_step(prob, A, b, c, st0, 0.0, 0.5)
    assert ens(u1) < ens(st0) * (1 - 1e-8)


def test_dae_equals_reduced_ode():
    """A linear, uniquely solvable constraint: the DAE step equals the step of
    the reduced ODE omega' = J_A(psi(omega), omega) + nu Lap omega with
    psi(omega) the spectral inverse of -Lap_h; psi_{n+1} stays consistent."""
    n, nu, dt = 12, 1e-2, 1e-2
    prob = pb.VorticityStreamfunction2D(n, nu)
    st0 = inputs.vsf_state0(n, 5, 5)
    h = 1.0 / n

    def reduced_rhs(om_flat):
        om = om_flat.reshape(n, n)
        psi = inputs.vsf_psi0(om)
        return (pb.arakawa(psi, om, h) + nu * pb.laplacian(om, h)).ravel()

    for fam, s in (("radau", 2), ("gauss", 2), ("radau", 3)):
        A, b, c = tb.tableau(fam, s)
        u1, _, _ = nw.irk_step(prob, A, b, c, st0.ravel(), 0.0, dt)
        om0 = st0[0].ravel()
        res = lambda z: np.concatenate([
            z.reshape(s, -1)[i] - reduced_rhs(om0 + dt * (A[i] @ z.reshape(s, -1))) for i in range(s)])
        # plain Newton on the reduced stage equations with a dense
        # central-difference Jacobian (independent of the DAE formulation)
        z = np.concatenate([reduced_rhs(om0)] * s)
        for _ in range(30):
            r = res(z)
            if np.linalg.norm(r) <= 1e-13 * np.linalg.norm(z):
                break
            eps = 1e-7 * max(1.0, np.abs(z).max())
            Jd = np.empty((z.size, z.size))
            for q in range(z.size):
                e = np.zeros(z.size)
                e[q] = eps
                Jd[:, q] = (res(z + e) - res(z - e)) / (2 * eps)
            z = z - np.linalg.solve(Jd, r)
        om1 = om0 + dt * (b @ z.reshape(s, -1))
        assert np.linalg.norm(u1[: n * n] - om1) / np.linalg.norm(om1) < 1e-11
        psi1 = u1[n * n:].reshape(n, n)
        assert np.max(np.abs(psi1 - inputs.vsf_psi0(u1[: n * n].reshape(n, n)))) < 1e-11 * np.abs(psi1).max()


def test_radau_update_equals_last_stage():
    """Radau IIA is stiffly accurate: u_n + dt sum b_i k_i = U_s."""
    A, b, c = tb.tableau("radau", 3)
    prob = pb.NonlinearDiffusion2D(8)
    u0 = inputs.nldiff_u0(8).ravel()
    u1, K, _ = nw.irk_step(prob, A, b, c, u0, 0.0, 5e-3)
    Us = nw.stage_values(A, u0, 5e-3, K)[-1]
    assert np.max(np.abs(u1 - Us)) < 1e-15 * max(1.0, np.abs(u1).max()) * 10


def test_starting_vectors_choice_and_independence():
    """The starting stage vectors are the better of K = 0 and the explicit
    k_i = N(u_n, t_n): the explicit one for smooth motion resolved by the
    grid (the manufactured solution at t = 0.2 on 256^2), zero for a stiff
    decaying transient (modes up to 3 per direction at dt = 5e-3, where
    dt * lambda ~ 4 makes the explicit guess overshoot).  Either start
    converges to the same stage vectors."""
    A, b, c = tb.tableau("gauss", 3)
    fine = pb.NonlinearDiffusion2D(256)
    u_f = inputs.nldiff_u0(256).ravel() * np.cos(0.2)        # u*(t = 0.2)
    K0, pick = nw.initial_stages(fine, A, c, u_f, 0.2, 5e-3)
    assert pick == 1
    np.testing.assert_array_equal(K0[2], fine.rhs(u_f, 0.2))
    smooth = pb.NonlinearDiffusion2D(16)
    u_s = inputs.nldiff_u0(16).ravel()
    stiff = pb.NonlinearDiffusion2D(32)
    u_r = inputs.nldiff_random_u0(32, 579470083).ravel()
    K0, pick = nw.initial_stages(stiff, A, c, u_r, 0.0, 5e-3)
    assert pick == 0
    assert not np.any(K0)
    for prob, u in ((smooth, u_s), (stiff, u_r)):
        Ka, _ = nw.irk_stages(prob, A, c, u, 0.0, 5e-3, K0=np.zeros((3, prob.size)))
        Kb, _ = nw.irk_stages(prob, A, c, u, 0.0, 5e-3, K0=np.stack([prob.rhs(u, 0.0)] * 3))
        assert np.linalg.norm(Ka - Kb) <= 1e-12 * np.linalg.norm(Ka)
    # algebraic rows of the DAE start at zero in the explicit candidate
    vsf = pb.VorticityStreamfunction2D(12, nu=1e-3)
    x = inputs.vsf_state0(12, 3, 6).ravel()
    Ar, br, cr = tb.tableau("radau", 2)
    K0, _ = nw.initial_stages(vsf, Ar, cr, x, 0.0, 1e-3)
    assert not np.any(K0[:, vsf.size // 2:])


@pytest.mark.parametrize("s", [1, 2, 3, 5])
def test_extrapolated_stages_reproduce_polynomials(s):
    """The extrapolation weights are those of polynomial interpolation on the
    nodes: stage vectors sampled from any polynomial of degree < s at the
    previous step's nodes continue exactly to the new nodes, for any step
    ratio."""
    _, _, c = tb.tableau("gauss", s)
    rng = np.random.default_rng(s)
    coef = rng.standard_normal((s, 4))                  # 4 independent polynomials
    for ratio in (1.0, 0.5, 2.0):
        K_prev = np.stack([sum(coef[p] * cj ** p for p in range(s)) for cj in c])
        got = nw.extrapolated_stages(c, K_prev, 1e-2, ratio * 1e-2)
        x = 1.0 + np.asarray(c) * ratio
        want = np.stack([sum(coef[p] * xi ** p for p in range(s)) for xi in x])
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_extrapolated_start_on_continued_steps():
    """With the semi-discrete manufactured forcing (u* solves the discrete
    system exactly, no initial layer) a continued step starts from the
    extrapolated stage vectors: their residual is orders of magnitude below
    the explicit candidate's (the extrapolation error is O(dt^s) against
    O(dt) for the explicit guess), and the converged stages equal those
    reached from K = 0.  (With the continuous forcing u* is off the discrete
    slow manifold and the first steps carry a decaying transient that
    polynomial extrapolation amplifies; the residual rule then keeps the
    explicit or zero start.)"""
    A, b, c = tb.tableau("gauss", 3)
    prob = pb.NonlinearDiffusion2D(16, forcing="discrete")
    u = inputs.nldiff_u0(16).ravel()
    dt = 5e-3
    u1, K1, _ = nw.irk_step(prob, A, b, c, u, 0.0, dt)
    K0, pick = nw.initial_stages(prob, A, c, u1, dt, dt, prev=(K1, dt))
    assert pick == 2
    r_ex = np.linalg.norm(nw.stage_residual(prob, A, c, u1, dt, dt, K0))
    r_expl = np.linalg.norm(nw.stage_residual(prob, A, c, u1, dt, dt, np.stack([prob.rhs(u1, dt)] * 3)))
    assert r_ex < 1e-3 * r_expl
    Ka, _ = nw.irk_stages(prob, A, c, u1, dt, dt, prev=(K1, dt))
    Kz, _ = nw.irk_stages(prob, A, c, u1, dt, dt, K0=np.zeros_like(K1))
    # K (~0.1 here) is the small difference of operator terms of size ~1e3:
    # the stage solve resolves it to ~1e-12 absolute
    assert np.linalg.norm(Ka - Kz) <= 1e-10 * np.linalg.norm(Ka)


@pytest.mark.parametrize("t", [0.0, 0.3, 1.1])
def test_discrete_forcing_makes_ustar_exact(t):
    """With forcing="discrete" the manufactured u*(t) = sin2pix sin2piy cos t
    solves the semi-discrete system exactly: N_h(u*(t), t) equals du*/dt,
    here taken by a fourth-order central difference of u* in time (step
    1e-3: truncation ~1e-14, rounding ~1e-13 of |N_h(u*)|).  A wrong sign of
    the time derivative or a missing flux term leaves an O(1) mismatch."""
    n = 16
    prob = pb.NonlinearDiffusion2D(n, forcing="discrete")
    S = np.sin(2 * np.pi * prob.X) * np.sin(2 * np.pi * prob.Y)

    def ustar(tt):
        return (S * np.cos(tt)).ravel()

    tau = 1e-3
    dudt = (-ustar(t + 2 * tau) + 8 * ustar(t + tau) - 8 * ustar(t - tau) + ustar(t - 2 * tau)) / (12 * tau)
    scale = np.linalg.norm(prob.flux_operator(ustar(t).reshape(n, n)))
    assert np.linalg.norm(prob.rhs(ustar(t), t) - dudt) <= 1e-11 * scale


@pytest.mark.parametrize("family,s,rate", [("gauss", 2, 3.5), ("radau", 2, 2.3), ("gauss", 3, 4.5)])
def test_discrete_forcing_trajectory_converges_to_ustar(family, s, rate):
    """The oracle's steps on the semi-discrete manufactured problem track
    u*(t) up to the time-discretization error only: from u*(0) to T = 0.4 the
    error falls monotonically as dt halves (0.2 -> 0.025), at an observed rate
    of at least `rate` on the last halving (the stiff modes, dt lambda up to
    ~800 here, reduce the classical orders 2s / 2s-1 towards the stage order
    at these dt), and stays below 1e-7 (4e-10 for Gauss-3) at dt = 0.025."""
    n = 16
    prob = pb.NonlinearDiffusion2D(n, forcing="discrete")
    S = np.sin(2 * np.pi * prob.X) * np.sin(2 * np.pi * prob.Y)
    A, b, c = tb.tableau(family, s)
    errs = []
    for dt in (0.2, 0.1, 0.05, 0.025):
        u, t = (S * np.cos(0.0)).ravel(), 0.0
        for _ in range(int(round(0.4 / dt))):
            u, _, _ = nw.irk_step(prob, A, b, c, u, t, dt)
            t += dt
        want = (S * np.cos(t)).ravel()
        errs.append(np.linalg.norm(u - want) / np.linalg.norm(want))
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1)), errs
    assert np.log2(errs[-2] / errs[-1]) >= rate, errs
    assert errs[-1] < (4e-10 if s == 3 else 1e-7), errs
