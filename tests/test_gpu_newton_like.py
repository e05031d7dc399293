"""GPU eigen-block operators and steps under the four Newton-like
truncations of Section 3.2 (0: last-stage Jacobian, 1: lumped to the
largest stage weight, 2: the row's stage weights, 3: plus the coupling of
the two rows of a pair), against the oracle's written-out block operators
and its full-Newton step."""
import numpy as np
import pytest

from gpu_common import gpu, oracle_problem, oracle_step, rel
from oracle import newton as nw
from oracle import tableau as tb
from paper_2101_01776_amd import inputs, irk

pytestmark = gpu

OPS = {
    "burgers64": lambda: irk.make_operator(irk.OP_BURGERS_1D, 64, nu=0.01),
    "nldiff24": lambda: irk.make_operator(irk.OP_NLDIFF_2D, 24, forcing=irk.FORCING_MMS),
}
FAMS = [("gauss", 2), ("gauss", 3), ("gauss", 5), ("radau", 3), ("lobatto", 3)]


def _field(name, op):
    if op.kind == irk.OP_BURGERS_1D:
        return inputs.burgers_u0(op.nx, 4)
    return inputs.nldiff_random_u0(op.nx, 21)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("family,s", FAMS)
@pytest.mark.parametrize("name", sorted(OPS))
def test_block_operator_matches_oracle(name, family, s, variant):
    """irk_apply_block equals the oracle's block operator D_b x for every
    eigen-block, at the stage values of seeded stage vectors K (1e-12
    relative: the same sums up to rounding order).  The oracle builds its
    own eigenbasis; it must coincide with the library's (the normalization
    makes it unique).  Under (1) rows whose two largest weights tie (Gauss-3,
    Gauss-5, Lobatto-3) lump to the lower stage index on both sides."""
    op = OPS[name]()
    prob = oracle_problem(op)
    A, _, c = tb.tableau(family, s)
    T, blocks = tb.real_eigenbasis(A)
    e = irk.irk_eigen_blocks(family, s)
    assert np.abs(T - e["T"]).max() < 1e-12
    u = _field(name, op)
    rng = np.random.default_rng(100 * s + variant)
    K = 0.5 * rng.standard_normal((s,) + tuple(np.shape(u)))
    t, dt = 0.05, 5e-3
    sol = irk.Solver(family, s, op, irk.make_options(newton_like=variant, prec_fp32=0))
    sol.eval_residual(u, t, dt, K)
    for b, blk in enumerate(blocks):
        width = blk[1]
        x = rng.standard_normal((width,) + tuple(np.shape(u)))
        y = sol.apply_block(b, x).cpu().numpy()
        D = nw.block_operator(prob, A, c, np.ravel(u), t, dt, K.reshape(s, -1), T, blk, variant)
        want = D @ x.ravel()
        assert rel(y, want) < 1e-12, (b, rel(y, want))
    sol.close()


STEP = [
    ("nldiff32-gauss3", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "gauss", 3, 5e-3),
    ("nldiff32-radau2", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "radau", 2, 1e-2),
    ("burgers128-gauss3", lambda: irk.make_operator(irk.OP_BURGERS_1D, 128, nu=0.01), "gauss", 3, 1e-2),
    ("vsf24-radau3", lambda: irk.make_operator(irk.OP_VSF_2D, 24, nu=1e-3), "radau", 3, 2e-3),
]


@pytest.mark.parametrize("prec_fp32,bar", [(0, 1e-10), (1, 1e-8)], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name,mk,family,s,dt", STEP, ids=[c[0] for c in STEP])
def test_step_newton_like_2_3_matches_oracle(name, mk, family, s, dt, prec_fp32, bar):
    """Newton-like (2) and (3) reach the same step as the oracle's full
    Newton (the truncation only changes the iteration, Section 3.2), at the
    parity bars of the other step tests; iteration counts are printed with
    those of (0) and (1)."""
    op = mk()
    if op.kind == irk.OP_VSF_2D:
        u = inputs.vsf_state0(op.nx, 2, n_vortices=8)
    elif op.kind == irk.OP_BURGERS_1D:
        u = inputs.burgers_u0(op.nx, 2)
    else:
        u = inputs.nldiff_u0(op.nx)
    want, _, _ = oracle_step(op, family, s, u, 0.0, dt)
    its = {}
    for v in (0, 1, 2, 3):
        sol = irk.Solver(family, s, op, irk.make_options(newton_like=v, prec_fp32=prec_fp32))
        out, st = sol.step(u, 0.0, dt)
        its[v] = (st["newton_its"], st["krylov_its"])
        assert rel(out.cpu().numpy(), want) < bar, (v, rel(out.cpu().numpy(), want))
        sol.close()
    print(f"  {name}: Newton / Krylov its by Newton-like variant {its}")


GAMMA_ETA = [
    ("nldiff48-gauss3", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 48, forcing=irk.FORCING_MMS), "gauss", 3, 5e-3),
    ("nldiff64-radau3", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 64, forcing=irk.FORCING_MMS), "radau", 3, 5e-3),
    ("vsf32-radau3", lambda: irk.make_operator(irk.OP_VSF_2D, 32, nu=1e-3), "radau", 3, 2e-3),
]


@pytest.mark.parametrize("prec_fp32,bar", [(0, 1e-10), (1, 1e-8)], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name,mk,family,s,dt", GAMMA_ETA, ids=[c[0] for c in GAMMA_ETA])
def test_step_gamma_eta_matches_oracle(name, mk, family, s, dt, prec_fp32, bar):
    """The Schur-complement approximation with gamma = eta (equation
    (schur-approx) without the gamma_* of equation (gamma*); the comparison
    of Table 4) changes only the preconditioner: the step equals the
    oracle's (the pair blocks' Krylov iterations of both are printed)."""
    op = mk()
    u = inputs.vsf_state0(op.nx, 2, n_vortices=8) if op.kind == irk.OP_VSF_2D else inputs.nldiff_random_u0(op.nx, 5)
    want, _, _ = oracle_step(op, family, s, u, 0.0, dt)
    its = {}
    for gm in (1, 0):
        sol = irk.Solver(family, s, op, irk.make_options(gamma_mode=gm, prec_fp32=prec_fp32, krylov_adaptive=0))
        out, st = sol.step(u, 0.0, dt)
        err = rel(out.cpu().numpy(), want)
        its[gm] = st["krylov_its_block"]
        print(f"  {name} gamma_mode={gm}: rel err {err:.3e} krylov per block {st['krylov_its_block']}", flush=True)
        assert err < bar, (gm, err)
        sol.close()
    blocks = irk.irk_eigen_blocks(family, s)
    pair = [b for b in range(blocks["nblocks"]) if blocks["width"][b] == 2]
    print(f"  pair-block Krylov iterations gamma*: {[its[0][b] for b in pair]}, "
          f"eta: {[its[1][b] for b in pair]}", flush=True)


SLOW = [
    ("nldiff32-gauss3-dt2e-2", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "gauss", 3, 2e-2),
    ("nldiff32-gauss5-dt4e-2", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "gauss", 5, 4e-2),
]


@pytest.mark.parametrize("name,mk,family,s,dt", SLOW, ids=[c[0] for c in SLOW])
def test_slowly_contracting_iteration_reaches_threshold(name, mk, family, s, dt):
    """Simplified Newton (truncation (0), every row at the last stage's
    Jacobian) on a strongly nonlinear field with a large step contracts only
    linearly; it must still run to the acceptance threshold (not be stopped
    by the stagnation safety net: acceptance 0 or 1) and reach the oracle's
    step at the float64 bar."""
    op = mk()
    u = inputs.nldiff_random_u0(op.nx, 9)
    want, _, _ = oracle_step(op, family, s, u, 0.0, dt)
    sol = irk.Solver(family, s, op, irk.make_options(newton_like=0, prec_fp32=0))
    out, st = sol.step(u, 0.0, dt)
    err = rel(out.cpu().numpy(), want)
    print(f"  {name}: newton its {st['newton_its']} res0 {st['res0']:.3e} final {st['final_res']:.3e} "
          f"acceptance {st['acceptance']} rel err {err:.3e}", flush=True)
    assert st["acceptance"] in (0, 1), st
    assert err < 1e-10, err
    sol.close()


SCHUR = [
    ("nldiff64-gauss3", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 64, forcing=irk.FORCING_MMS), "gauss", 3, 5e-3),
    ("nldiff32-gauss5", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "gauss", 5, 1e-2),
    ("nldiff48-radau3", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 48, forcing=irk.FORCING_MMS), "radau", 3, 5e-3),
    ("nldiff40-gauss4", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 40, forcing=irk.FORCING_MMS), "gauss", 4, 5e-3),
    ("burgers128-radau5", lambda: irk.make_operator(irk.OP_BURGERS_1D, 128, nu=0.01), "radau", 5, 1e-2),
]


@pytest.mark.parametrize("prec_fp32,bar", [(0, 1e-10), (1, 1e-8)], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name,mk,family,s,dt", SCHUR, ids=[c[0] for c in SCHUR])
def test_step_schur_basis_matches_oracle(name, mk, family, s, dt, prec_fp32, bar):
    """The real Schur basis (option transform = 1): blocks solved last to
    first by back-substitution (Section 5, equation (D+U)), under Newton-like
    (1) (the couplings R0_ij M) and (3) (also the stage-weighted Jacobian
    terms of the truncation to R0's block-upper pattern), reach the oracle's
    full-Newton step at the parity bars; two steps, the second continued."""
    op = mk()
    u0 = inputs.burgers_u0(op.nx, 3) if op.kind == irk.OP_BURGERS_1D else inputs.nldiff_random_u0(op.nx, 6)
    w1, K1, _ = oracle_step(op, family, s, u0, 0.0, dt)
    w2, _, _ = oracle_step(op, family, s, w1, dt, dt)
    for v in (1, 3):
        sol = irk.Solver(family, s, op, irk.make_options(newton_like=v, transform=1, prec_fp32=prec_fp32))
        a = sol._dev(u0)
        b = torch_empty_like(a)
        _, st1 = sol.step(a, 0.0, dt, out=b)
        e1 = rel(b.cpu().numpy(), w1)
        _, st2 = sol.step(b, dt, dt, out=a)
        e2 = rel(a.cpu().numpy(), w2)
        print(f"  {name} Schur NL({v}): rel err {e1:.3e} {e2:.3e}; Newton/Krylov "
              f"{st1['newton_its']}/{st1['krylov_its']}, {st2['newton_its']}/{st2['krylov_its']}", flush=True)
        assert e1 < bar and e2 < bar, (v, e1, e2)
        sol.close()


def torch_empty_like(t):
    import torch
    return torch.empty_like(t)
