"""The spectral solve of the streamfunction rows (option psi_solve = 0).

The Poisson block -dt Lap_h of the streamfunction rows has constant
coefficients on the periodic grid, so its discrete Fourier modes diagonalize
it and the preconditioner can apply its inverse exactly.  Checks:

* exactness: in the reordered DAE system (eq (vsf-system-2)) the
  streamfunction rows are a Krylov solve of their own, preconditioned by this
  solve; with an exact inverse it converges in one iteration per block and
  Newton iteration (the V-cycle of psi_solve = 1 needs more);
* parity: the step agrees with the oracle's with either setting, and the two
  settings agree with each other;
* the sides it takes: powers of two (a ragged or odd side, and 48, fall back
  to the V-cycle and still reach the oracle's step).
"""
import numpy as np
import pytest

from gpu_common import gpu, oracle_step, rel
from paper_2101_01776_amd import inputs, irk

pytestmark = gpu


@pytest.mark.parametrize("prec_fp32", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("n,family,s", [(32, "radau", 3), (64, "gauss", 2)], ids=["32-radau3", "64-gauss2"])
def test_streamfunction_solve_is_exact(n, family, s, prec_fp32):
    op = irk.make_operator(irk.OP_VSF_2D, n, nu=1e-3)
    u = inputs.vsf_state0(n, 3, n_vortices=8)
    nblocks = len(irk.irk_eigen_blocks(family, s)["eta"])
    res = {}
    for psi in (0, 1):
        sol = irk.Solver(family, s, op, irk.make_options(prec_fp32=prec_fp32, dae_reorder=1, psi_solve=psi))
        out, st = sol.step(u, 0.0, 2e-3)
        res[psi] = (out.cpu().numpy(), st)
        sol.close()
        print(f"  psi_solve={psi}: Newton {st['newton_its']} Krylov {st['krylov_its']} "
              f"streamfunction Krylov {st['krylov_its_psi']}", flush=True)
    st0, st1 = res[0][1], res[1][1]
    assert st0["krylov_its_psi"] == st0["newton_its"] * nblocks
    assert st1["krylov_its_psi"] > st1["newton_its"] * nblocks
    assert rel(res[0][0], res[1][0]) < (1e-10 if prec_fp32 == 0 else 1e-8)


@pytest.mark.parametrize("prec_fp32,bar", [(0, 1e-10), (1, 1e-8)], ids=["fp64", "mixed"])
@pytest.mark.parametrize("n", [64, 48, 30], ids=["64-spectral", "48-vcycle", "30-vcycle"])
def test_step_matches_oracle_with_either_streamfunction_solve(n, prec_fp32, bar):
    op = irk.make_operator(irk.OP_VSF_2D, n, nu=1e-3)
    u = inputs.vsf_state0(n, 4, n_vortices=8)
    want, _, _ = oracle_step(op, "radau", 3, u, 0.0, 2e-3)
    its = {}
    for psi in (0, 1):
        sol = irk.Solver("radau", 3, op, irk.make_options(prec_fp32=prec_fp32, psi_solve=psi))
        out, st = sol.step(u, 0.0, 2e-3)
        its[psi] = st["krylov_its"]
        assert rel(out.cpu().numpy(), want) < bar, (psi, rel(out.cpu().numpy(), want))
        sol.close()
    print(f"  n={n}: Krylov its spectral {its[0]}, V-cycle {its[1]}", flush=True)
    if n & (n - 1):
        assert its[0] == its[1]        # not a power of two: both settings use the V-cycle


def test_full_size_spectral_solve_matches_vcycle():
    """The bench's 1024^2 DAE step (Radau IIA-3, dt 2e-3, 32 vortices; mixed
    precision) with the spectral streamfunction solve and with the Poisson
    V-cycle: the converged steps agree (the preconditioner changes, the fixed
    point does not).  In the reordered system with float64 transforms
    (float64 V-cycle precision) every streamfunction solve is a one-iteration
    Krylov solve at full size; float32 transforms are exact only to about
    the Laplacian's condition number (1e5 here) times float32 rounding."""
    import torch
    n = 1024
    op = irk.make_operator(irk.OP_VSF_2D, n, nu=1e-3)
    u = torch.tensor(inputs.vsf_state0(n, 0, 32), dtype=torch.float64, device="cuda")
    outs = {}
    for psi in (0, 1):
        sol = irk.Solver("radau", 3, op, irk.make_options(psi_solve=psi))
        out, st = sol.step(u, 0.0, 2e-3)
        outs[psi] = out.cpu().numpy()
        sol.close()
        print(f"  psi_solve={psi}: Newton {st['newton_its']} Krylov {st['krylov_its']}", flush=True)
    assert rel(outs[0], outs[1]) < 1e-8, rel(outs[0], outs[1])
    sol = irk.Solver("radau", 3, op, irk.make_options(psi_solve=0, dae_reorder=1, prec_fp32=0))
    out, st = sol.step(u, 0.0, 2e-3)
    sol.close()
    print(f"  reordered, float64: Newton {st['newton_its']} streamfunction Krylov {st['krylov_its_psi']}", flush=True)
    assert st["krylov_its_psi"] == st["newton_its"] * 2          # one real block and one pair
    assert rel(out.cpu().numpy(), outs[0]) < 1e-8
