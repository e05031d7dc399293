"""GPU parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bars: float64 path (prec_fp32=0) within 1e-10 relative L2 per step; mixed
precision (float32 V-cycles inside float64 FGMRES) within 1e-8; the stage
residual kernel within 1e-13 of the oracle's residual on the same inputs."""
import numpy as np
import pytest

from gpu_common import (gpu, initial_field, oracle_residual, oracle_step, rel)
from paper_2101_01776_amd import irk

pytestmark = gpu

RES_CASES = [
    ("nldiff", irk.make_operator(irk.OP_NLDIFF_2D, 64, forcing=irk.FORCING_MMS), "gauss", 3),
    ("nldiff-ragged", irk.make_operator(irk.OP_NLDIFF_2D, 50, forcing=irk.FORCING_MMS_DISCRETE), "radau", 2),
    ("nldiff-s5", irk.make_operator(irk.OP_NLDIFF_2D, 40, forcing=irk.FORCING_NONE), "gauss", 5),
    ("burgers", irk.make_operator(irk.OP_BURGERS_1D, 256, nu=0.01), "gauss", 2),
    ("burgers-ragged", irk.make_operator(irk.OP_BURGERS_1D, 250, nu=0.01), "radau", 3),
    ("vsf", irk.make_operator(irk.OP_VSF_2D, 48, nu=1e-3), "radau", 3),
    ("vsf-ragged", irk.make_operator(irk.OP_VSF_2D, 30, nu=1e-3), "gauss", 2),
    ("nldiff-lobatto4", irk.make_operator(irk.OP_NLDIFF_2D, 36, forcing=irk.FORCING_MMS), "lobatto", 4),
]


@pytest.mark.parametrize("name,op,family,s", RES_CASES, ids=[c[0] for c in RES_CASES])
def test_stage_residual_matches_oracle(name, op, family, s):
    print(f"[residual] {name} n={op.nx} {family}{s}", flush=True)
    solver = irk.Solver(family, s, op)
    u = initial_field(op, 3)
    rng = np.random.default_rng(11)
    K = rng.standard_normal((s,) + solver.field_shape)
    t, dt = 0.37, 4e-3
    F = solver.eval_residual(u, t, dt, K).cpu().numpy()
    Fo = oracle_residual(op, family, s, u, t, dt, K)
    assert rel(F, Fo) < 1e-13
    solver.close()


# grids of 64 and up run their finest levels through the LDS-tiled multigrid
# kernels (ragged tiles at 96); smaller grids run the whole V-cycle in one
# work-group
STEP_CASES = [
    ("nldiff-gauss3-64", irk.make_operator(irk.OP_NLDIFF_2D, 64, forcing=irk.FORCING_MMS), "gauss", 3, 5e-3),
    ("nldiff-gauss3-96", irk.make_operator(irk.OP_NLDIFF_2D, 96, forcing=irk.FORCING_MMS), "gauss", 3, 5e-3),
    ("nldiff-gauss2-128", irk.make_operator(irk.OP_NLDIFF_2D, 128, forcing=irk.FORCING_MMS), "gauss", 2, 5e-3),
    ("vsf-radau3-64", irk.make_operator(irk.OP_VSF_2D, 64, nu=1e-3), "radau", 3, 2e-3),
    ("nldiff-gauss3", irk.make_operator(irk.OP_NLDIFF_2D, 48, forcing=irk.FORCING_MMS), "gauss", 3, 5e-3),
    ("nldiff-radau3", irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "radau", 3, 5e-3),
    ("nldiff-gauss2-ragged", irk.make_operator(irk.OP_NLDIFF_2D, 40, forcing=irk.FORCING_MMS), "gauss", 2, 5e-3),
    ("nldiff-midpoint", irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "gauss", 1, 2e-3),
    ("nldiff-gauss5", irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "gauss", 5, 1e-2),
    ("burgers-gauss2", irk.make_operator(irk.OP_BURGERS_1D, 256, nu=0.01), "gauss", 2, 1e-2),
    ("burgers-radau3", irk.make_operator(irk.OP_BURGERS_1D, 128, nu=0.01), "radau", 3, 1e-2),
    ("vsf-radau3", irk.make_operator(irk.OP_VSF_2D, 32, nu=1e-3), "radau", 3, 2e-3),
    ("vsf-gauss2", irk.make_operator(irk.OP_VSF_2D, 24, nu=1e-3), "gauss", 2, 2e-3),
    ("nldiff-lobatto2", irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "lobatto", 2, 5e-3),
    ("nldiff-lobatto3-96", irk.make_operator(irk.OP_NLDIFF_2D, 96, forcing=irk.FORCING_MMS), "lobatto", 3, 5e-3),
    ("burgers-lobatto4", irk.make_operator(irk.OP_BURGERS_1D, 128, nu=0.01), "lobatto", 4, 1e-2),
    ("vsf-lobatto3", irk.make_operator(irk.OP_VSF_2D, 24, nu=1e-3), "lobatto", 3, 2e-3),
    # SDIRK comparison methods: stages solved one after another on the same
    # kernels (one real block per stage)
    ("nldiff-sdirk2", irk.make_operator(irk.OP_NLDIFF_2D, 48, forcing=irk.FORCING_MMS), "sdirk", 2, 5e-3),
    ("nldiff-sdirk3-96", irk.make_operator(irk.OP_NLDIFF_2D, 96, forcing=irk.FORCING_MMS), "sdirk", 3, 5e-3),
    ("nldiff-sdirk4", irk.make_operator(irk.OP_NLDIFF_2D, 40, forcing=irk.FORCING_MMS), "sdirk", 5, 5e-3),
    # 96^2: large enough that a context-setup fill sized by the method's s
    # instead of the solver's would reach the forcing tables
    ("nldiff-sdirk4-96", irk.make_operator(irk.OP_NLDIFF_2D, 96, forcing=irk.FORCING_MMS), "sdirk", 5, 5e-3),
    ("burgers-sdirk3", irk.make_operator(irk.OP_BURGERS_1D, 128, nu=0.01), "sdirk", 3, 1e-2),
    ("vsf-sdirk4", irk.make_operator(irk.OP_VSF_2D, 24, nu=1e-3), "sdirk", 5, 2e-3),
    ("nldiff-backward-euler", irk.make_operator(irk.OP_NLDIFF_2D, 32, forcing=irk.FORCING_MMS), "sdirk", 1, 5e-3),
]


@pytest.mark.parametrize("prec_fp32,bar", [(0, 1e-10), (1, 1e-8)], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name,op,family,s,dt", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_step_matches_oracle(name, op, family, s, dt, prec_fp32, bar):
    print(f"[step] {name} n={op.nx} {family}{s} fp32={prec_fp32}", flush=True)
    solver = irk.Solver(family, s, op, irk.make_options(prec_fp32=prec_fp32))
    u = initial_field(op, 0)
    t = 0.0
    for step in range(2 if op.nx <= 48 else 1):
        out, st = solver.step(u, t, dt)
        u1 = out.cpu().numpy()
        uo, Ko, _ = oracle_step(op, family, s, u, t, dt)
        err = rel(u1, uo)
        print(f"  step {step}: rel err {err:.3e} stats {st}", flush=True)
        assert err < bar, (err, st)
        Kg = solver.stages().cpu().numpy()
        assert rel(Kg, Ko) < 100 * bar
        u, t = u1, t + dt
    solver.close()
