"""Option lane_threads: each eigen-block's solve driven by a host thread of
its own.  The device work is the same as with one host thread (the blocks
are independent, their reductions deterministic), so steps, iteration
counts and outputs must agree bit for bit; contexts start and stop their
threads cleanly, also many in a row."""
import numpy as np
import pytest

from gpu_common import gpu, initial_field
from paper_2101_01776_amd import irk

pytestmark = gpu

CASES = [
    ("nldiff64-gauss5", irk.OP_NLDIFF_2D, 64, "gauss", 5, {}),
    ("vsf64-radau3", irk.OP_VSF_2D, 64, "radau", 3, {}),
    ("vsf48-radau3-vcycle", irk.OP_VSF_2D, 48, "radau", 3, {}),
    ("vsf64-radau3-reordered", irk.OP_VSF_2D, 64, "radau", 3, {"dae_reorder": 1}),
    ("burgers256-lobatto4", irk.OP_BURGERS_1D, 256, "lobatto", 4, {}),
    ("nldiff64-gauss4-fp64", irk.OP_NLDIFF_2D, 64, "gauss", 4, {"prec_fp32": 0}),
]


def _run(kind, n, family, s, extra, threads, nsteps=4):
    op = irk.make_operator(kind, n, nu=1e-3 if kind == irk.OP_VSF_2D else 1e-2)
    u = initial_field(op, 1)
    dt = 2e-3 if kind == irk.OP_VSF_2D else 1e-2
    sol = irk.Solver(family, s, op, irk.make_options(lane_threads=threads, **extra))
    outs, stats = [], []
    t = 0.0
    for _ in range(nsteps):
        out, st = sol.step(u, t, dt)
        u = out.cpu().numpy()
        outs.append(u.copy())
        stats.append((st["newton_its"], st["krylov_its"], tuple(st["krylov_its_block"])))
        t += dt
    sol.close()
    return outs, stats


@pytest.mark.parametrize("name,kind,n,family,s,extra", CASES, ids=[c[0] for c in CASES])
def test_threads_give_the_same_steps(name, kind, n, family, s, extra):
    o0, s0 = _run(kind, n, family, s, extra, 0)
    o1, s1 = _run(kind, n, family, s, extra, 1)
    print(f"  {name}: per step (Newton, Krylov, per block) {s1}", flush=True)
    assert s0 == s1
    for a, b in zip(o0, o1):
        assert np.array_equal(a, b)


def test_many_contexts_start_and_stop_their_threads():
    op = irk.make_operator(irk.OP_NLDIFF_2D, 32)
    u = initial_field(op, 2)
    ref = None
    for k in range(24):
        sol = irk.Solver("gauss", 3, op, irk.make_options(lane_threads=1))
        if k % 3 == 0:
            out, _ = sol.step(u, 0.0, 1e-2)
            out = out.cpu().numpy()
            if ref is None:
                ref = out
            assert np.array_equal(out, ref)
        sol.close()
