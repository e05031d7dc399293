"""Time convergence on the 1024^2 nonlinear-diffusion problem with 5-stage
Gauss (order 10), float64 and float32 V-cycles.

The errors are measured against a small-dt Gauss-5 solution of the same
semi-discrete system (the spatial error, ~1e-6, would mask the temporal one
against u*).  The problem is stiff (8 kappa dt / h^2 ~ 1e5), so the observed
rate sits between the stage order plus one and the classical order 10; the
checks are that the error falls at high order as dt halves and that the
float32 preconditioner does not move the converged steps."""
import numpy as np

from gpu_common import gpu, rel
from paper_2101_01776_amd import inputs, irk

pytestmark = gpu

N = 1024


def _run(dt, T, prec, s=5, n=N):
    import torch
    op = irk.make_operator(irk.OP_NLDIFF_2D, n, forcing=irk.FORCING_MMS)
    sol = irk.Solver("gauss", s, op, irk.make_options(prec_fp32=prec))
    u = torch.tensor(inputs.nldiff_u0(n), dtype=torch.float64, device="cuda")
    out = torch.empty_like(u)
    steps = int(round(T / dt))
    t = 0.0
    its = 0
    for _ in range(steps):
        _, st = sol.step(u, t, dt, out=out)
        u, out = out, u
        t += dt
        its += st["newton_its"]
    res = u.cpu().numpy()
    sol.close()
    return res, its / steps


def test_gauss5_convergence_at_config_steps():
    """dt in {0.04, 0.02, 0.01} to T = 0.2 against dt = 0.0025."""
    ref, _ = _run(0.0025, 0.2, 0)
    errs = []
    for dt in (0.04, 0.02, 0.01):
        u64, n64 = _run(dt, 0.2, 0)
        u32, n32 = _run(dt, 0.2, 1)
        e64, e32 = rel(u64, ref), rel(u32, ref)
        errs.append(e64)
        print(f"  dt {dt}: err fp64 {e64:.3e} mixed {e32:.3e} |mixed - fp64| {rel(u32, u64):.3e} "
              f"newton/step {n64:.2f} {n32:.2f}")
        assert rel(u32, u64) < 1e-10
        # the same error in both precisions; at dt = 0.01 the error sits at
        # the float64 rounding floor (about 1e-15), where the two differ by
        # rounding alone
        assert abs(e32 - e64) <= max(1e-3 * e64, 1e-14)
    orders = [np.log2(errs[k] / errs[k + 1]) for k in range(2)]
    print("  observed orders", orders)
    assert errs[0] > errs[1] > errs[2]
    assert min(orders) > 4.0


def test_gauss5_large_dt_still_converges():
    """dt in {0.4, 0.2, 0.1} to T = 0.4 against dt = 0.0125: every step
    converges and the error falls as dt halves.  At these step sizes the
    stiff components are poorly damped by Gauss (|R(inf)| = 1) and the
    observed order is reduced (about 1 and 3 here), unlike the order 9-12
    seen at dt <= 0.04 above."""
    ref, _ = _run(0.0125, 0.4, 0)
    errs = []
    for dt in (0.4, 0.2, 0.1):
        u, nits = _run(dt, 0.4, 0)
        errs.append(rel(u, ref))
        print(f"  dt {dt}: err {errs[-1]:.3e} newton/step {nits:.2f}")
    print("  observed orders", [float(np.log2(errs[k] / errs[k + 1])) for k in range(2)])
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6
