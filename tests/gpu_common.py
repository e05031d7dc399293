"""Shared helpers of the GPU tests: map a C-ABI operator to the oracle's
problem, seeded inputs, relative errors."""
import numpy as np
import pytest

from oracle import newton as nw
from oracle import problems as pb
from oracle import tableau as tb
from paper_2101_01776_amd import inputs, irk

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    HAVE_GPU = False

gpu = [pytest.mark.gpu, pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")]

FORCING_NAME = {irk.FORCING_NONE: "none", irk.FORCING_MMS: "continuous",
                irk.FORCING_MMS_DISCRETE: "discrete"}


def oracle_problem(op):
    if op.kind == irk.OP_NLDIFF_2D:
        return pb.NonlinearDiffusion2D(op.nx, forcing=FORCING_NAME[op.forcing], length=op.length)
    if op.kind == irk.OP_BURGERS_1D:
        return pb.Burgers1D(op.nx, op.nu, length=op.length)
    return pb.VorticityStreamfunction2D(op.nx, op.nu, length=op.length)


def initial_field(op, seed=0):
    if op.kind == irk.OP_NLDIFF_2D:
        return inputs.nldiff_u0(op.nx) if seed == 0 else inputs.nldiff_random_u0(op.nx, seed)
    if op.kind == irk.OP_BURGERS_1D:
        return inputs.burgers_u0(op.nx, seed)
    return inputs.vsf_state0(op.nx, seed, n_vortices=8)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_step(op, family, s, u, t, dt):
    A, b, c = tb.tableau(family, s)
    u1, K, info = nw.irk_step(oracle_problem(op), A, b, c, np.asarray(u, dtype=np.float64).ravel(), t, dt)
    return u1, K, info


def oracle_residual(op, family, s, u, t, dt, K):
    A, _, c = tb.tableau(family, s)
    Kf = np.asarray(K, dtype=np.float64).reshape(s, -1)
    return nw.stage_residual(oracle_problem(op), A, c, np.asarray(u, dtype=np.float64).ravel(), t, dt, Kf)
