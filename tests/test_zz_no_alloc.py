"""The no-allocation entry point (irk_eval_residual_noalloc) against the
context entry point it varies (irk_eval_residual): the same stage residual
on the same seeded inputs, called twice in a row on one GPU, the second call
smaller than the first (the shared scratch keeps the first call's contents,
so a value read before it is written would show)."""
import numpy as np
import pytest

from gpu_common import gpu, initial_field, rel
from paper_2101_01776_amd import irk

CALLS = [
    # (name, operator, family, s): each pair runs large first, then small
    ("nldiff-mms", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 96, forcing=irk.FORCING_MMS), "gauss", 3),
    ("nldiff-discrete-small", lambda: irk.make_operator(irk.OP_NLDIFF_2D, 40, forcing=irk.FORCING_MMS_DISCRETE),
     "radau", 2),
    ("vsf", lambda: irk.make_operator(irk.OP_VSF_2D, 64, nu=1e-3), "radau", 3),
    ("vsf-ragged-small", lambda: irk.make_operator(irk.OP_VSF_2D, 30, nu=1e-3), "gauss", 2),
    ("burgers", lambda: irk.make_operator(irk.OP_BURGERS_1D, 256, nu=0.01), "gauss", 5),
    ("burgers-small", lambda: irk.make_operator(irk.OP_BURGERS_1D, 250, nu=0.01), "lobatto", 3),
]


def _noalloc(torch, family, s, op, u, t, dt, K):
    F = torch.empty_like(K)
    stream = torch.cuda.current_stream()
    irk.irk_eval_residual_noalloc(family, s, op, u.data_ptr(), t, dt, K.data_ptr(), F.data_ptr(),
                                  stream.cuda_stream)
    torch.cuda.synchronize()
    return F


@pytest.mark.gpu
@pytest.mark.parametrize("first,second", [(0, 1), (2, 3), (4, 5)], ids=["nldiff", "vsf", "burgers"])
def test_noalloc_residual_matches_context_entry(first, second):
    import torch
    assert torch.cuda.is_available()
    for idx in (first, second):
        name, mk, family, s = CALLS[idx]
        op = mk()
        print(f"[noalloc] {name} n={op.nx} {family}{s}", flush=True)
        solver = irk.Solver(family, s, op, irk.make_options(prec_fp32=0))
        u0 = initial_field(op, 5)
        rng = np.random.default_rng(17 + idx)
        K = rng.standard_normal((s,) + solver.field_shape)
        t, dt = 0.21, 3e-3
        want = solver.eval_residual(u0, t, dt, K).cpu().numpy()
        u = torch.tensor(u0, dtype=torch.float64, device="cuda")
        Kd = torch.tensor(K, dtype=torch.float64, device="cuda")
        got = _noalloc(torch, family, s, op, u, t, dt, Kd).cpu().numpy()
        err = rel(got, want)
        print(f"  rel diff {err:.3e}", flush=True)
        assert err < 1e-13, (name, err)
        solver.close()


def test_noalloc_refuses_oversized_problems_before_any_device_call():
    """s * field beyond the fixed scratch: IRK_E_NOMEM, checked on the host
    (no device memory is touched, so this runs without a GPU)."""
    op = irk.make_operator(irk.OP_VSF_2D, 1024, nu=1e-3)
    with pytest.raises(irk.IrkError) as e:
        irk.irk_eval_residual_noalloc("radau", 4, op, 8, 0.0, 1e-3, 8, 8)
    assert e.value.status == -2
    op = irk.make_operator(irk.OP_NLDIFF_2D, 1024, forcing=irk.FORCING_MMS)
    with pytest.raises(irk.IrkError) as e:
        irk.irk_eval_residual_noalloc("gauss", 5, op, 0, 0.0, 1e-3, 8, 8)
    assert e.value.status == -1          # null u_n
    with pytest.raises(irk.IrkError) as e:
        irk.irk_eval_residual_noalloc("sdirk", 2, op, 8, 0.0, 1e-3, 8, 8)
    assert e.value.status == -6
