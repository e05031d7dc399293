"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and its host-only logic (tableaux, eigenbasis of A0^{-1},
options, workspace sizing, argument validation) agrees with the oracle and
the paper."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from oracle import tableau as tb
from paper_2101_01776_amd import irk

HEADER = os.path.join(ROOT, "include", "irk.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(irk_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = irk.lib()
    names = _declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_lobatto_needs_two_stages():
    import ctypes
    A = (ctypes.c_double * 1)()
    b = (ctypes.c_double * 1)()
    c = (ctypes.c_double * 1)()
    assert irk.lib().irk_tableau(irk.LOBATTO_IIIC, 1, A, b, c) == -1
    assert irk.irk_workspace_bytes("lobatto", 1, irk.make_operator(irk.OP_NLDIFF_2D, 32)) == 0


@pytest.mark.parametrize("s", [1, 2, 3, 5])
def test_host_sdirk_tableau_matches_oracle(s):
    A, b, c = irk.irk_tableau("sdirk", s)
    Ao, bo, co = tb.tableau("sdirk", s)
    assert np.max(np.abs(np.asarray(A) - Ao)) < 2e-16 * max(1.0, np.abs(Ao).max())
    assert np.max(np.abs(np.asarray(b) - bo)) < 2e-16 * max(1.0, np.abs(bo).max())
    assert np.max(np.abs(np.asarray(c) - co)) < 2e-16


def test_sdirk_shapes_and_unsupported_calls():
    op = irk.make_operator(irk.OP_NLDIFF_2D, 64)
    assert irk.irk_workspace_bytes("sdirk", 4, op) == 0          # no 4-stage method provided
    assert irk.irk_workspace_bytes("sdirk", 5, op) > irk.irk_workspace_bytes("sdirk", 1, op)
    with pytest.raises(irk.IrkError):
        irk.irk_eigen_blocks("sdirk", 2)


def test_status_strings_and_defaults():
    L = irk.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.irk_status_str(code)
    o = irk.irk_default_options()
    assert o.newton_rtol == 1e-12 and o.krylov_rtol == 1e-5 and o.restart == 30
    assert o.prec_fp32 == 1 and o.cheb_degree == 3 and o.newton_like == 1 and o.gamma_mode == 0
    assert o.batch_mg == 0 and o.start_extrapolate == 1 and o.krylov_adaptive == 1 and o.dae_reorder == 0


def test_struct_layouts_match_the_header():
    """The binding's structures have the header's size: irk_default_options
    writes exactly sizeof(Options) bytes (a guard region after it stays
    untouched) and its last field lands where the binding expects it."""
    import ctypes
    n = ctypes.sizeof(irk.Options)
    buf = (ctypes.c_ubyte * (n + 64))(*([0xAB] * (n + 64)))
    irk.lib().irk_default_options(ctypes.cast(buf, ctypes.POINTER(irk.Options)))
    assert bytes(buf[n:]) == b"\xab" * 64
    o = irk.Options.from_buffer_copy(bytes(buf[:n]))
    assert o.krylov_adaptive == 1 and o.dae_reorder == 0 and o.coarse_iters == 24


@pytest.mark.parametrize("family,s", [(f, s) for f in ("gauss", "radau", "lobatto") for s in (1, 2, 3, 4, 5)
                                      if not (f == "lobatto" and s == 1)])
def test_host_tableau_matches_oracle(family, s):
    A, b, c = irk.irk_tableau(family, s)
    A2, b2, c2 = tb.tableau(family, s)
    assert np.max(np.abs(A - A2)) <= 1e-16 and np.max(np.abs(b - b2)) <= 1e-16
    assert np.max(np.abs(c - c2)) <= 1e-16


@pytest.mark.parametrize("family,s", [(f, s) for f in ("gauss", "radau", "lobatto") for s in (1, 2, 3, 4, 5)
                                      if not (f == "lobatto" and s == 1)])
def test_host_eigenbasis(family, s):
    """A0^{-1} = T Lambda T^{-1} with Lambda in the real block form, eigenvalues
    and gamma_* equal to the oracle's."""
    e = irk.irk_eigen_blocks(family, s)
    A2, _, _ = tb.tableau(family, s)
    Ainv = np.linalg.inv(A2)
    Lam = np.zeros((s, s))
    for k in range(e["nblocks"]):
        r = e["first_row"][k]
        Lam[r, r] = e["eta"][k]
        if e["width"][k] == 2:
            Lam[r, r + 1] = e["beta"][k]
            Lam[r + 1, r] = -e["beta"][k]
            Lam[r + 1, r + 1] = e["eta"][k]
    assert np.max(np.abs(e["T"] @ Lam @ e["Tinv"] - Ainv)) <= 1e-14 * np.abs(Ainv).max()
    assert np.max(np.abs(e["T"] @ e["Tinv"] - np.eye(s))) <= 1e-14
    want = tb.inverse_eigs(A2)
    got = list(zip(e["eta"], e["beta"]))
    assert len(got) == len(want)
    for (ge, gb), (we, wb) in zip(got, want):
        assert abs(ge - we) < 1e-12 * we and abs(gb - wb) < 1e-12 * max(1.0, wb)
    for k in range(e["nblocks"]):
        assert abs(e["gamma_star"][k] - tb.gamma_star(e["eta"][k], e["beta"][k])) < 1e-13 * e["gamma_star"][k]
    # columns of a pair: Re v orthogonal to Im v
    for k in range(e["nblocks"]):
        if e["width"][k] == 2:
            r = e["first_row"][k]
            assert abs(e["T"][:, r] @ e["T"][:, r + 1]) < 1e-14


def test_workspace_sizing_and_validation():
    op = irk.make_operator(irk.OP_NLDIFF_2D, 512, forcing=irk.FORCING_MMS)
    n = irk.irk_workspace_bytes("gauss", 3, op)
    # at least K, Y, Fh, U (4 s fields) and the Krylov bases V (31 vectors of 2
    # fields) and Z (30 vectors of 2 fields)
    assert n >= (4 * 3 + 31 * 2 + 30 * 2) * 512 * 512 * 8
    fp64 = irk.irk_workspace_bytes("gauss", 3, op, irk.make_options(prec_fp32=0))
    assert fp64 > n
    bad = [irk.make_operator(irk.OP_NLDIFF_2D, 512, 256),            # nx != ny
           irk.make_operator(irk.OP_BURGERS_1D, 256, 2),             # 1-D with ny > 1
           irk.make_operator(7, 64)]                                 # unknown kind
    for b in bad:
        assert irk.irk_workspace_bytes("gauss", 3, b) == 0
    assert irk.irk_workspace_bytes("gauss", 6, op) == 0              # s > 5
    assert irk.irk_workspace_bytes("gauss", 3, op, irk.make_options(restart=0)) == 0
    # a coarsest level larger than one work-group can hold is refused
    assert irk.irk_workspace_bytes("gauss", 3, irk.make_operator(irk.OP_NLDIFF_2D, 66)) == 0


def test_create_rejects_bad_workspace_without_gpu_work():
    op = irk.make_operator(irk.OP_NLDIFF_2D, 32)
    ctx = ctypes.c_void_p()
    L = irk.lib()
    st = L.irk_create(irk.GAUSS, 3, ctypes.byref(op), None, None, 0, None, ctypes.byref(ctx))
    assert st == -1 and not ctx.value
    st = L.irk_create(irk.GAUSS, 3, ctypes.byref(op), None, ctypes.c_void_p(256), 16, None, ctypes.byref(ctx))
    assert st == -2 and not ctx.value
    L.irk_destroy(None)


def test_server_create_without_a_device_fails_cleanly():
    """A server makes every slot's streams, events and pinned staging when it
    is created; without a GPU that fails with IRK_E_DEVICE (and releases
    what it made) instead of deferring the failure to an admission."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible: the server would be created")
    except ImportError:  # pragma: no cover
        pass
    with pytest.raises(irk.IrkError) as e:
        irk.irk_server_create(256, 1 << 20, 2)
    assert e.value.status == -5


@pytest.mark.parametrize("family,s", [(f, s) for f in ("gauss", "radau", "lobatto") for s in (2, 3, 4, 5)])
def test_host_schur_basis(family, s):
    """Real Schur basis of A0^{-1} (Section 3.1): Q0 orthogonal, Q0^T A0^{-1} Q0
    = R0 block upper triangular with the eigenvalues of the eigen-blocks on
    its diagonal blocks, each 2x2 block standardized (equal diagonal entries,
    |phi| <= beta)."""
    Q, R = irk.irk_schur_blocks(family, s)
    A, _, _ = tb.tableau(family, s)
    Ainv = np.linalg.inv(A)
    assert np.abs(Q.T @ Q - np.eye(s)).max() < 1e-14
    assert np.abs(Q.T @ Ainv @ Q - R).max() < 1e-12 * np.abs(Ainv).max()
    e = irk.irk_eigen_blocks(family, s)
    for k in range(e["nblocks"]):
        r, w = e["first_row"][k], e["width"][k]
        assert np.all(R[r:r + w, :r] == 0.0)                 # nothing left of the block
        if w == 1:
            assert abs(R[r, r] - e["eta"][k]) < 1e-12 * e["eta"][k]
        else:
            blk = R[r:r + 2, r:r + 2]
            assert abs(blk[0, 0] - blk[1, 1]) < 1e-12 * abs(blk[0, 0])
            assert abs(blk[0, 0] - e["eta"][k]) < 1e-12 * e["eta"][k]
            assert abs(-blk[0, 1] * blk[1, 0] - e["beta"][k] ** 2) < 1e-11 * e["beta"][k] ** 2
            assert abs(blk[0, 1]) <= e["beta"][k] * (1 + 1e-12)


@pytest.mark.parametrize("family", ["gauss", "radau"])
def test_host_schur_basis_reproduces_worked_example(family):
    """The d weights d_kl,i = (Q0^T)_ki (Q0)_il of equation (Q0approx) in the
    host's Schur basis against the worked example printed for the two-stage
    methods (equation (Gauss4Radau3_example)): diagonal entries, and the
    magnitudes of the off-diagonal ones (their sign follows the sign chosen for
    each Schur vector)."""
    from conftest import read_golden
    Q, _ = irk.irk_schur_blocks(family, 2)
    rows = [r for r in read_golden("worked_example_d.txt") if r[0] == family]
    assert len(rows) == 4
    for _, _, k, l, d1, d2 in rows:
        k, l = int(k) - 1, int(l) - 1
        d = [Q[i, k] * Q[i, l] for i in range(2)]
        want = [float(d1), float(d2)]
        if k == l:
            assert np.allclose(d, want, atol=6e-4)
        else:
            assert np.allclose(np.abs(d), np.abs(want), atol=6e-4)


def test_schur_basis_option_scope():
    """transform = 1 runs on the ODE operators; the DAE and SDIRK refuse it."""
    opt = irk.make_options(transform=1)
    nl = irk.make_operator(irk.OP_NLDIFF_2D, 64, forcing=irk.FORCING_MMS)
    assert irk.irk_workspace_bytes("gauss", 3, nl, opt) > 0
    assert irk.irk_workspace_bytes("gauss", 3, irk.make_operator(irk.OP_VSF_2D, 64, nu=1e-3), opt) == 0
    assert irk.irk_workspace_bytes("sdirk", 2, nl, opt) == 0
    assert irk.irk_workspace_bytes("gauss", 3, nl, irk.make_options(transform=2)) == 0


def test_streamfunction_solve_option():
    """psi_solve: 0 (default) the spectral solve on power-of-two grids, 1 the
    Poisson V-cycle; other values are refused.  The spectral solve keeps a
    half spectrum per lane in the workspace, so the sizes differ exactly
    where it applies."""
    assert irk.irk_default_options().psi_solve == 0
    sizes = {}
    for n in (64, 48):
        vsf = irk.make_operator(irk.OP_VSF_2D, n, nu=1e-3)
        assert irk.irk_workspace_bytes("radau", 3, vsf, irk.make_options(psi_solve=2)) == 0
        sizes[n] = [irk.irk_workspace_bytes("radau", 3, vsf, irk.make_options(psi_solve=p)) for p in (0, 1)]
    assert sizes[64][0] != sizes[64][1] and sizes[48][0] == sizes[48][1]
    # float64 V-cycles: sides up to 1024 (2048 needs more than 64 KiB of LDS per row work-group)
    big = irk.make_operator(irk.OP_VSF_2D, 2048, nu=1e-3)
    f32 = irk.irk_workspace_bytes("radau", 3, big, irk.make_options(psi_solve=0))
    f32_mg = irk.irk_workspace_bytes("radau", 3, big, irk.make_options(psi_solve=1))
    f64 = irk.irk_workspace_bytes("radau", 3, big, irk.make_options(psi_solve=0, prec_fp32=0))
    f64_mg = irk.irk_workspace_bytes("radau", 3, big, irk.make_options(psi_solve=1, prec_fp32=0))
    assert f32 != f32_mg and f64 == f64_mg


def test_lane_threads_option():
    """lane_threads: 1 (default) a host thread per eigen-block solve, 0 the
    calling thread only; other values are refused.  It needs no device
    memory of its own."""
    assert irk.irk_default_options().lane_threads == 1
    nl = irk.make_operator(irk.OP_NLDIFF_2D, 64)
    assert irk.irk_workspace_bytes("gauss", 5, nl, irk.make_options(lane_threads=2)) == 0
    sizes = [irk.irk_workspace_bytes("gauss", 5, nl, irk.make_options(lane_threads=t)) for t in (0, 1)]
    assert sizes[0] == sizes[1] > 0
