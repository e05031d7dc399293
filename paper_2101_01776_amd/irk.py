"""ctypes binding of libirk.so (include/irk.h).

Argument marshalling only: every function below forwards to the C entry point
of the same name; fields live in PyTorch device tensors (float64, contiguous)
whose data pointers are passed through, and the HIP stream is PyTorch's
current stream.  The library must have been built
(``python -m paper_2101_01776_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libirk.so")

IRK_MAX_STAGES = 5

GAUSS, RADAU_IIA, LOBATTO_IIIC, SDIRK = 0, 1, 2, 3
OP_BURGERS_1D, OP_NLDIFF_2D, OP_VSF_2D = 0, 1, 2
FORCING_NONE, FORCING_MMS, FORCING_MMS_DISCRETE = 0, 1, 2

STATUS = {0: "IRK_OK", -1: "IRK_E_ARG", -2: "IRK_E_NOMEM", -3: "IRK_E_NOCONV",
          -4: "IRK_E_NONFINITE", -5: "IRK_E_DEVICE", -6: "IRK_E_UNSUPPORTED", -7: "IRK_E_BUSY"}

FAMILY = {"gauss": GAUSS, "radau": RADAU_IIA, "lobatto": LOBATTO_IIIC, "sdirk": SDIRK}


class IrkError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


class Operator(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("length", ctypes.c_double), ("nu", ctypes.c_double), ("forcing", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("newton_rtol", ctypes.c_double), ("newton_atol", ctypes.c_double),
                ("krylov_rtol", ctypes.c_double), ("restart", ctypes.c_int),
                ("max_krylov", ctypes.c_int), ("max_newton", ctypes.c_int),
                ("newton_like", ctypes.c_int), ("gamma_mode", ctypes.c_int),
                ("prec_fp32", ctypes.c_int), ("cheb_degree", ctypes.c_int),
                ("mg_coarsest", ctypes.c_int), ("coarse_iters", ctypes.c_int), ("batch_mg", ctypes.c_int),
                ("start_extrapolate", ctypes.c_int), ("krylov_adaptive", ctypes.c_int),
                ("dae_reorder", ctypes.c_int), ("transform", ctypes.c_int),
                ("psi_solve", ctypes.c_int), ("lane_threads", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int), ("krylov_its", ctypes.c_int),
                ("krylov_its_block", ctypes.c_int * IRK_MAX_STAGES), ("vcycles", ctypes.c_int),
                ("prec_applications", ctypes.c_int), ("res0", ctypes.c_double),
                ("final_res", ctypes.c_double), ("start", ctypes.c_int), ("acceptance", ctypes.c_int),
                ("krylov_its_psi", ctypes.c_int)]

    def as_dict(self):
        return {"newton_its": self.newton_its, "krylov_its": self.krylov_its,
                "krylov_its_block": list(self.krylov_its_block), "vcycles": self.vcycles,
                "prec_applications": self.prec_applications, "res0": self.res0,
                "final_res": self.final_res, "start": self.start, "acceptance": self.acceptance,
                "krylov_its_psi": self.krylov_its_psi}


class Request(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int), ("s", ctypes.c_int), ("op", Operator), ("opt", Options),
                ("use_options", ctypes.c_int), ("t0", ctypes.c_double), ("dt", ctypes.c_double),
                ("nsteps", ctypes.c_int), ("tol", ctypes.c_double), ("u0", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("stream", ctypes.c_void_p)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("status", ctypes.c_int), ("steps_done", ctypes.c_int),
                ("newton_its", ctypes.c_int), ("krylov_its", ctypes.c_int), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


REQ_STATE = {0: "queued", 1: "running", 2: "done", 3: "failed"}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2101_01776_amd.build`")
    # PyTorch ships its own HIP runtime with the same soname; loading torch
    # first makes libirk bind to that one, so that torch's device pointers and
    # streams are valid in the library (one runtime per process).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, D, I, Z = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_size_t
    L.irk_status_str.restype = ctypes.c_char_p
    L.irk_status_str.argtypes = [I]
    L.irk_default_options.restype = None
    L.irk_default_options.argtypes = [ctypes.POINTER(Options)]
    L.irk_tableau.restype = I
    L.irk_tableau.argtypes = [I, I, P, P, P]
    L.irk_eigen_blocks.restype = I
    L.irk_eigen_blocks.argtypes = [I, I, P, P, P, P, P, P, P, P]
    L.irk_schur_blocks.restype = I
    L.irk_schur_blocks.argtypes = [I, I, P, P]
    L.irk_workspace_bytes.restype = Z
    L.irk_workspace_bytes.argtypes = [I, I, ctypes.POINTER(Operator), ctypes.POINTER(Options)]
    L.irk_create.restype = I
    L.irk_create.argtypes = [I, I, ctypes.POINTER(Operator), ctypes.POINTER(Options), P, Z, P,
                             ctypes.POINTER(P)]
    L.irk_step.restype = I
    L.irk_step.argtypes = [P, P, D, D, D, P, ctypes.POINTER(Stats)]
    L.irk_eval_residual.restype = I
    L.irk_eval_residual.argtypes = [P, P, D, D, P, P]
    L.irk_eval_residual_noalloc.restype = I
    L.irk_eval_residual_noalloc.argtypes = [I, I, ctypes.POINTER(Operator), P, D, D, P, P, P]
    L.irk_get_stages.restype = I
    L.irk_get_stages.argtypes = [P, P]
    L.irk_apply_block.restype = I
    L.irk_apply_block.argtypes = [P, I, P, P]
    L.irk_destroy.restype = None
    L.irk_destroy.argtypes = [P]
    L.irk_server_create.restype = I
    L.irk_server_create.argtypes = [P, Z, I, ctypes.POINTER(P)]
    L.irk_server_submit.restype = I
    L.irk_server_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_long)]
    L.irk_server_progress.restype = I
    L.irk_server_progress.argtypes = [P]
    L.irk_server_info.restype = I
    L.irk_server_info.argtypes = [P, ctypes.c_long, ctypes.POINTER(RequestInfo)]
    L.irk_server_stats.restype = I
    L.irk_server_stats.argtypes = [P, ctypes.POINTER(D), I, ctypes.POINTER(I), ctypes.POINTER(I),
                                   ctypes.POINTER(Z)]
    L.irk_server_destroy.restype = None
    L.irk_server_destroy.argtypes = [P]
    L.irk_profile_enable.restype = I
    L.irk_profile_enable.argtypes = [P, I]
    L.irk_profile_count.restype = I
    L.irk_profile_count.argtypes = [P]
    L.irk_profile_entry.restype = I
    L.irk_profile_entry.argtypes = [P, I, ctypes.c_char_p, I, ctypes.POINTER(ctypes.c_long),
                                    ctypes.POINTER(D), ctypes.POINTER(D)]
    L.irk_profile_replay.restype = I
    L.irk_profile_replay.argtypes = [P, ctypes.c_char_p, I, ctypes.POINTER(D), ctypes.POINTER(D)]
    _lib = L
    return L


def _check(st: int, where: str):
    if st != 0:
        raise IrkError(st, where)


# ----------------------------- host entry points -----------------------------
def irk_default_options() -> Options:
    o = Options()
    lib().irk_default_options(ctypes.byref(o))
    return o


def irk_tableau(family: str, s: int):
    A = np.zeros((s, s))
    b = np.zeros(s)
    c = np.zeros(s)
    _check(lib().irk_tableau(FAMILY[family], s, A.ctypes.data, b.ctypes.data, c.ctypes.data), "irk_tableau")
    return A, b, c


def irk_eigen_blocks(family: str, s: int) -> dict:
    T = np.zeros((s, s))
    Ti = np.zeros((s, s))
    nb = np.zeros(1, dtype=np.int32)
    width = np.zeros(IRK_MAX_STAGES, dtype=np.int32)
    eta = np.zeros(IRK_MAX_STAGES)
    beta = np.zeros(IRK_MAX_STAGES)
    gam = np.zeros(IRK_MAX_STAGES)
    first = np.zeros(IRK_MAX_STAGES, dtype=np.int32)
    _check(lib().irk_eigen_blocks(FAMILY[family], s, T.ctypes.data, Ti.ctypes.data, nb.ctypes.data,
                                  width.ctypes.data, eta.ctypes.data, beta.ctypes.data, gam.ctypes.data,
                                  first.ctypes.data), "irk_eigen_blocks")
    k = int(nb[0])
    return {"T": T, "Tinv": Ti, "nblocks": k, "width": width[:k].tolist(), "eta": eta[:k].tolist(),
            "beta": beta[:k].tolist(), "gamma_star": gam[:k].tolist(), "first_row": first[:k].tolist()}


def make_operator(kind: int, nx: int, ny: int = None, length: float = 1.0, nu: float = 0.0,
                  forcing: int = FORCING_NONE) -> Operator:
    if ny is None:
        ny = 1 if kind == OP_BURGERS_1D else nx
    return Operator(kind, nx, ny, length, nu, forcing)


def make_options(**kw) -> Options:
    o = irk_default_options()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def irk_schur_blocks(family: str, s: int):
    """(Q0, R0) of the real Schur basis of A0^{-1}."""
    Q = np.zeros((s, s))
    R = np.zeros((s, s))
    _check(lib().irk_schur_blocks(FAMILY[family], s, Q.ctypes.data, R.ctypes.data), "irk_schur_blocks")
    return Q, R


def irk_workspace_bytes(family: str, s: int, op: Operator, opt: Options = None) -> int:
    return int(lib().irk_workspace_bytes(FAMILY[family], s, ctypes.byref(op),
                                         ctypes.byref(opt) if opt is not None else None))


# ----------------------------- device entry points ---------------------------
def irk_create(family: str, s: int, op: Operator, opt: Options, workspace_ptr: int, workspace_bytes: int,
               stream_handle: int) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(lib().irk_create(FAMILY[family], s, ctypes.byref(op), ctypes.byref(opt) if opt is not None else None,
                            ctypes.c_void_p(workspace_ptr), workspace_bytes, ctypes.c_void_p(stream_handle),
                            ctypes.byref(ctx)), "irk_create")
    return ctx


def irk_step(ctx, u_ptr: int, t_n: float, dt: float, tol: float, out_ptr: int) -> Stats:
    st = Stats()
    code = lib().irk_step(ctx, ctypes.c_void_p(u_ptr), t_n, dt, tol, ctypes.c_void_p(out_ptr), ctypes.byref(st))
    if code != 0:
        err = IrkError(code, "irk_step")
        err.stats = st.as_dict()
        raise err
    return st


def irk_eval_residual(ctx, u_ptr: int, t_n: float, dt: float, K_ptr: int, F_ptr: int):
    _check(lib().irk_eval_residual(ctx, ctypes.c_void_p(u_ptr), t_n, dt, ctypes.c_void_p(K_ptr),
                                   ctypes.c_void_p(F_ptr)), "irk_eval_residual")


def irk_eval_residual_noalloc(family: str, s: int, op: Operator, u_ptr: int, t_n: float, dt: float, K_ptr: int,
                              F_ptr: int, stream: int = 0):
    """The stage residual without a context or workspace (enqueued on
    ``stream``; nothing is allocated and nothing waits)."""
    _check(lib().irk_eval_residual_noalloc(FAMILY[family], s, ctypes.byref(op), ctypes.c_void_p(u_ptr), t_n, dt,
                                           ctypes.c_void_p(K_ptr), ctypes.c_void_p(F_ptr), ctypes.c_void_p(stream)),
           "irk_eval_residual_noalloc")


def irk_get_stages(ctx, K_ptr: int):
    _check(lib().irk_get_stages(ctx, ctypes.c_void_p(K_ptr)), "irk_get_stages")


def irk_apply_block(ctx, block: int, x_ptr: int, y_ptr: int):
    _check(lib().irk_apply_block(ctx, block, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr)), "irk_apply_block")


def irk_destroy(ctx):
    lib().irk_destroy(ctx)


def irk_profile_enable(ctx, enable: bool):
    _check(lib().irk_profile_enable(ctx, 1 if enable else 0), "irk_profile_enable")


def irk_profile_read(ctx) -> list:
    """[{name, launches, ms, bytes}] per kernel symbol."""
    L = lib()
    out = []
    buf = ctypes.create_string_buffer(256)
    for i in range(L.irk_profile_count(ctx)):
        n = ctypes.c_long()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(L.irk_profile_entry(ctx, i, buf, 256, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)),
               "irk_profile_entry")
        out.append({"name": buf.value.decode(), "launches": n.value, "ms": ms.value, "bytes": by.value})
    return out


def irk_profile_replay(ctx, name: str, reps: int = 20) -> dict:
    """Average duration (ms) and algorithmic bytes of one launch of a kernel
    group, from back-to-back replays of its most recent recorded launches."""
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(lib().irk_profile_replay(ctx, name.encode(), reps, ctypes.byref(ms), ctypes.byref(by)),
           "irk_profile_replay")
    return {"ms": ms.value, "bytes": by.value}


class Solver:
    """One context: workspace and stream from PyTorch, compute in libirk.

    ``field_shape`` is (ny, nx) for scalar problems, (2, ny, nx) for the
    vorticity-streamfunction state, (nx,) for Burgers-1D."""

    def __init__(self, family: str, s: int, op: Operator, opt: Options = None, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.family, self.s, self.op = family, s, op
        self.opt = opt if opt is not None else irk_default_options()
        self.device = torch.device(device)
        nbytes = irk_workspace_bytes(family, s, op, self.opt)
        if nbytes == 0:
            raise IrkError(-1, "irk_workspace_bytes")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.workspace_bytes = nbytes
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = irk_create(family, s, op, self.opt, self._ws_ptr, nbytes, self.stream.cuda_stream)
        if op.kind == OP_BURGERS_1D:
            self.field_shape = (op.nx,)
        elif op.kind == OP_VSF_2D:
            self.field_shape = (2, op.ny, op.nx)
        else:
            self.field_shape = (op.ny, op.nx)

    def _dev(self, x):
        t = self.torch.as_tensor(x, dtype=self.torch.float64, device=self.device)
        return t.contiguous()

    def step(self, u, t_n: float, dt: float, tol: float = 0.0, out=None):
        u = self._dev(u)
        if tuple(u.shape) != self.field_shape:
            raise ValueError(f"field shape {tuple(u.shape)} != {self.field_shape}")
        if out is None:
            out = self.torch.empty_like(u)
        st = irk_step(self.ctx, u.data_ptr(), t_n, dt, tol, out.data_ptr())
        return out, st.as_dict()

    def eval_residual(self, u, t_n: float, dt: float, K):
        u = self._dev(u)
        K = self._dev(K)
        F = self.torch.empty_like(K)
        irk_eval_residual(self.ctx, u.data_ptr(), t_n, dt, K.data_ptr(), F.data_ptr())
        return F

    def apply_block(self, block: int, x):
        """D_b x for eigen-block ``block`` at the last evaluated stage values;
        x: (width,) + field shape."""
        x = self._dev(x)
        y = self.torch.empty_like(x)
        irk_apply_block(self.ctx, block, x.data_ptr(), y.data_ptr())
        return y

    def stages(self):
        K = self.torch.empty((self.s,) + self.field_shape, dtype=self.torch.float64, device=self.device)
        irk_get_stages(self.ctx, K.data_ptr())
        return K

    def close(self):
        if self.ctx is not None:
            irk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------- serving -------------------------------------
def irk_server_create(arena_ptr: int, arena_bytes: int, max_slots: int):
    srv = ctypes.c_void_p()
    _check(lib().irk_server_create(ctypes.c_void_p(arena_ptr), arena_bytes, max_slots, ctypes.byref(srv)),
           "irk_server_create")
    return srv


def irk_server_submit(srv, req: Request) -> int:
    rid = ctypes.c_long()
    _check(lib().irk_server_submit(srv, ctypes.byref(req), ctypes.byref(rid)), "irk_server_submit")
    return rid.value


def irk_server_progress(srv) -> int:
    return int(lib().irk_server_progress(srv))


def irk_server_info(srv, rid: int) -> dict:
    info = RequestInfo()
    _check(lib().irk_server_info(srv, rid, ctypes.byref(info)), "irk_server_info")
    return {"state": REQ_STATE[info.state], "status": STATUS.get(info.status, info.status),
            "steps_done": info.steps_done, "newton_its": info.newton_its, "krylov_its": info.krylov_its,
            "t_submit": info.t_submit, "t_admit": info.t_admit, "t_done": info.t_done}


def irk_server_stats(srv) -> dict:
    L = lib()
    n = ctypes.c_int()
    peak = ctypes.c_int()
    pb = ctypes.c_size_t()
    _check(L.irk_server_stats(srv, None, 0, ctypes.byref(n), ctypes.byref(peak), ctypes.byref(pb)),
           "irk_server_stats")
    buf = (ctypes.c_double * max(1, n.value))()
    _check(L.irk_server_stats(srv, buf, n.value, ctypes.byref(n), ctypes.byref(peak), ctypes.byref(pb)),
           "irk_server_stats")
    return {"step_ms": list(buf)[: n.value], "peak_running": peak.value, "peak_bytes": pb.value}


def irk_server_destroy(srv):
    lib().irk_server_destroy(srv)


class Server:
    """A serving loop on a PyTorch-allocated device arena (the HBM budget)."""

    def __init__(self, arena_bytes: int, max_slots: int, device: str = "cuda:0", arena=None):
        """``arena``: an existing uint8 device tensor of at least
        ``arena_bytes + 256`` bytes to serve from (reused across servers);
        by default one is allocated."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        lib()
        if arena is None:
            arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=self.device)
        elif arena.dtype != torch.uint8 or arena.numel() < arena_bytes + 256 or arena.device != self.device:
            raise ValueError("arena must be a uint8 tensor of at least arena_bytes + 256 bytes on the device")
        self._arena = arena
        ptr = (self._arena.data_ptr() + 255) & ~255
        self.srv = irk_server_create(ptr, arena_bytes, max_slots)
        self._keep = {}

    def submit(self, family: str, s: int, op: Operator, u0, dt: float, nsteps: int, t0: float = 0.0,
               opt: Options = None, tol: float = 0.0, out=None) -> int:
        torch = self.torch
        u0 = torch.as_tensor(u0, dtype=torch.float64, device=self.device).contiguous()
        if out is None:
            out = torch.empty_like(u0)
        req = Request()
        req.family = FAMILY[family]
        req.s = s
        req.op = op
        if opt is not None:
            req.opt = opt
            req.use_options = 1
        req.t0, req.dt, req.nsteps, req.tol = t0, dt, nsteps, tol
        req.u0 = u0.data_ptr()
        req.out = out.data_ptr()
        req.stream = torch.cuda.current_stream(self.device).cuda_stream
        rid = irk_server_submit(self.srv, req)
        self._keep[rid] = (u0, out)
        return rid

    def progress(self) -> int:
        return irk_server_progress(self.srv)

    def run_until_idle(self):
        while self.progress() > 0:
            pass

    def info(self, rid: int) -> dict:
        return irk_server_info(self.srv, rid)

    def result(self, rid: int):
        return self._keep[rid][1]

    def stats(self) -> dict:
        return irk_server_stats(self.srv)

    def close(self):
        if self.srv is not None:
            irk_server_destroy(self.srv)
            self.srv = None
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
