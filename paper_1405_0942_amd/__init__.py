"""MI355X (gfx950) Lagrangian mimetic magneto-frictional relaxation.

A thin ctypes binding of librelax.so (include/relax.h).  It only marshals arguments:
every step of the relaxation runs in the library's HIP kernels.  PyTorch supplies device
memory (the caller-owned workspace and the field tensors) and the HIP stream.

Low level: the C functions under their own names (relax_init, relax_step, ...).
High level: :class:`Relaxation`, which owns a workspace tensor and a context.

There is no CPU fallback: if librelax.so is missing or cannot be loaded, using the
library raises :class:`RelaxUnavailable`.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RELAX_LIB", os.path.join(HERE, "librelax.so"))

RELAX_OK, RELAX_E_ARG, RELAX_E_HIP, RELAX_E_FOLD, RELAX_E_DT, RELAX_E_NAN, RELAX_E_STATE, RELAX_E_SPACE = (
    0, -1, -2, -3, -4, -5, -6, -7)
RELAX_LINE_TIED, RELAX_PERIODIC = 0, 1
RELAX_FP64, RELAX_FP32_MIXED = 0, 1
RELAX_CURL_NN, RELAX_CURL_NNN = 0, 1

# every symbol include/relax.h declares
EXPORTS = ("relax_workspace_bytes", "relax_init", "relax_step", "relax_diagnostics", "relax_diagnostics_noalloc",
           "relax_velocity", "relax_fields", "relax_monitors", "relax_backward",
           "relax_get_state", "relax_set_state", "relax_profile", "relax_stream_probe",
           "relax_strerror",
           "relax_last_error",
           "relax_destroy")


class RelaxUnavailable(RuntimeError):
    """librelax.so could not be loaded (not built, or no HIP runtime)."""


class RelaxError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        msg = f"{where}: {relax_strerror(code)} ({code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)
        self.code = code


class relax_config(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("h", C.c_double * 3), ("bc", C.c_int * 3), ("precision", C.c_int),
                ("gamma", C.c_double), ("dt0", C.c_double), ("dt_min", C.c_double), ("tol", C.c_double),
                ("adaptive", C.c_int), ("record", C.c_int), ("checkpoint_every", C.c_int),
                ("xi_null_tau", C.c_double), ("safety", C.c_double), ("curl", C.c_int)]


class relax_diag(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("E_M", C.c_double), ("xi", C.c_double),
                ("R2", C.c_double), ("Lambda", C.c_double), ("min_det", C.c_double), ("rejects", C.c_int),
                ("concave", C.c_int)]


_lib = None


def lib():
    """The loaded librelax.so (raises RelaxUnavailable if it cannot be loaded)."""
    global _lib
    if _lib is None:
        _lib = _load(LIB_PATH)
    return _lib


@contextlib.contextmanager
def using_library(path: str):
    """Route every call of this binding to another build of the library (the tests' 64 x 4
    tile build) inside the block."""
    global _lib
    saved = lib()
    _lib = _load(path)
    try:
        yield _lib
    finally:
        _lib = saved


def _load(path: str):
    if not os.path.exists(path):
        raise RelaxUnavailable(f"{path} is not built (run python -m paper_1405_0942_amd.build)")
    try:
        L = C.CDLL(path)
    except OSError as e:  # pragma: no cover - depends on the machine
        raise RelaxUnavailable(f"cannot load {path}: {e}") from e
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    L.relax_workspace_bytes.argtypes = [C.POINTER(relax_config), C.c_int]
    L.relax_workspace_bytes.restype = C.c_size_t
    L.relax_init.argtypes = [C.POINTER(relax_config), C.c_int, vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.relax_step.argtypes = [vp, C.c_int, C.POINTER(relax_diag), C.POINTER(C.c_int)]
    L.relax_diagnostics.argtypes = [vp, C.POINTER(relax_diag)]
    L.relax_diagnostics_noalloc.argtypes = [C.POINTER(relax_config), vp, vp, vp, C.POINTER(relax_diag)]
    L.relax_velocity.argtypes = [vp, vp]
    L.relax_fields.argtypes = [vp, vp, vp]
    L.relax_monitors.argtypes = [vp, vp, vp]
    L.relax_backward.argtypes = [vp, C.c_double, C.c_double, vp, vp]
    L.relax_get_state.argtypes = [vp, vp, dp, dp]
    L.relax_set_state.argtypes = [vp, vp, C.c_double, C.c_double]
    L.relax_profile.argtypes = [vp, C.c_int, dp, C.POINTER(C.c_longlong)]
    L.relax_profile.restype = C.c_int
    L.relax_stream_probe.argtypes = [C.c_int, vp, vp, C.c_longlong, C.c_int, vp, dp]
    L.relax_stream_probe.restype = C.c_int
    L.relax_strerror.argtypes = [C.c_int]
    L.relax_strerror.restype = C.c_char_p
    L.relax_last_error.argtypes = [vp]
    L.relax_last_error.restype = C.c_char_p
    L.relax_destroy.argtypes = [vp]
    L.relax_destroy.restype = None
    for name in ("relax_init", "relax_step", "relax_diagnostics", "relax_diagnostics_noalloc", "relax_velocity",
                 "relax_fields", "relax_monitors", "relax_backward", "relax_get_state",
                 "relax_set_state"):
        getattr(L, name).restype = C.c_int
    return L


# ---- the C functions, same names ------------------------------------------------------------

def relax_workspace_bytes(cfg: relax_config, K_record: int = 0) -> int:
    return int(lib().relax_workspace_bytes(C.byref(cfg), int(K_record)))


def relax_init(cfg, K_record, d_x0, d_B0, d_workspace, workspace_bytes, hip_stream):
    ctx = C.c_void_p()
    rc = lib().relax_init(C.byref(cfg), int(K_record), C.c_void_p(d_x0), C.c_void_p(d_B0),
                          C.c_void_p(d_workspace), C.c_size_t(workspace_bytes), C.c_void_p(hip_stream),
                          C.byref(ctx))
    return rc, ctx


def relax_step(ctx, K, host_diag=None):
    done = C.c_int(0)
    rc = lib().relax_step(ctx, int(K), host_diag, C.byref(done))
    return rc, done.value


def relax_diagnostics(ctx):
    d = relax_diag()
    rc = lib().relax_diagnostics(ctx, C.byref(d))
    return rc, d


def relax_diagnostics_noalloc(cfg, d_x, d_B0, stream):
    d = relax_diag()
    rc = lib().relax_diagnostics_noalloc(C.byref(cfg), d_x, d_B0, stream, C.byref(d))
    return rc, d


def relax_velocity(ctx, d_u_out):
    return lib().relax_velocity(ctx, C.c_void_p(d_u_out))


def relax_fields(ctx, d_B_out, d_J_out):
    return lib().relax_fields(ctx, C.c_void_p(d_B_out), C.c_void_p(d_J_out))


def relax_monitors(ctx, d_alpha_out, d_kappa_out):
    return lib().relax_monitors(ctx, C.c_void_p(d_alpha_out), C.c_void_p(d_kappa_out))


def relax_backward(ctx, seed_EM, seed_R2, d_grad_x0, d_grad_B0):
    return lib().relax_backward(ctx, float(seed_EM), float(seed_R2), C.c_void_p(d_grad_x0), C.c_void_p(d_grad_B0))


def relax_get_state(ctx, d_x_out=None):
    t, dt = C.c_double(0.0), C.c_double(0.0)
    rc = lib().relax_get_state(ctx, None if d_x_out is None else C.c_void_p(d_x_out), C.byref(t), C.byref(dt))
    return rc, t.value, dt.value


def relax_set_state(ctx, d_x_in, t, dt):
    return lib().relax_set_state(ctx, C.c_void_p(d_x_in), float(t), float(dt))


def relax_profile(ctx, on):
    """Switch per-kernel timing on/off; returns (rc, ms[7], launches[7]) accumulated so far."""
    ms = (C.c_double * 7)()
    n = (C.c_longlong * 7)()
    rc = lib().relax_profile(ctx, int(on), ms, n)
    return rc, list(ms), list(n)


def relax_stream_probe(kind, d_in, d_out, n, reps, hip_stream):
    """Streaming reference kernel (measurement aid); returns (rc, mean ms of one run)."""
    ms = C.c_double(0.0)
    rc = lib().relax_stream_probe(int(kind), C.c_void_p(d_in), C.c_void_p(d_out), int(n), int(reps),
                                  C.c_void_p(hip_stream), C.byref(ms))
    return rc, ms.value


def relax_strerror(code: int) -> str:
    try:
        return lib().relax_strerror(int(code)).decode()
    except RelaxUnavailable:
        return f"status {code}"


def relax_last_error(ctx) -> str:
    return lib().relax_last_error(ctx).decode()


def relax_destroy(ctx) -> None:
    lib().relax_destroy(ctx)


# ---- high level --------------------------------------------------------------------------------

DIAG_FIELDS = ("t", "dt", "E_M", "xi", "R2", "Lambda", "min_det", "rejects", "concave")


def make_config(grid, precision=RELAX_FP64, gamma=1.0, dt0=1e-3, dt_min=1e-12, tol=1e-7, adaptive=True,
                record=False, checkpoint_every=20, xi_null_tau=1e-12, safety=1.0, curl=RELAX_CURL_NN) -> relax_config:
    """Build a relax_config from any grid with attributes n, h, bc."""
    c = relax_config()
    c.n[:] = [int(v) for v in grid.n]
    c.h[:] = [float(v) for v in grid.h]
    c.bc[:] = [int(v) for v in grid.bc]
    c.precision = int(precision)
    c.gamma = float(gamma)
    c.dt0 = float(dt0)
    c.dt_min = float(dt_min)
    c.tol = float(tol)
    c.adaptive = 1 if adaptive else 0
    c.record = 1 if record else 0
    c.checkpoint_every = int(checkpoint_every)
    c.xi_null_tau = float(xi_null_tau)
    c.safety = float(safety)
    c.curl = int(curl)
    return c


class Relaxation:
    """One relaxation context on the current CUDA/HIP device and stream.

    x0, B0: torch float64 device tensors of shape (3, nz, ny, nx) (copied at init).
    """

    def __init__(self, cfg: relax_config, x0, B0, K_record: int = 0, stream=None):
        import torch

        self.cfg = cfg
        self.K_record = int(K_record)
        shape = (3, cfg.n[2], cfg.n[1], cfg.n[0])
        for name, t in (("x0", x0), ("B0", B0)):
            if tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {shape}")
        nbytes = relax_workspace_bytes(cfg, self.K_record)
        if nbytes == 0:
            raise RelaxError(RELAX_E_ARG, "relax_workspace_bytes", "invalid configuration")
        self.device = x0.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._ws_bytes = nbytes
        rc, ctx = relax_init(cfg, self.K_record, x0.data_ptr(), B0.data_ptr(), self._ws_ptr, nbytes,
                             self.stream.cuda_stream)
        if rc != RELAX_OK:
            raise RelaxError(rc, "relax_init")
        self.ctx = ctx
        self.shape = shape

    def _check(self, rc, where):
        if rc != RELAX_OK:
            raise RelaxError(rc, where, relax_last_error(self.ctx))

    def step(self, K: int, diag: bool = True, raise_on_error: bool = True):
        """K accepted steps. Returns a list of per-step dicts (pre-step diagnostics)."""
        buf = (relax_diag * max(int(K), 1))() if diag else None
        rc, done = relax_step(self.ctx, K, buf)
        out = [{f: getattr(buf[i], f) for f in DIAG_FIELDS} for i in range(done)] if diag else []
        if raise_on_error:
            self._check(rc, "relax_step")
        self.last_status = rc
        self.last_done = done
        return out

    def diagnostics(self) -> dict:
        rc, d = relax_diagnostics(self.ctx)
        self._check(rc, "relax_diagnostics")
        return {f: getattr(d, f) for f in DIAG_FIELDS}

    def velocity(self):
        """u(x) of the current positions (FP64), as a new device tensor."""
        import torch
        u = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._check(relax_velocity(self.ctx, u.data_ptr()), "relax_velocity")
        return u

    def fields(self):
        """(B, J) of the current positions (FP64; J is zero on line-tied faces), as new device
        tensors."""
        import torch
        B = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        J = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._check(relax_fields(self.ctx, B.data_ptr(), J.data_ptr()), "relax_fields")
        return B, J

    def monitors(self):
        """(alpha*, kappa) of the current positions as new device tensors of shape (nz, ny, nx):
        alpha* = J.B / B^2 (FP64) and the node convexity +1 / -1 (int32)."""
        import torch
        alpha = torch.empty(self.shape[1:], dtype=torch.float64, device=self.device)
        kappa = torch.empty(self.shape[1:], dtype=torch.int32, device=self.device)
        self._check(relax_monitors(self.ctx, alpha.data_ptr(), kappa.data_ptr()), "relax_monitors")
        return alpha, kappa

    def state(self):
        """(x as a new device tensor, t, dt)"""
        import torch
        x = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        rc, t, dt = relax_get_state(self.ctx, x.data_ptr())
        self._check(rc, "relax_get_state")
        return x, t, dt

    def set_state(self, x, t, dt):
        self._check(relax_set_state(self.ctx, x.data_ptr(), t, dt), "relax_set_state")

    def backward(self, seed_EM=1.0, seed_R2=0.0):
        """(dL/dx0, dL/dB0) for L = seed_EM E_M(x_K) + seed_R2 R2(x_K)."""
        import torch
        gx = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        gb = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._check(relax_backward(self.ctx, seed_EM, seed_R2, gx.data_ptr(), gb.data_ptr()), "relax_backward")
        return gx, gb

    def profile(self, on: bool):
        """Switch kernel timing on/off; returns {kernel: (total ms, launches)} accumulated so far."""
        rc, ms, n = relax_profile(self.ctx, 1 if on else 0)
        self._check(rc, "relax_profile")
        names = [f"stage{s}" for s in range(1, 7)] + ["control"]
        return {k: (ms[i], n[i]) for i, k in enumerate(names)}

    def close(self):
        if getattr(self, "ctx", None):
            relax_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _relax_function():
    import torch

    class RelaxK(torch.autograd.Function):
        """(E_M(x_K), R2(x_K)) after K fixed-dt steps from (x0, B0); backward through the
        library's reverse-mode sweeps (checkpointed every cfg.checkpoint_every steps).

        Gradients flow to x0 and B0 only (cfg must have record = 1 and adaptive = 0 for an
        exact gradient; with adaptive = 1 the recorded dt sequence is held fixed)."""

        @staticmethod
        def forward(ctx, x0, B0, cfg, K):
            r = Relaxation(cfg, x0.detach().contiguous(), B0.detach().contiguous(), K_record=K)
            if K > 0:
                r.step(K, diag=False)
            d = r.diagnostics()
            ctx.relax = r
            dev = x0.device
            return (torch.tensor(d["E_M"], dtype=torch.float64, device=dev),
                    torch.tensor(d["R2"], dtype=torch.float64, device=dev))

        @staticmethod
        def backward(ctx, gE, gR):
            r = ctx.relax
            sE = 0.0 if gE is None else float(gE)
            sR = 0.0 if gR is None else float(gR)
            gx, gb = r.backward(sE, sR)
            r.close()
            ctx.relax = None
            return gx, gb, None, None

    return RelaxK


_RelaxK = None


def relax_energy(x0, B0, cfg: relax_config, K: int):
    """Differentiable (E_M(x_K), R2(x_K)) of K steps from (x0, B0) (torch.autograd.Function)."""
    global _RelaxK
    if _RelaxK is None:
        _RelaxK = _relax_function()
    if not cfg.record:
        raise ValueError("relax_energy needs cfg.record = 1")
    return _RelaxK.apply(x0, B0, cfg, int(K))
