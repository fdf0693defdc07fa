"""Thin Python binding of ``libapgp.so`` (C ABI in ``include/ap.h``).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels. PyTorch supplies device memory (caller-owned tensors, as the ABI
requires) and the HIP stream. Loading fails loudly when the library has not
been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapgp.so")

RBF, MATERN32, MATERN52 = 0, 1, 2
CYCLIC, GREEDY, RANDOM = 0, 1, 2
TILE_FP32, TILE_BF16, TILE_SPLIT, TILE_FP64 = 0, 1, 2, 3

OK, NOT_CONVERGED = 0, 1
ERR_INVALID_ARG, ERR_NOT_PD, ERR_NONFINITE = -1, -2, -3
ERR_WORKSPACE, ERR_HIP, ERR_UNSUPPORTED = -4, -5, -6

# every symbol include/ap.h declares
SYMBOLS = ("ap_workspace_bytes", "ap_factor_blocks", "ap_reset", "ap_epoch", "ap_update",
           "ap_rel_residual", "ap_solve", "ap_solve_from", "ap_warm_start", "ap_residual", "ap_block_inverse", "ap_set_tile",
           "ap_profile",
           "ap_profile_read", "ap_predict", "ap_mll_grad", "ap_batch_step", "ap_batch_peek", "ap_batch_release",
           "ap_destroy", "ap_status_str", "ap_last_error", "ap_residual_noalloc")
NOALLOC_MAX_N = 4194304
PHASES = ("block_solve", "fused_update", "select", "epoch_check", "true_residual")


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("l", ctypes.c_int32),
                ("b", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("lengthscale", ctypes.POINTER(ctypes.c_double)),
                ("outputscale", ctypes.c_double), ("noise", ctypes.c_double),
                ("order", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("refine_every", ctypes.c_int32), ("tol", ctypes.c_double),
                ("min_epochs", ctypes.c_int32), ("max_epochs", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class State(ctypes.Structure):
    _fields_ = [("B", ctypes.c_void_p), ("W", ctypes.c_void_p), ("R", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("refines", ctypes.c_int32),
                ("rho_maintained", ctypes.c_double), ("rho_true", ctypes.c_double),
                ("t_epochs", ctypes.c_double), ("t_refine", ctypes.c_double),
                ("tile", ctypes.c_int32), ("escalated_at", ctypes.c_int32),
                ("restarted_at", ctypes.c_int32)]


# ap_batch_state: why a problem of a batch is held
RUN, HOLD_REFINE, HOLD_TOL, HOLD_MAX, HOLD_NONFINITE = 0, 1, 2, 3, 4


class Progress(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("epoch", ctypes.c_int32),
                ("cursor", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rho", ctypes.c_double), ("rho_true", ctypes.c_double)]


class ApError(RuntimeError):
    def __init__(self, code: int, what: str, extra: str = ""):
        if code == ERR_HIP:
            extra += f" [{last_error()}]"
        super().__init__(f"{what}: {status_str(code)} ({code}){extra}")
        self.code = code


_lib = None


def _hip_runtimes() -> set[str]:
    """Files of the HIP runtime mapped into this process (Linux)."""
    found = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                path = line.split()[-1] if len(line.split()) >= 6 else ""
                if os.path.basename(path).startswith("libamdhip64.so"):
                    found.add(os.path.realpath(path))
    except OSError:
        pass
    return found


def load():
    """Load libapgp.so and declare its signatures (no GPU work).

    The library must share PyTorch's HIP runtime: the streams and device
    memory it is handed come from torch. torch's libraries ask for the
    unversioned libamdhip64.so next to them, the library for libamdhip64.so.7;
    when torch is loaded first the loader resolves the library's request to
    torch's copy by its soname, so torch is imported before the library, and a
    second runtime in the process is an error."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2310_17137_amd.build`")
        import torch  # noqa: F401  (maps torch's HIP runtime first)
        lib = ctypes.CDLL(LIB_PATH)
        runtimes = _hip_runtimes()
        if len(runtimes) > 1:
            raise RuntimeError("two HIP runtimes are loaded in this process "
                               f"({', '.join(sorted(runtimes))}); libapgp.so must share torch's")
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        C, S, St = ctypes.POINTER(Config), ctypes.POINTER(State), ctypes.POINTER(Stats)
        D = ctypes.POINTER(ctypes.c_double)
        sig = {
            "ap_workspace_bytes": (ctypes.c_size_t, [C]),
            "ap_factor_blocks": (I32, [C, P, P, ctypes.c_size_t, P, ctypes.POINTER(P),
                                       ctypes.POINTER(I64)]),
            "ap_reset": (I32, [P, S, P]),
            "ap_epoch": (I32, [ctypes.POINTER(P), S, I32, I32, P]),
            "ap_update": (I32, [P, S, I32, P]),
            "ap_rel_residual": (I32, [P, P, D, D]),
            "ap_solve": (I32, [P, S, P, St]),
            "ap_solve_from": (I32, [P, S, P, St]),
            "ap_warm_start": (I32, [P, S, P]),
            "ap_residual": (I32, [P, S, P, D, P]),
            "ap_residual_noalloc": (I32, [C, P, P, P, P, D, P]),
            "ap_block_inverse": (I32, [P, I32, P, P]),
            "ap_predict": (I32, [P, P, P, I64, P, P]),
            "ap_mll_grad": (I32, [P, S, D, P, P]),
            "ap_set_tile": (I32, [P, I32]),
            "ap_profile": (I32, [P, I32]),
            "ap_profile_read": (I32, [P, P, D, ctypes.POINTER(I64)]),
            "ap_batch_step": (I32, [ctypes.POINTER(P), S, I32, I32, P]),
            "ap_batch_peek": (I32, [P, ctypes.POINTER(Progress)]),
            "ap_batch_release": (I32, [P, I32, P]),
            "ap_destroy": (None, [P]),
            "ap_status_str": (ctypes.c_char_p, [I32]),
            "ap_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def status_str(code: int) -> str:
    return load().ap_status_str(code).decode()


def last_error() -> str:
    """The library's description of the last HIP failure on this thread."""
    return load().ap_last_error().decode()


def _check(code: int, what: str, ok=(OK,)):
    if code not in ok:
        raise ApError(code, what)
    return code


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_config(n, d, l, b, kernel, lengthscale, outputscale=1.0, noise=0.1, order=CYCLIC,
                tile=TILE_FP32, refine_every=0, tol=1e-2, min_epochs=0, max_epochs=1000,
                seed=0):
    ls = np.ascontiguousarray(np.broadcast_to(np.asarray(lengthscale, dtype=np.float64), (d,)))
    cfg = Config(int(n), int(d), int(l), int(b), int(kernel),
                 ls.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(outputscale),
                 float(noise), int(order), int(tile), int(refine_every), float(tol),
                 int(min_epochs), int(max_epochs), int(seed) & 0xFFFFFFFFFFFFFFFF)
    return cfg, ls


def workspace_bytes(**kw) -> int:
    cfg, _ls = make_config(**kw)
    return int(load().ap_workspace_bytes(ctypes.byref(cfg)))


@dataclass
class SolveStats:
    status: int
    epochs: int
    refines: int
    rho_maintained: float
    rho_true: float
    t_epochs: float
    t_refine: float
    tile: int = 0
    escalated_at: int = -1
    restarted_at: int = -1

    @property
    def converged(self) -> bool:
        return self.status == OK


class Solver:
    """One problem: borrowed features X (n x d FP32 on the GPU), a workspace
    tensor it owns, and the library handle with the cached block inverses."""

    def __init__(self, X, *, l: int, b: int, kernel: int, lengthscale, outputscale=1.0,
                 noise=0.1, order=CYCLIC, tile=TILE_FP32, refine_every=0, tol=1e-2,
                 min_epochs=0, max_epochs=1000, seed=0, stream=None, workspace=None):
        import torch
        if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.is_contiguous()):
            raise ValueError("X must be a contiguous n x d float32 CUDA tensor")
        self.X = X
        n, d = X.shape
        self.n, self.d, self.l, self.b = int(n), int(d), int(l), int(b)
        self.m = (self.n + self.b - 1) // self.b if self.b > 0 else 0
        self.cfg, self._ls = make_config(n, d, l, b, kernel, lengthscale, outputscale, noise,
                                         order, tile, refine_every, tol, min_epochs, max_epochs,
                                         seed)
        lib = load()
        need = int(lib.ap_workspace_bytes(ctypes.byref(self.cfg)))
        if need == 0:
            raise ApError(ERR_INVALID_ARG, "ap_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(need + 256, dtype=torch.uint8, device=X.device)
        self.ws = workspace
        base = workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = need
        if self._ws_ptr + need > base + workspace.numel():
            raise ApError(ERR_WORKSPACE, "workspace")
        self.handle = ctypes.c_void_p(0)
        bad = ctypes.c_int64(-1)
        code = lib.ap_factor_blocks(ctypes.byref(self.cfg), ctypes.c_void_p(X.data_ptr()),
                                    ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(need),
                                    _stream(stream), ctypes.byref(self.handle), ctypes.byref(bad))
        if code != OK:
            extra = f" (block {bad.value})" if code == ERR_NOT_PD else ""
            raise ApError(code, "ap_factor_blocks", extra)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.ap_destroy(h)
            self.handle = ctypes.c_void_p(0)

    def new_state(self, B):
        """(W, R) device tensors for right-hand sides B (n x l float32)."""
        import torch
        if not (B.is_cuda and B.dtype == torch.float32 and B.shape == (self.n, self.l)
                and B.is_contiguous()):
            raise ValueError("B must be a contiguous n x l float32 CUDA tensor")
        W = torch.zeros((self.n, self.l), dtype=torch.float64, device=B.device)
        R = torch.empty((self.n, self.l), dtype=torch.float32, device=B.device)
        return W, R

    @staticmethod
    def cstate(B, W, R) -> State:
        return State(B.data_ptr(), W.data_ptr(), R.data_ptr())

    def reset(self, B, W, R, stream=None):
        st = self.cstate(B, W, R)
        _check(load().ap_reset(self.handle, ctypes.byref(st), _stream(stream)), "ap_reset")

    def warm_start(self, B, W, R, stream=None):
        """Restart from the given W: R = B - K^ W (FP64), fresh epoch state."""
        st = self.cstate(B, W, R)
        _check(load().ap_warm_start(self.handle, ctypes.byref(st), _stream(stream)),
               "ap_warm_start")

    def epoch(self, B, W, R, epochs: int = 1, stream=None):
        st = self.cstate(B, W, R)
        h = (ctypes.c_void_p * 1)(self.handle.value)
        _check(load().ap_epoch(h, ctypes.byref(st), 1, int(epochs), _stream(stream)), "ap_epoch")

    def update(self, B, W, R, block: int, stream=None):
        st = self.cstate(B, W, R)
        _check(load().ap_update(self.handle, ctypes.byref(st), int(block), _stream(stream)),
               "ap_update")

    def rel_residual(self, stream=None):
        rho = ctypes.c_double(0.0)
        cols = (ctypes.c_double * self.l)()
        _check(load().ap_rel_residual(self.handle, _stream(stream), ctypes.byref(rho), cols),
               "ap_rel_residual")
        return rho.value, np.array(cols[:], dtype=np.float64)

    def solve(self, B, W, R, warm: bool = False, stream=None) -> SolveStats:
        """ap_solve (from W = 0), or ap_solve_from (from the given W) if warm."""
        st = self.cstate(B, W, R)
        s = Stats()
        fn = load().ap_solve_from if warm else load().ap_solve
        code = fn(self.handle, ctypes.byref(st), _stream(stream), ctypes.byref(s))
        _check(code, "ap_solve_from" if warm else "ap_solve", ok=(OK, NOT_CONVERGED))
        return SolveStats(code, s.epochs, s.refines, s.rho_maintained, s.rho_true, s.t_epochs,
                          s.t_refine, s.tile, s.escalated_at, s.restarted_at)

    def residual(self, B, W, R, R_out=None, want_col_rel: bool = True, stream=None):
        """FP64 true residual into R_out (None: refine R in place)."""
        st = self.cstate(B, W, R)
        cols = (ctypes.c_double * self.l)() if want_col_rel else None
        out = ctypes.c_void_p(R_out.data_ptr()) if R_out is not None else ctypes.c_void_p(0)
        _check(load().ap_residual(self.handle, ctypes.byref(st), out, cols, _stream(stream)),
               "ap_residual")
        if cols is None:
            return None
        return np.array(cols[:], dtype=np.float64)

    def set_tile(self, tile: int):
        _check(load().ap_set_tile(self.handle, int(tile)), "ap_set_tile")

    def profile(self, enable: bool = True):
        _check(load().ap_profile(self.handle, int(bool(enable))), "ap_profile")

    def profile_read(self, stream=None) -> dict:
        secs = (ctypes.c_double * 5)()
        cnt = (ctypes.c_int64 * 5)()
        _check(load().ap_profile_read(self.handle, _stream(stream), secs, cnt), "ap_profile_read")
        return {name: (secs[i], int(cnt[i])) for i, name in enumerate(PHASES)}

    def peek(self) -> Progress:
        """Snapshot of this problem's batch progress (ap_batch_peek)."""
        out = Progress()
        _check(load().ap_batch_peek(self.handle, ctypes.byref(out)), "ap_batch_peek")
        return out

    def release(self, next_refine: int = 0, stream=None):
        """Resume a held batch problem; next_refine > 0 sets the epoch of its
        next true-residual hold (0: the refine_every schedule)."""
        _check(load().ap_batch_release(self.handle, int(next_refine), _stream(stream)),
               "ap_batch_release")

    def predict(self, W, Xs, stream=None):
        """Posterior mean K(Xs, X) W (ns x l FP64) at test points Xs (ns x d
        float32 CUDA tensor)."""
        import torch
        if not (Xs.is_cuda and Xs.dtype == torch.float32 and Xs.dim() == 2
                and Xs.shape[1] == self.d and Xs.is_contiguous()):
            raise ValueError("Xs must be a contiguous ns x d float32 CUDA tensor")
        if not (W.is_cuda and W.dtype == torch.float64 and W.shape == (self.n, self.l)):
            raise ValueError("W must be the n x l float64 weights")
        ns = int(Xs.shape[0])
        out = torch.empty((ns, self.l), dtype=torch.float64, device=Xs.device)
        _check(load().ap_predict(self.handle, ctypes.c_void_p(W.data_ptr()),
                                 ctypes.c_void_p(Xs.data_ptr()), ns,
                                 ctypes.c_void_p(out.data_ptr()), _stream(stream)), "ap_predict")
        return out

    def mll_grad(self, B, W, R, partials: bool = False, stream=None):
        """Stochastic gradient of the negative log marginal likelihood in
        (lengthscales, outputscale, noise) from W = K^^{-1} B, B = [y, probes].
        With partials=True also returns the per-64-row partial sums (device)."""
        import torch
        st = self.cstate(B, W, R)
        grad = (ctypes.c_double * (self.d + 2))()
        part = None
        if partials:
            part = torch.zeros(((self.n + 63) // 64, 22), dtype=torch.float64, device=W.device)
        _check(load().ap_mll_grad(self.handle, ctypes.byref(st), grad,
                                  ctypes.c_void_p(part.data_ptr() if part is not None else 0),
                                  _stream(stream)), "ap_mll_grad")
        g = np.array(grad[:], dtype=np.float64)
        return (g, part) if partials else g

    def block_inverse(self, j: int, stream=None):
        import torch
        ln = min(self.b, self.n - j * self.b)
        out = torch.empty((ln, ln), dtype=torch.float64, device=self.X.device)
        _check(load().ap_block_inverse(self.handle, int(j), ctypes.c_void_p(out.data_ptr()),
                                       _stream(stream)), "ap_block_inverse")
        return out


def residual_noalloc(X, B, W, R_out, *, kernel: int, lengthscale, outputscale=1.0, noise=0.1,
                     want_col_rel: bool = True, stream=None):
    """ap_residual_noalloc: R_out = B - K^ W in FP64 (written as FP32) with no
    handle and no workspace; returns the per-column ratios (synchronizes) or
    None."""
    import torch
    for t, dt in ((X, torch.float32), (B, torch.float32), (W, torch.float64),
                  (R_out, torch.float32)):
        if not (t.is_cuda and t.dtype == dt and t.dim() == 2 and t.is_contiguous()):
            raise ValueError("X, B, R_out: contiguous float32 CUDA tensors; W: float64")
    n, d = X.shape
    l = B.shape[1]
    if B.shape != (n, l) or W.shape != (n, l) or R_out.shape != (n, l):
        raise ValueError("B, W and R_out must be n x l")
    cfg, _ls = make_config(n, d, l, min(n, 4096), kernel, lengthscale, outputscale, noise)
    cols = (ctypes.c_double * l)() if want_col_rel else None
    _check(load().ap_residual_noalloc(ctypes.byref(cfg), ctypes.c_void_p(X.data_ptr()),
                                      ctypes.c_void_p(B.data_ptr()),
                                      ctypes.c_void_p(W.data_ptr()),
                                      ctypes.c_void_p(R_out.data_ptr()), cols, _stream(stream)),
           "ap_residual_noalloc")
    return None if cols is None else np.array(cols[:], dtype=np.float64)


def epoch_many(solvers, states, epochs: int = 1, stream=None):
    """ap_epoch over several problems in one call (states: (B, W, R) tuples)."""
    count = len(solvers)
    hs = (ctypes.c_void_p * count)(*[s.handle.value for s in solvers])
    sts = (State * count)(*[Solver.cstate(*st) for st in states])
    _check(load().ap_epoch(hs, sts, count, int(epochs), _stream(stream)), "ap_epoch")


def batch_step(solvers, states, steps: int = 1, stream=None):
    """ap_batch_step over the problems (states: (B, W, R) tuples)."""
    count = len(solvers)
    hs = (ctypes.c_void_p * count)(*[s.handle.value for s in solvers])
    sts = (State * count)(*[Solver.cstate(*st) for st in states])
    _check(load().ap_batch_step(hs, sts, count, int(steps), _stream(stream)), "ap_batch_step")


def from_workload(w, device="cuda", tile=TILE_FP32, **over):
    """Upload a gen.Workload and build its Solver; returns (solver, B, W, R)."""
    import torch
    X = torch.from_numpy(w.X).to(device)
    B = torch.from_numpy(w.B).to(device)
    kw = dict(l=w.l, b=w.b, kernel=w.kernel, lengthscale=w.lengthscale,
              outputscale=w.outputscale, noise=w.noise, order=w.order, tile=tile,
              refine_every=w.refine_every, tol=w.tol, min_epochs=w.min_epochs,
              max_epochs=w.max_epochs, seed=w.seed)
    kw.update(over)
    s = Solver(X, **kw)
    W, R = s.new_state(B)
    return s, B, W, R

