"""Python binding of libaltgdmin.so (the C ABI declared in include/altgdmin.h).

Argument marshalling only: torch tensors on the GPU are passed as raw device
pointers with the layouts the header states, and every step runs in the HIP
kernels of the library.  There is no CPU fallback: if the library is not built,
or no GPU is present, the calls raise.

Function names match the C entry points.  ``Solver`` is a convenience owner of
the problem tensors and the workspace.
"""
from __future__ import annotations

import contextlib
import ctypes
import functools
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libaltgdmin.so")

ALTGDMIN_OK = 0
ALTGDMIN_ENOTCONV = 1
ALTGDMIN_EINVAL = -1
ALTGDMIN_ENOWS = -2
ALTGDMIN_EHIP = -3
ALTGDMIN_ENONFINITE = -4
ALTGDMIN_ENOTBUILT = -5
ALTGDMIN_A_F32 = 0
ALTGDMIN_A_BF16X2 = 1
ALTGDMIN_A_PHILOX = 2
ALTGDMIN_A_PFOURIER = 3
FLAG_EAGER = 1      # params.flags bit 0: launch the iteration's kernels without a HIP graph
FLAG_AUTOTUNE = 2   # params.flags bit 1: time the streaming-kernel variants at init and keep the fastest
FLAG_BF16_MIXED = 4  # params.flags bit 2: BF16X2 planes, hi plane alone for the transposed products

c_i32, c_i64, c_f64, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class Problem(ctypes.Structure):
    _fields_ = [("n", c_i32), ("q", c_i32), ("m", c_i32), ("r", c_i32), ("rho", c_i32),
                ("a_format", c_i32), ("A", c_vp), ("A_lo", c_vp), ("lda", c_i64),
                ("a_stride_k", c_i64), ("Y", c_vp), ("ldy", c_i64), ("U_start", c_vp),
                ("a_seed", ctypes.c_uint64), ("normal_table", c_vp), ("n1", c_i32), ("n2", c_i32),
                ("fourier_mask", c_vp)]


class Params(ctypes.Structure):
    _fields_ = [("tau0", c_i32), ("tau", c_i32), ("t_max", c_i32), ("power_iters", c_i32),
                ("poll_every", c_i32), ("flags", c_i32), ("eta_c", c_f64), ("power_tol", c_f64),
                ("tol_resid", c_f64), ("bf16_hi_max", c_i32), ("pad0", c_i32), ("bf16_stall", c_f64),
                ("rank_energy", c_f64), ("rank_iters", c_i32), ("pad1", c_i32)]


class Report(ctypes.Structure):
    _fields_ = [("iterations", c_i32), ("power_iterations", c_i32), ("error_flags", c_i32),
                ("converged", c_i32), ("refine_iteration", c_i32), ("rank", c_i32), ("eta", c_f64),
                ("resid", c_f64), ("power_sd", c_f64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class AltGDminError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"altgdmin error {code}: {msg}")
        self.code = code


_lib = None

_SIGS = {
    "altgdmin_default_params": (None, [c_vp]),
    "altgdmin_workspace_bytes": (c_i32, [c_vp, c_vp, c_vp]),
    "altgdmin_init": (c_i32, [c_vp, c_vp, c_vp, c_sz, c_vp, c_vp]),
    "altgdmin_step": (c_i32, [c_vp, c_i32, c_vp]),
    "altgdmin_get": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "altgdmin_status": (c_i32, [c_vp, c_vp, c_vp]),
    "altgdmin_status_many": (c_i32, [c_vp, c_i32, c_vp, c_vp]),
    "altgdmin_residual_log": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "altgdmin_solve": (c_i32, [c_vp, c_vp, c_vp, c_sz, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "altgdmin_destroy": (c_i32, [c_vp]),
    "altgdmin_state_bytes": (c_i32, [c_vp, c_vp]),
    "altgdmin_get_state": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
    "altgdmin_set_state": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
    "altgdmin_profile_iteration": (c_i32, [c_vp, c_i32, c_vp, c_vp]),
    "altgdmin_group_bytes": (c_i32, [c_vp, c_i32, c_vp]),
    "altgdmin_step_many": (c_i32, [c_vp, c_i32, c_i32, c_vp, c_sz, c_vp]),
    "altgdmin_strerror": (ctypes.c_char_p, [c_i32]),
    "altgdmin_last_error": (ctypes.c_char_p, []),
    "altgdmin_tuning": (c_i32, [c_vp, c_vp, c_vp]),
    "altgdmin_op_select": (c_i32, [c_vp, c_i32, c_i32, c_i64, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "altgdmin_op_au": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "altgdmin_op_philox_fill": (c_i32, [ctypes.c_uint64, c_vp, c_i32, c_i32, c_i32, c_i64, c_vp, c_vp]),
    "altgdmin_op_make_a": (c_i32, [ctypes.c_uint64, c_vp, c_i32, c_i32, c_i32, c_i64, c_i32, c_vp, c_vp, c_vp]),
    "altgdmin_op_measure": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "altgdmin_op_iht": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "altgdmin_op_lsgrad": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "altgdmin_op_backproject": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "altgdmin_op_scratch_bytes": (c_i32, [c_i32, c_i32, c_i32, c_vp]),
    "altgdmin_op_grad": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_sz, c_vp]),
    "altgdmin_op_qr_step": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_f64, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "altgdmin_op_subspace": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_vp, c_i32, c_f64, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "altgdmin_op_subspace_noalloc": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_vp, c_i32, c_f64, c_vp, c_vp, c_vp]),
    "altgdmin_op_rank_scratch_bytes": (c_i32, [c_i32, c_i32, c_i32, c_vp]),
    "altgdmin_op_rank": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_f64, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp]),
}

EXPORTED = tuple(_SIGS)


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2311_03824_amd.build`")
    # torch ships its own HIP runtime under the same SONAME as the system one;
    # importing torch first makes the library bind to that already-loaded
    # runtime, so torch and the library share one HIP runtime (streams, memory).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int) -> int:
    """Raise on errors (negative codes); pass OK and the ENOTCONV warning through."""
    if rc < 0:
        raise AltGDminError(rc, _lib.altgdmin_last_error().decode())
    return rc


# ------------------------------------------------------------------ torch plumbing

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("altgdmin needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


_lib_streams = {}


def _library_stream(device):
    """One created stream per device (default priority) for calls made from torch's
    null stream: the library never enqueues on the null stream."""
    torch = _torch()
    idx = torch.device(device).index
    idx = torch.cuda.current_device() if idx is None else idx
    s = _lib_streams.get(idx)
    if s is None:
        s = torch.cuda.Stream(device=idx)
        _lib_streams[idx] = s
    return s


@contextlib.contextmanager
def _stream_scope(stream=None):
    """The stream a call enqueues on: the caller's (or torch's current) stream when it is
    a created stream; otherwise the library stream, ordered after the work already on
    the caller's stream and before any work the caller enqueues next."""
    torch = _torch()
    caller = stream if stream is not None else torch.cuda.current_stream()
    if caller.cuda_stream != 0:
        yield caller
        return
    ls = _library_stream(caller.device)
    ls.wait_stream(caller)
    try:
        yield ls
    finally:
        caller.wait_stream(ls)


def _on_stream(fn):
    """Entry points taking `stream=`: run `fn` with the stream of _stream_scope."""
    @functools.wraps(fn)
    def wrapper(*args, stream=None, **kw):
        with _stream_scope(stream) as s:
            return fn(*args, stream=s, **kw)
    return wrapper


def stream_ptr(stream) -> int:
    p = stream.cuda_stream
    if not p:
        raise ValueError("the library never enqueues on the null stream")
    return p


def default_params(**kw) -> Params:
    load()
    p = Params()
    _lib.altgdmin_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def make_fourier_problem(mask, Y, n1: int, n2: int, r: int, rho: int, U_start=None) -> Problem:
    """Partial Fourier form: mask (q, m) int32 and Y (q, m) complex64 device tensors
    (Y may also be a (q, m, 2) float32 view); frames of n1 x n2."""
    p = Problem()
    q, m = mask.shape[0], mask.shape[1]
    p.a_format = ALTGDMIN_A_PFOURIER
    p.n, p.q, p.m, p.r, p.rho = n1 * n2, q, m, r, rho
    p.n1, p.n2 = n1, n2
    p.fourier_mask = ptr(mask)
    p.Y, p.ldy = ptr(Y), Y.shape[1]
    p.U_start = ptr(U_start)
    return p


def make_problem(A, Y, r: int, rho: int, A_lo=None, U_start=None, m: Optional[int] = None,
                 philox_seed: Optional[int] = None, normal_table=None, n: Optional[int] = None) -> Problem:
    """A: (q, n, lda) float32 (or int16/uint16 bf16 hi plane with A_lo), Y: (q, ldy) float32.

    Philox form: A=None, philox_seed and normal_table (device FP32) given, n given.
    """
    p = Problem()
    if philox_seed is not None:
        q = Y.shape[0]
        p.a_format = ALTGDMIN_A_PHILOX
        p.a_seed, p.normal_table = int(philox_seed), ptr(normal_table)
        p.lda = p.a_stride_k = 0
    else:
        q, n, lda = A.shape
        p.a_format = ALTGDMIN_A_BF16X2 if A_lo is not None else ALTGDMIN_A_F32
        p.A, p.A_lo = ptr(A), ptr(A_lo)
        p.lda, p.a_stride_k = lda, n * lda
    p.n, p.q, p.r, p.rho = n, q, r, rho
    p.m = int(m) if m is not None else int(Y.shape[1])
    p.Y, p.ldy = ptr(Y), Y.shape[1]
    p.U_start = ptr(U_start)
    return p


# ------------------------------------------------------------------ entry points (same names as the C ABI)

def altgdmin_workspace_bytes(prob: Problem, par: Params) -> int:
    load()
    b = c_sz(0)
    _check(_lib.altgdmin_workspace_bytes(ctypes.byref(prob), ctypes.byref(par), ctypes.byref(b)))
    return b.value


@_on_stream
def altgdmin_init(prob: Problem, par: Params, workspace, stream=None) -> c_vp:
    load()
    h = c_vp()
    _check(_lib.altgdmin_init(ctypes.byref(prob), ctypes.byref(par), ptr(workspace),
                              workspace.numel() * workspace.element_size(), stream_ptr(stream),
                              ctypes.byref(h)))
    return h


@_on_stream
def altgdmin_step(h, iters: int, stream=None) -> None:
    _check(_lib.altgdmin_step(h, iters, stream_ptr(stream)))


@_on_stream
def altgdmin_get(h, U=None, Bt=None, S_idx=None, S_val=None, U_next=None, stream=None) -> None:
    _check(_lib.altgdmin_get(h, ptr(U), ptr(Bt), ptr(S_idx), ptr(S_val), ptr(U_next), stream_ptr(stream)))


@_on_stream
def altgdmin_status(h, stream=None) -> dict:
    rep = Report()
    _check(_lib.altgdmin_status(h, stream_ptr(stream), ctypes.byref(rep)))
    return rep.as_dict()


@_on_stream
def altgdmin_status_many(hs, stream=None) -> list:
    """Status of several handles with one synchronisation (serving polls)."""
    reps = (Report * max(1, len(hs)))()
    _check(_lib.altgdmin_status_many(_handle_array(hs), len(hs), stream_ptr(stream), reps))
    return [reps[i].as_dict() for i in range(len(hs))]


@_on_stream
def altgdmin_residual_log(h, t_max: int, stream=None) -> np.ndarray:
    buf = (c_f64 * max(1, t_max))()
    cnt = c_i32(0)
    _check(_lib.altgdmin_residual_log(h, stream_ptr(stream), buf, ctypes.byref(cnt)))
    return np.array(buf[: cnt.value])


def _handle_array(hs):
    arr = (c_vp * len(hs))()
    for i, h in enumerate(hs):
        arr[i] = h.value if isinstance(h, c_vp) else h
    return arr


def altgdmin_group_bytes(hs) -> int:
    load()
    b = c_sz(0)
    _check(_lib.altgdmin_group_bytes(_handle_array(hs), len(hs), ctypes.byref(b)))
    return b.value


@_on_stream
def altgdmin_step_many(hs, iters: int, group_ws, stream=None) -> None:
    """One batched launch sequence per iteration over all handles (serving)."""
    _check(_lib.altgdmin_step_many(_handle_array(hs), len(hs), iters, ptr(group_ws),
                                   group_ws.numel() * group_ws.element_size(), stream_ptr(stream)))


KERNELS = ("k_au", "k_col", "k_grad", "k_qr")


@_on_stream
def altgdmin_profile_iteration(h, iters: int, stream=None) -> dict:
    """Average per-kernel milliseconds of `iters` eager GDmin iterations (HIP events on the launch stream)."""
    ms = (c_f64 * 4)()
    _check(_lib.altgdmin_profile_iteration(h, iters, stream_ptr(stream), ms))
    return dict(zip(KERNELS, list(ms)))


def altgdmin_tuning(h) -> dict:
    """The autotuned column-kernel unroll and A_k U depth of a handle (0: defaults)."""
    ju, aud = c_i32(0), c_i32(0)
    _check(_lib.altgdmin_tuning(h, ctypes.byref(ju), ctypes.byref(aud)))
    return {"col_unroll": ju.value, "au_depth": aud.value}


def altgdmin_state_bytes(h) -> int:
    load()
    b = c_sz(0)
    _check(_lib.altgdmin_state_bytes(h, ctypes.byref(b)))
    return b.value


@_on_stream
def altgdmin_get_state(h, state, stream=None) -> None:
    """Save the solver state into the device tensor `state` (uint8, >= altgdmin_state_bytes)."""
    _check(_lib.altgdmin_get_state(h, ptr(state), state.numel() * state.element_size(), stream_ptr(stream)))


@_on_stream
def altgdmin_set_state(h, state, stream=None) -> None:
    """Load a state saved from a handle of the same problem into h."""
    _check(_lib.altgdmin_set_state(h, ptr(state), state.numel() * state.element_size(), stream_ptr(stream)))


def altgdmin_destroy(h) -> None:
    if h:
        _lib.altgdmin_destroy(h)


@_on_stream
def altgdmin_solve(prob: Problem, par: Params, workspace, U=None, Bt=None, S_idx=None, S_val=None,
                   stream=None):
    load()
    rep = Report()
    rc = _check(_lib.altgdmin_solve(ctypes.byref(prob), ctypes.byref(par), ptr(workspace),
                                    workspace.numel() * workspace.element_size(), stream_ptr(stream),
                                    ptr(U), ptr(Bt), ptr(S_idx), ptr(S_val), ctypes.byref(rep)))
    return rc, rep.as_dict()


@_on_stream
def altgdmin_op_select(V, rho: int, idx, val, flags=None, stream=None) -> None:
    load()
    count, n = V.shape
    _check(_lib.altgdmin_op_select(ptr(V), n, count, n, rho, ptr(idx), ptr(val), ptr(flags), stream_ptr(stream)))


@_on_stream
def altgdmin_op_philox_fill(seed: int, normal_table, q: int, n: int, m: int, A, stream=None) -> None:
    """Write the Philox form of A (q, n, lda) FP32 into the device tensor A."""
    load()
    _check(_lib.altgdmin_op_philox_fill(int(seed), ptr(normal_table), q, n, m, A.shape[2], ptr(A), stream_ptr(stream)))


@_on_stream
def altgdmin_op_make_a(seed: int, normal_table, q: int, n: int, m: int, A, A_lo=None, stream=None) -> None:
    """Write the canonical synthetic A: FP32 (q, n, lda) into A, or, with A_lo given,
    the BF16 hi plane into A and the lo plane into A_lo (int16/uint16 (q, n, lda))."""
    load()
    fmt = ALTGDMIN_A_BF16X2 if A_lo is not None else ALTGDMIN_A_F32
    _check(_lib.altgdmin_op_make_a(int(seed), ptr(normal_table), q, n, m, A.shape[2], fmt, ptr(A), ptr(A_lo),
                                   stream_ptr(stream)))


@_on_stream
def altgdmin_op_measure(prob: Problem, Xt, Y, stream=None) -> None:
    """Y[k, :m] = A_k x_k with FP64 accumulation; Xt (q, n) float64 on the device."""
    load()
    _check(_lib.altgdmin_op_measure(ctypes.byref(prob), ptr(Xt), ptr(Y), stream_ptr(stream)))


@_on_stream
def altgdmin_op_au(prob: Problem, U, P, Ginv, flags=None, stream=None) -> None:
    load()
    _check(_lib.altgdmin_op_au(ctypes.byref(prob), ptr(U), ptr(P), ptr(Ginv), ptr(flags), stream_ptr(stream)))


@_on_stream
def altgdmin_op_iht(prob: Problem, project: bool, P, Ginv, tau: int, has_support: bool, S_idx, S_val,
                    G_out=None, mu_out=None, flags=None, stream=None) -> None:
    load()
    _check(_lib.altgdmin_op_iht(ctypes.byref(prob), int(project), ptr(P), ptr(Ginv), tau, int(has_support),
                                ptr(S_idx), ptr(S_val), ptr(G_out), ptr(mu_out), ptr(flags), stream_ptr(stream)))


@_on_stream
def altgdmin_op_lsgrad(prob: Problem, P, Ginv, S_idx, S_val, Bt, H, rr=None, flags=None, stream=None) -> None:
    load()
    _check(_lib.altgdmin_op_lsgrad(ctypes.byref(prob), ptr(P), ptr(Ginv), ptr(S_idx), ptr(S_val), ptr(Bt),
                                   ptr(H), ptr(rr), ptr(flags), stream_ptr(stream)))


@_on_stream
def altgdmin_op_backproject(prob: Problem, S_idx, S_val, L0t, stream=None) -> None:
    load()
    _check(_lib.altgdmin_op_backproject(ctypes.byref(prob), ptr(S_idx), ptr(S_val), ptr(L0t), stream_ptr(stream)))


def altgdmin_op_scratch_bytes(n: int, q: int, r: int) -> int:
    load()
    b = c_sz(0)
    _check(_lib.altgdmin_op_scratch_bytes(n, q, r, ctypes.byref(b)))
    return b.value


def _scratch(n, q, r):
    torch = _torch()
    return torch.empty(altgdmin_op_scratch_bytes(n, q, r) + 256, dtype=torch.uint8, device="cuda")


@_on_stream
def altgdmin_op_grad(H, Bt, grad, scratch=None, stream=None) -> None:
    load()
    q, n = H.shape
    r = Bt.shape[1]
    scratch = _scratch(n, q, r) if scratch is None else scratch
    _check(_lib.altgdmin_op_grad(ptr(H), ptr(Bt), n, q, r, ptr(grad), ptr(scratch), scratch.numel(),
                                 stream_ptr(stream)))


@_on_stream
def altgdmin_op_qr_step(U, grad, eta_c: float, eta_io, U_out, scratch=None, stream=None) -> None:
    load()
    n, r = U.shape
    scratch = _scratch(n, 1, r) if scratch is None else scratch
    _check(_lib.altgdmin_op_qr_step(ptr(U), ptr(grad), n, r, eta_c, ptr(eta_io), ptr(U_out), ptr(scratch),
                                    scratch.numel(), stream_ptr(stream)))


@_on_stream
def altgdmin_op_subspace(L0t, r: int, U_start, iters: int, tol: float, U_out, iters_out=None, scratch=None,
                         stream=None) -> None:
    load()
    q, n = L0t.shape
    scratch = _scratch(n, q, r) if scratch is None else scratch
    _check(_lib.altgdmin_op_subspace(ptr(L0t), n, q, r, ptr(U_start), iters, tol, ptr(U_out), ptr(iters_out),
                                     ptr(scratch), scratch.numel(), stream_ptr(stream)))


def altgdmin_op_rank_scratch_bytes(n: int, q: int, m: int) -> int:
    load()
    b = c_sz(0)
    _check(_lib.altgdmin_op_rank_scratch_bytes(n, q, m, ctypes.byref(b)))
    return b.value


@_on_stream
def altgdmin_op_rank(L0t, m: int, energy: float, iters: int, r_out, sv_out=None, scratch=None,
                     stream=None) -> None:
    """Automatic rank of Sec. 2.6 on L_0 (given as L0t, q x n): r into r_out (device int32),
    the K leading singular-value estimates into sv_out (device float64, optional)."""
    load()
    torch = _torch()
    q, n = L0t.shape
    if scratch is None:
        scratch = torch.empty(altgdmin_op_rank_scratch_bytes(n, q, m) + 256, dtype=torch.uint8, device="cuda")
    _check(_lib.altgdmin_op_rank(ptr(L0t), n, q, m, energy, iters, ptr(r_out), ptr(sv_out), ptr(scratch),
                                 scratch.numel(), stream_ptr(stream)))


@_on_stream
def altgdmin_op_subspace_noalloc(L0t, r: int, U_start, iters: int, tol: float, U_out, iters_out=None,
                                 stream=None) -> None:
    """altgdmin_op_subspace with the library's static device scratch (no allocation)."""
    load()
    q, n = L0t.shape
    _check(_lib.altgdmin_op_subspace_noalloc(ptr(L0t), n, q, r, ptr(U_start), iters, tol, ptr(U_out),
                                             ptr(iters_out), stream_ptr(stream)))


# ------------------------------------------------------------------ convenience owner

class Solver:
    """Owns the device copies of one problem and its workspace; drives init/step/get."""

    def __init__(self, At: np.ndarray, Y: np.ndarray, m: int, r: int, rho: int, params: Optional[Params] = None,
                 A_hi: Optional[np.ndarray] = None, A_lo: Optional[np.ndarray] = None,
                 U_start: Optional[np.ndarray] = None, device="cuda", philox_seed: Optional[int] = None,
                 normal_table: Optional[np.ndarray] = None, n: Optional[int] = None):
        torch = _torch()
        load()
        self.table = None
        if philox_seed is not None:
            self.A = self.A_lo = None
            self.table = torch.from_numpy(np.ascontiguousarray(normal_table, dtype=np.float32)).to(device)
        elif A_hi is not None:
            self.A = torch.from_numpy(np.ascontiguousarray(A_hi).view(np.int16)).to(device)
            self.A_lo = torch.from_numpy(A_lo.view(np.int16)).to(device)
        else:
            self.A = torch.from_numpy(np.ascontiguousarray(At, dtype=np.float32)).to(device)
            self.A_lo = None
        self.Y = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.float32)).to(device)
        self.U_start = None if U_start is None else torch.from_numpy(np.ascontiguousarray(U_start, dtype=np.float32)).to(device)
        if philox_seed is not None:
            self.q, self.n = self.Y.shape[0], int(n)
        else:
            self.q, self.n, _ = self.A.shape
        self.m, self.r, self.rho = m, r, rho
        self.prob = make_problem(self.A, self.Y, r, rho, A_lo=self.A_lo, U_start=self.U_start, m=m,
                                 philox_seed=philox_seed, normal_table=self.table, n=self.n)
        self.par = params if params is not None else default_params()
        nb = altgdmin_workspace_bytes(self.prob, self.par)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        self.h = None

    def init(self, stream=None):
        if self.h is not None:
            altgdmin_destroy(self.h)
        self.h = altgdmin_init(self.prob, self.par, self.ws, stream=stream)
        if self.prob.r == 0:    # automatic rank: the one the initialisation chose
            self.r = altgdmin_status(self.h, stream=stream)["rank"]
        return self

    def step(self, iters: int, stream=None):
        altgdmin_step(self.h, iters, stream=stream)
        return self

    def get(self, stream=None):
        torch = _torch()
        U = torch.empty((self.n, self.r), dtype=torch.float32, device="cuda")
        Un = torch.empty_like(U)
        Bt = torch.empty((self.q, self.r), dtype=torch.float32, device="cuda")
        Si = torch.zeros((self.q, max(self.rho, 1)), dtype=torch.int32, device="cuda")
        Sv = torch.zeros((self.q, max(self.rho, 1)), dtype=torch.float32, device="cuda")
        altgdmin_get(self.h, U, Bt, Si if self.rho else None, Sv if self.rho else None, Un, stream=stream)
        torch.cuda.synchronize()
        return dict(U=U.cpu().numpy(), U_next=Un.cpu().numpy(), Bt=Bt.cpu().numpy(),
                    S_idx=Si.cpu().numpy()[:, : self.rho], S_val=Sv.cpu().numpy()[:, : self.rho])

    def status(self, stream=None) -> dict:
        return altgdmin_status(self.h, stream=stream)

    def profile_iteration(self, iters: int) -> dict:
        return altgdmin_profile_iteration(self.h, iters)

    def residual_log(self) -> np.ndarray:
        return altgdmin_residual_log(self.h, max(1, self.par.t_max))

    def close(self):
        if self.h is not None:
            altgdmin_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FourierSolver:
    """Owns the device copies of one partial Fourier problem (complex64) and its workspace."""

    def __init__(self, mask: np.ndarray, Y: np.ndarray, n1: int, n2: int, r: int, rho: int,
                 params: Optional[Params] = None, U_start: Optional[np.ndarray] = None, device="cuda"):
        torch = _torch()
        load()
        self.mask = torch.from_numpy(np.ascontiguousarray(mask, dtype=np.int32)).to(device)
        self.Y = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.complex64)).to(device)
        self.U_start = (None if U_start is None else
                        torch.from_numpy(np.ascontiguousarray(U_start, dtype=np.complex64)).to(device))
        self.q, self.m = mask.shape
        self.n, self.r, self.rho = n1 * n2, r, rho
        self.prob = make_fourier_problem(self.mask, self.Y, n1, n2, r, rho, self.U_start)
        self.par = params if params is not None else default_params()
        self.ws = torch.empty(altgdmin_workspace_bytes(self.prob, self.par), dtype=torch.uint8, device=device)
        self.h = None

    def init(self, stream=None):
        if self.h is not None:
            altgdmin_destroy(self.h)
        self.h = altgdmin_init(self.prob, self.par, self.ws, stream=stream)
        if self.prob.r == 0:    # automatic rank: the one the initialisation chose
            self.r = altgdmin_status(self.h, stream=stream)["rank"]
        return self

    def step(self, iters: int, stream=None):
        altgdmin_step(self.h, iters, stream=stream)
        return self

    def get(self, stream=None):
        torch = _torch()
        U = torch.empty((self.n, self.r), dtype=torch.complex64, device="cuda")
        Un = torch.empty_like(U)
        Bt = torch.empty((self.q, self.r), dtype=torch.complex64, device="cuda")
        Si = torch.zeros((self.q, max(self.rho, 1)), dtype=torch.int32, device="cuda")
        Sv = torch.zeros((self.q, max(self.rho, 1)), dtype=torch.complex64, device="cuda")
        altgdmin_get(self.h, U, Bt, Si if self.rho else None, Sv if self.rho else None, Un, stream=stream)
        torch.cuda.synchronize()
        return dict(U=U.cpu().numpy(), U_next=Un.cpu().numpy(), Bt=Bt.cpu().numpy(),
                    S_idx=Si.cpu().numpy()[:, : self.rho], S_val=Sv.cpu().numpy()[:, : self.rho])

    def status(self, stream=None) -> dict:
        return altgdmin_status(self.h, stream=stream)

    def profile_iteration(self, iters: int) -> dict:
        return altgdmin_profile_iteration(self.h, iters)

    def close(self):
        if self.h is not None:
            altgdmin_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
