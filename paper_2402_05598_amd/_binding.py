"""ctypes binding of libfcgno.so.  Argument marshalling only: every step of the
solve and of the operator runs in the HIP library.  Tensors are torch device
tensors (float64, contiguous); torch supplies device memory and the stream."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_size_t, c_void_p, c_char_p

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfcgno.so")

OP = {"fp64": 0, "fp32": 1, "bf16": 2, "identity": 3, "jacobi": 4, "sgs_rb": 5}
# operators that take no model
MODEL_FREE = ("identity", "jacobi", "sgs_rb")
SYS_OK, SYS_NOT_CONVERGED, SYS_BREAKDOWN, SYS_NONFINITE = 0, 1, 2, 3
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "BREAKDOWN", 3: "NONFINITE"}


class Arch(ctypes.Structure):
    _fields_ = [("layers", c_int32), ("width", c_int32), ("modes", c_int32), ("in_channels", c_int32),
                ("basis", c_int32)]


BASIS = {"fourier": 0, "sine": 1}


class SolveDesc(ctypes.Structure):
    _fields_ = [("n", c_int32), ("batch", c_int32), ("m_max", c_int32), ("max_iter", c_int32),
                ("rtol", c_double), ("op", c_int32), ("check_every", c_int32), ("precond_steps", c_int32),
                ("streams", c_int32)]


class EngineDesc(ctypes.Structure):
    _fields_ = [("op", c_int32), ("m_max", c_int32), ("check_every", c_int32), ("max_slots", c_int32),
                ("budget_bytes", c_size_t)]


class EngineResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", c_int32), ("iters", c_int32), ("true_rel_res", c_double),
                ("true_rel_res_f", c_double)]


class FcgnoError(RuntimeError):
    pass


_lib = None


def lib():
    """Load the HIP library; fail loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FcgnoError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                         "(hipcc for gfx950); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    L.fcgno_weight_count.argtypes = [POINTER(Arch)]
    L.fcgno_weight_count.restype = c_size_t
    L.fcgno_model_create.argtypes = [POINTER(Arch), POINTER(c_double), c_size_t, POINTER(vp)]
    L.fcgno_model_create.restype = c_int32
    L.fcgno_model_get_weights.argtypes = [vp, POINTER(c_double), c_size_t]
    L.fcgno_model_get_weights.restype = c_int32
    L.fcgno_model_set_weights.argtypes = [vp, POINTER(c_double), c_size_t]
    L.fcgno_model_set_weights.restype = c_int32
    L.fcgno_model_destroy.argtypes = [vp]
    L.fcgno_model_destroy.restype = None
    L.fcgno_solve_workspace_bytes.argtypes = [vp, POINTER(SolveDesc)]
    L.fcgno_solve_workspace_bytes.restype = c_size_t
    L.fcgno_solve.argtypes = [vp, POINTER(SolveDesc), vp, vp, vp, vp, POINTER(c_int32), POINTER(c_int32),
                              POINTER(c_double), POINTER(c_double), POINTER(c_double), vp, c_size_t, vp]
    L.fcgno_solve.restype = c_int32
    L.fcgno_precond_workspace_bytes.argtypes = [vp, c_int32, c_int32, c_int32]
    L.fcgno_precond_workspace_bytes.restype = c_size_t
    L.fcgno_precond_apply.argtypes = [vp, c_int32, c_int32, c_int32, vp, vp, vp, vp, c_size_t, vp]
    L.fcgno_precond_apply.restype = c_int32
    L.fcgno_precond_apply_noalloc.argtypes = [vp, c_int32, c_int32, c_int32, vp, vp, vp, vp]
    L.fcgno_precond_apply_noalloc.restype = c_int32
    L.fcgno_optim_create.argtypes = [vp, c_double, c_double, c_double, c_double, c_double, POINTER(vp)]
    L.fcgno_optim_create.restype = c_int32
    L.fcgno_optim_set_lr.argtypes = [vp, c_double]
    L.fcgno_optim_set_lr.restype = c_int32
    L.fcgno_optim_destroy.argtypes = [vp]
    L.fcgno_optim_destroy.restype = None
    L.fcgno_train_workspace_bytes.argtypes = [vp, c_int32, c_int32, c_int32]
    L.fcgno_train_workspace_bytes.restype = c_size_t
    L.fcgno_op_forward.argtypes = [vp, c_int32, c_int32, c_int32, vp, vp, vp, vp, c_size_t, vp]
    L.fcgno_op_forward.restype = c_int32
    L.fcgno_op_backward.argtypes = [vp, c_int32, c_int32, c_int32, vp, vp, vp, vp, vp, vp, c_size_t, vp]
    L.fcgno_op_backward.restype = c_int32
    L.fcgno_energy_loss_workspace_bytes.argtypes = [c_int32, c_int32]
    L.fcgno_energy_loss_workspace_bytes.restype = c_size_t
    L.fcgno_energy_loss.argtypes = [c_int32, c_int32, vp, vp, vp, vp, vp, vp, c_size_t, vp]
    L.fcgno_energy_loss.restype = c_int32
    L.fcgno_train_step.argtypes = [vp, vp, c_int32, c_int32, c_int32, vp, vp, vp, POINTER(c_double), vp,
                                   c_size_t, vp]
    L.fcgno_train_step.restype = c_int32
    L.fcgno_krylov_samples_workspace_bytes.argtypes = [c_int32, c_int32, c_int32]
    L.fcgno_krylov_samples_workspace_bytes.restype = c_size_t
    L.fcgno_krylov_samples.argtypes = [c_int32, c_int32, c_int32, c_int32, vp, vp, vp, vp, vp, vp, c_size_t, vp]
    L.fcgno_krylov_samples.restype = c_int32
    L.fcgno_residual_samples.argtypes = [c_int32, c_int32, c_int32, vp, vp, vp, vp, vp, vp, c_size_t, vp]
    L.fcgno_residual_samples.restype = c_int32
    L.fcgno_loss.argtypes = [c_int32, c_int32, c_int32, vp, vp, vp, vp, vp, vp, c_size_t, vp]
    L.fcgno_loss.restype = c_int32
    L.fcgno_train_step_loss.argtypes = [vp, vp, c_int32, c_int32, c_int32, c_int32, vp, vp, vp, POINTER(c_double),
                                        vp, c_size_t, vp]
    L.fcgno_train_step_loss.restype = c_int32
    L.fcgno_engine_request_bytes.argtypes = [vp, POINTER(EngineDesc), c_int32, c_int32]
    L.fcgno_engine_request_bytes.restype = c_size_t
    L.fcgno_engine_create.argtypes = [vp, POINTER(EngineDesc), vp, POINTER(vp)]
    L.fcgno_engine_create.restype = c_int32
    L.fcgno_engine_submit.argtypes = [vp, c_int32, vp, vp, vp, c_double, c_int32, POINTER(ctypes.c_int64)]
    L.fcgno_engine_submit.restype = c_int32
    L.fcgno_engine_step.argtypes = [vp, POINTER(c_int32), POINTER(c_int32)]
    L.fcgno_engine_step.restype = c_int32
    L.fcgno_engine_poll.argtypes = [vp, POINTER(EngineResult), c_int32]
    L.fcgno_engine_poll.restype = c_int32
    L.fcgno_engine_destroy.argtypes = [vp]
    L.fcgno_engine_destroy.restype = None
    L.fcgno_profile_enable.argtypes = [c_int32]
    L.fcgno_profile_enable.restype = None
    L.fcgno_profile_reset.argtypes = []
    L.fcgno_profile_reset.restype = None
    L.fcgno_profile_read.argtypes = [c_int32, POINTER(ctypes.c_int64), POINTER(c_double)]
    L.fcgno_profile_read.restype = c_int32
    L.fcgno_last_error.argtypes = []
    L.fcgno_last_error.restype = c_char_p
    _lib = L
    return L


def _check(status, what):
    if status < 0:
        msg = lib().fcgno_last_error().decode(errors="replace")
        raise FcgnoError(f"{what} failed with status {status}: {msg}")
    return status


def _dev_f64(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise FcgnoError(f"{name} must be a device tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise FcgnoError(f"{name} must be contiguous float64")
    return ctypes.c_void_p(t.data_ptr())


def _grid(t, name, lead=1):
    """(B, N) of a field [B][N][N] (lead=1) or [N][N] (lead=0), refusing any
    other shape before a pointer reaches the library."""
    if not isinstance(t, torch.Tensor) or t.dim() != 2 + lead or t.shape[-1] != t.shape[-2]:
        want = "[B][N][N]" if lead else "[N][N]"
        raise FcgnoError(f"{name} must have shape {want}, got {tuple(getattr(t, 'shape', ()))}")
    return (t.shape[0] if lead else 1), t.shape[-1]


def _same(t, shape, name):
    """Refuse a tensor that does not have exactly this shape."""
    if not isinstance(t, torch.Tensor) or tuple(t.shape) != tuple(shape):
        raise FcgnoError(f"{name} must have shape {tuple(shape)}, got {tuple(getattr(t, 'shape', ()))}")


def _nbytes(ws):
    return ws.numel() * ws.element_size()


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes, device, workspace):
    if workspace is not None:
        if _nbytes(workspace) < nbytes:
            raise FcgnoError("workspace too small")
        return workspace
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def weight_count(C, M, L=4, Cin=4):
    a = Arch(L, C, M, Cin)
    return int(lib().fcgno_weight_count(ctypes.byref(a)))


class Model:
    """Operator weights resident on the current device (library-owned)."""

    def __init__(self, weights, C, M, L=4, Cin=4, basis="fourier"):
        self.arch = Arch(L, C, M, Cin, BASIS[basis])
        self.basis = basis
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        self.n_weights = w.size
        h = ctypes.c_void_p()
        _check(lib().fcgno_model_create(ctypes.byref(self.arch),
                                        w.ctypes.data_as(POINTER(c_double)), w.size, ctypes.byref(h)),
               "fcgno_model_create")
        self.handle = h
        self.C, self.M, self.L = C, M, L
        # weights version: bumped whenever the device weights change (set_weights,
        # train_step), so that OperatorFunction never pairs saved activations with
        # other weights; _loaded caches the blob OperatorFunction last loaded
        self._version = 0
        self._loaded = None

    def get_weights(self):
        out = np.empty(self.n_weights, dtype=np.float64)
        _check(lib().fcgno_model_get_weights(self.handle, out.ctypes.data_as(POINTER(c_double)), out.size),
               "fcgno_model_get_weights")
        return out

    def set_weights(self, weights):
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        _check(lib().fcgno_model_set_weights(self.handle, w.ctypes.data_as(POINTER(c_double)), w.size),
               "fcgno_model_set_weights")
        self._version += 1
        self._loaded = None

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().fcgno_model_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_workspace_bytes(model, n, batch, op="bf16", m_max=5, max_iter=300, rtol=1e-6, precond_steps=1):
    d = SolveDesc(n, batch, m_max, max_iter, rtol, OP[op], 0, precond_steps)
    h = model.handle if (model is not None and op not in MODEL_FREE) else None
    return int(lib().fcgno_solve_workspace_bytes(h, ctypes.byref(d)))


def solve(model, k, f, u, op="bf16", m_max=5, max_iter=300, rtol=1e-6, r_out=None, hist=True,
          check_every=0, workspace=None, stream=None, precond_steps=1, streams=0):
    """Run Algorithm 1 on a batch: k [B][N+2][N+2], f [B][N][N], u [B][N][N]
    (in: u0, out: u_iter), all float64 device tensors.  op: a neural-operator
    precision, "identity" (CG) or a classical preconditioner ("jacobi",
    "sgs_rb") applied precond_steps times.  streams > 1 splits the batch into
    that many sub-batches on library-owned streams (same bits, overlapped
    kernels).  Returns a dict with numpy arrays iters, status, true_rel_res
    true_rel_res_f (||f - A u|| / ||f||) and (if hist) hist [B][max_iter+1]."""
    B, N = _grid(f, "f")
    if tuple(k.shape) != (B, N + 2, N + 2) or tuple(u.shape) != (B, N, N):
        raise FcgnoError("shape mismatch: k [B][N+2][N+2], f and u [B][N][N]")
    if r_out is not None and tuple(r_out.shape) != (B, N, N):
        raise FcgnoError("shape mismatch: r_out [B][N][N]")
    d = SolveDesc(N, B, m_max, max_iter, rtol, OP[op], check_every, precond_steps, streams)
    h = model.handle if (model is not None and op not in MODEL_FREE) else None
    nbytes = lib().fcgno_solve_workspace_bytes(h, ctypes.byref(d))
    if nbytes == 0:
        raise FcgnoError("invalid solve descriptor: " + lib().fcgno_last_error().decode(errors="replace"))
    ws = _workspace(nbytes, f.device, workspace)
    iters = np.zeros(B, dtype=np.int32)
    status = np.zeros(B, dtype=np.int32)
    tres = np.zeros(B, dtype=np.float64)
    tresf = np.zeros(B, dtype=np.float64)
    hh = np.full((B, max_iter + 1), np.nan) if hist else None
    rc = lib().fcgno_solve(
        h, ctypes.byref(d), _dev_f64(k, "k"), _dev_f64(f, "f"), _dev_f64(u, "u"),
        _dev_f64(r_out, "r_out") if r_out is not None else None,
        iters.ctypes.data_as(POINTER(c_int32)), status.ctypes.data_as(POINTER(c_int32)),
        hh.ctypes.data_as(POINTER(c_double)) if hist else None,
        tres.ctypes.data_as(POINTER(c_double)), tresf.ctypes.data_as(POINTER(c_double)),
        ctypes.c_void_p(ws.data_ptr()), _nbytes(ws), _stream(stream))
    _check(rc, "fcgno_solve")
    out = {"iters": iters, "status": status, "true_rel_res": tres, "true_rel_res_f": tresf, "rc": rc}
    if hist:
        out["hist"] = hh
    return out


def precond_apply(model, k, r, op="bf16", w=None, workspace=None, stream=None):
    """w = B(r; theta) for a batch (asynchronous on the stream)."""
    B, N = _grid(r, "r")
    if tuple(k.shape) != (B, N + 2, N + 2):
        raise FcgnoError("shape mismatch: k [B][N+2][N+2], r [B][N][N]")
    if w is not None and tuple(w.shape) != (B, N, N):
        raise FcgnoError("shape mismatch: w [B][N][N]")
    if w is None:
        w = torch.empty_like(r)
    nbytes = lib().fcgno_precond_workspace_bytes(model.handle, N, B, OP[op])
    if nbytes == 0:
        raise FcgnoError("invalid operator application (need 2*modes <= N and a matrix precision)")
    ws = _workspace(nbytes, r.device, workspace)
    _check(lib().fcgno_precond_apply(model.handle, N, B, OP[op], _dev_f64(k, "k"), _dev_f64(r, "r"),
                                     _dev_f64(w, "w"), ctypes.c_void_p(ws.data_ptr()), _nbytes(ws),
                                     _stream(stream)), "fcgno_precond_apply")
    return w


NOALLOC_SCRATCH_BYTES = 64 << 20


def precond_apply_noalloc(model, k, r, op="bf16", w=None, stream=None):
    """w = B(r; theta) like precond_apply, with the library's static scratch
    array instead of a workspace (no device allocation inside the call; the
    output w is allocated here unless given)."""
    B, N = _grid(r, "r")
    _same(k, (B, N + 2, N + 2), "k")
    if w is None:
        w = torch.empty_like(r)
    _same(w, (B, N, N), "w")
    _check(lib().fcgno_precond_apply_noalloc(model.handle, N, B, OP[op], _dev_f64(k, "k"), _dev_f64(r, "r"),
                                             _dev_f64(w, "w"), _stream(stream)), "fcgno_precond_apply_noalloc")
    return w


PROFILE_KERNELS = {"layer": 0, "spectral": 1, "dir": 2, "wdots": 3, "update": 4, "rowdft": 5,
                   "train_fwd": 6, "train_bwd": 7, "layer_feat": 8, "layer_proj": 9}


def profile_enable(on=True, kernels=None):
    """Event timing of the kernel families named in ``kernels`` (all if None)."""
    if not on:
        mask = 0
    elif kernels is None:
        mask = (1 << len(PROFILE_KERNELS)) - 1
    else:
        mask = 0
        for name in kernels:
            mask |= 1 << PROFILE_KERNELS[name]
    lib().fcgno_profile_enable(mask)


def profile_reset():
    lib().fcgno_profile_reset()


def profile_read(kernel):
    """(launches, total milliseconds) of a kernel family since the last reset."""
    n = ctypes.c_int64(0)
    ms = c_double(0.0)
    _check(lib().fcgno_profile_read(PROFILE_KERNELS[kernel], ctypes.byref(n), ctypes.byref(ms)),
           "fcgno_profile_read")
    return int(n.value), float(ms.value)


# ---------------------------------------------------------------------------
# Training
# ---------------------------------------------------------------------------

class Optim:
    """AdamW state on the device for one model (decoupled weight decay)."""

    def __init__(self, model, lr=1e-3, weight_decay=1e-2, beta1=0.9, beta2=0.999, eps=1e-8):
        h = ctypes.c_void_p()
        _check(lib().fcgno_optim_create(model.handle, lr, weight_decay, beta1, beta2, eps, ctypes.byref(h)),
               "fcgno_optim_create")
        self.handle = h
        self.lr = lr

    def set_lr(self, lr):
        _check(lib().fcgno_optim_set_lr(self.handle, lr), "fcgno_optim_set_lr")
        self.lr = lr

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().fcgno_optim_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def train_workspace(model, n, batch, op="fp32", device=None):
    nbytes = lib().fcgno_train_workspace_bytes(model.handle, n, batch, OP[op])
    if nbytes == 0:
        raise FcgnoError("invalid training shape: " + lib().fcgno_last_error().decode(errors="replace"))
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device or torch.device("cuda"))


def op_forward(model, k, r, op="fp64", workspace=None, stream=None):
    """w = B(r), keeping the activations for op_backward in the workspace."""
    B, N = _grid(r, "r")
    _same(k, (B, N + 2, N + 2), "k")
    ws = workspace if workspace is not None else train_workspace(model, N, B, op, r.device)
    w = torch.empty_like(r)
    _check(lib().fcgno_op_forward(model.handle, N, B, OP[op], _dev_f64(k, "k"), _dev_f64(r, "r"),
                                  _dev_f64(w, "w"), ctypes.c_void_p(ws.data_ptr()), _nbytes(ws), _stream(stream)),
           "fcgno_op_forward")
    return w, ws


def op_backward(model, k, r, grad_w, ws, op="fp64", stream=None, input_grad=False):
    """Gradient of sum <grad_w, B(r)> with respect to the weight blob (device
    float64); with input_grad, also with respect to r: returns (g, g_r)."""
    B, N = _grid(r, "r")
    _same(k, (B, N + 2, N + 2), "k")
    grad_w = grad_w.contiguous()
    _same(grad_w, (B, N, N), "grad_w")
    g = torch.empty(model.n_weights, dtype=torch.float64, device=r.device)
    gr = torch.empty_like(r) if input_grad else None
    _check(lib().fcgno_op_backward(model.handle, N, B, OP[op], _dev_f64(k, "k"), _dev_f64(r, "r"),
                                   _dev_f64(grad_w, "grad_w"), _dev_f64(g, "grad"),
                                   _dev_f64(gr, "grad_r") if input_grad else None,
                                   ctypes.c_void_p(ws.data_ptr()), _nbytes(ws), _stream(stream)),
           "fcgno_op_backward")
    return (g, gr) if input_grad else g


LOSS = {"energy": 0, "l2": 1}


def energy_loss(k, w, e, grad=True, stream=None, kind="energy"):
    """Per-system ||w-e||/||e|| in the energy norm (or the Euclidean norm with
    kind="l2") and (optionally) the gradient of their mean."""
    B, N = _grid(w, "w")
    _same(k, (B, N + 2, N + 2), "k")
    _same(e, (B, N, N), "e")
    nbytes = lib().fcgno_energy_loss_workspace_bytes(N, B)
    if nbytes == 0:
        raise FcgnoError("invalid loss shape: " + lib().fcgno_last_error().decode(errors="replace"))
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=w.device)
    loss = torch.empty(B, dtype=torch.float64, device=w.device)
    g = torch.empty_like(w) if grad else None
    _check(lib().fcgno_loss(LOSS[kind], N, B, _dev_f64(k, "k"), _dev_f64(w, "w"), _dev_f64(e, "e"),
                            _dev_f64(loss, "loss"), _dev_f64(g, "grad") if grad else None,
                            ctypes.c_void_p(ws.data_ptr()), _nbytes(ws), _stream(stream)), "fcgno_loss")
    return loss, g


def train_step(model, opt, k, r, e, op="fp32", workspace=None, stream=None, return_loss=True, loss="energy"):
    """One AdamW step on the energy-norm loss (or loss="l2"); returns the
    batch-mean loss (which synchronises the stream), or None with
    ``return_loss=False``."""
    B, N = _grid(r, "r")
    _same(k, (B, N + 2, N + 2), "k")
    _same(e, (B, N, N), "e")
    ws = workspace if workspace is not None else train_workspace(model, N, B, op, r.device)
    out = c_double(0.0)
    model._version += 1    # AdamW updates the device weights in place
    model._loaded = None
    _check(lib().fcgno_train_step_loss(model.handle, opt.handle, N, B, OP[op], LOSS[loss], _dev_f64(k, "k"),
                                       _dev_f64(r, "r"), _dev_f64(e, "e"),
                                       ctypes.byref(out) if return_loss else None,
                                       ctypes.c_void_p(ws.data_ptr()), _nbytes(ws), _stream(stream)),
           "fcgno_train_step_loss")
    return float(out.value) if return_loss else None


def residual_samples(k, f, u, max_iter=None, stream=None):
    """(f - A u, A^-1 f - u) for a batch of random right-hand sides and points;
    returns two device tensors [B][N][N]."""
    B, N = _grid(f, "f")
    _same(k, (B, N + 2, N + 2), "k")
    _same(u, (B, N, N), "u")
    max_iter = max_iter or max(20 * N, 2000)
    nbytes = lib().fcgno_krylov_samples_workspace_bytes(N, B, max_iter)
    if nbytes == 0:
        raise FcgnoError("invalid sample shape: " + lib().fcgno_last_error().decode(errors="replace"))
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=f.device)
    r = torch.empty((B, N, N), dtype=torch.float64, device=f.device)
    e = torch.empty_like(r)
    _check(lib().fcgno_residual_samples(N, B, max_iter, _dev_f64(k, "k"), _dev_f64(f, "f"), _dev_f64(u, "u"),
                                        _dev_f64(r, "r"), _dev_f64(e, "e"), ctypes.c_void_p(ws.data_ptr()),
                                        _nbytes(ws), _stream(stream)), "fcgno_residual_samples")
    return r, e


def krylov_samples(k, f, u0, m_iter=100, max_iter=None, stream=None):
    """(r_i, e_i = u* - u_i), i = 1..m_iter, of conjugate gradients from u0;
    returns two device tensors [B][m_iter][N][N]."""
    B, N = _grid(f, "f")
    _same(k, (B, N + 2, N + 2), "k")
    _same(u0, (B, N, N), "u0")
    max_iter = max_iter or max(20 * N, 2000)
    nbytes = lib().fcgno_krylov_samples_workspace_bytes(N, B, max(max_iter, m_iter))
    if nbytes == 0:
        raise FcgnoError("invalid sample shape: " + lib().fcgno_last_error().decode(errors="replace"))
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=f.device)
    r = torch.empty((B, m_iter, N, N), dtype=torch.float64, device=f.device)
    e = torch.empty_like(r)
    _check(lib().fcgno_krylov_samples(N, B, m_iter, max_iter, _dev_f64(k, "k"), _dev_f64(f, "f"),
                                      _dev_f64(u0, "u0"), _dev_f64(r, "r"), _dev_f64(e, "e"),
                                      ctypes.c_void_p(ws.data_ptr()), _nbytes(ws), _stream(stream)),
           "fcgno_krylov_samples")
    return r, e


class Engine:
    """Continuous-batching solve engine (fcgno_engine_*).  Requests are single
    systems of any grid size; k, f, u stay referenced until the request is
    reported by poll()."""

    def __init__(self, model, op="bf16", m_max=5, check_every=8, max_slots=64, budget_bytes=8 << 30,
                 stream=None):
        self.model = model
        self.desc = EngineDesc(OP[op], m_max, check_every, max_slots, int(budget_bytes))
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        _check(lib().fcgno_engine_create(model.handle if (model is not None and op != "identity") else None,
                                         ctypes.byref(self.desc), ctypes.c_void_p(self._stream.cuda_stream),
                                         ctypes.byref(h)), "fcgno_engine_create")
        self.handle = h
        self._held = {}

    def request_bytes(self, n, max_iter):
        m = self.model.handle if self.model is not None else None
        return int(lib().fcgno_engine_request_bytes(m, ctypes.byref(self.desc), n, max_iter))

    def submit(self, k, f, u, rtol=1e-6, max_iter=None):
        """Queue one system: k [N+2][N+2], f and u [N][N] float64 device tensors
        (u: in u0, out the iterate).  Returns the request id."""
        _, N = _grid(f, "f", lead=0)
        if tuple(k.shape) != (N + 2, N + 2) or tuple(u.shape) != (N, N):
            raise FcgnoError("shape mismatch: k [N+2][N+2], f and u [N][N]")
        max_iter = max_iter or max(2 * N, 300)
        rid = ctypes.c_int64(0)
        _check(lib().fcgno_engine_submit(self.handle, N, _dev_f64(k, "k"), _dev_f64(f, "f"), _dev_f64(u, "u"),
                                         rtol, max_iter, ctypes.byref(rid)), "fcgno_engine_submit")
        self._held[rid.value] = (k, f, u)
        return rid.value

    def step(self):
        """Admit, advance every group by check_every iterations, release stopped
        requests.  Returns (active, queued)."""
        a, q = c_int32(0), c_int32(0)
        _check(lib().fcgno_engine_step(self.handle, ctypes.byref(a), ctypes.byref(q)), "fcgno_engine_step")
        return a.value, q.value

    def poll(self, max_results=4096):
        buf = (EngineResult * max_results)()
        n = lib().fcgno_engine_poll(self.handle, buf, max_results)
        out = []
        for i in range(n):
            r = buf[i]
            self._held.pop(r.id, None)
            out.append({"id": r.id, "status": r.status, "iters": r.iters, "true_rel_res": r.true_rel_res,
                        "true_rel_res_f": r.true_rel_res_f})
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().fcgno_engine_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class OperatorFunction(torch.autograd.Function):
    """w = B(r; theta) with the hand-written HIP backward for theta.

    ``weights`` is the float64 blob; it is loaded into ``model`` when it differs
    from the blob this function last loaded there (or the model's weights have
    changed since).  If the model's weights change between forward and
    backward, backward reloads the forward's blob first, so the gradient always
    pairs the saved activations with the weights that produced them.
    Gradients flow to the weights and to r (not to k)."""

    @staticmethod
    def forward(ctx, weights, model, k, r, op="fp64"):
        wh = weights.detach().to("cpu", torch.float64).contiguous().numpy()
        if model._loaded is None or not np.array_equal(model._loaded, wh):
            model.set_weights(wh)
            model._loaded = wh.copy()
        w, ws = op_forward(model, k, r, op)
        ctx.model, ctx.op, ctx.ws = model, op, ws
        ctx.version, ctx.wh = model._version, model._loaded
        ctx.save_for_backward(k, r)
        ctx.wdev = weights.device
        return w

    @staticmethod
    def backward(ctx, grad_w):
        k, r = ctx.saved_tensors
        if ctx.model._version != ctx.version:
            ctx.model.set_weights(ctx.wh)
            ctx.model._loaded = ctx.wh
        if ctx.needs_input_grad[3]:
            g, gr = op_backward(ctx.model, k, r, grad_w, ctx.ws, ctx.op, input_grad=True)
        else:
            g, gr = op_backward(ctx.model, k, r, grad_w, ctx.ws, ctx.op), None
        return g.to(ctx.wdev), None, None, gr, None
