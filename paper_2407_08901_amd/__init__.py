"""SPPC eigensolver on one MI355X: thin ctypes binding of libsppc.so (include/sppc.h).

The functions below carry the C ABI's names and only marshal arguments: torch
tensors on the GPU are passed as device pointers, the current torch stream as the
HIP stream.  Every step of the method runs in the library's HIP kernels; there is
no CPU fallback.  If the library is missing the import of `lib()` fails loudly.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional, Sequence

import torch  # loads the HIP runtime first, so libsppc.so binds to the same one

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsppc.so")

SPPC_OK, SPPC_E_ARG, SPPC_E_HIP, SPPC_E_NOMEM, SPPC_E_SINGULAR_E0, SPPC_E_BREAKDOWN, SPPC_E_NOCONV, \
    SPPC_E_NAN = range(8)
SPPC_F64, SPPC_F32 = 0, 1
SPPC_PREC_FP64, SPPC_PREC_MIXED = 0, 1
SPPC_CORR_PERTURBATIVE, SPPC_CORR_JACOBI, SPPC_CORR_MPNN, SPPC_CORR_SMALL, SPPC_CORR_RMMDIIS = 0, 1, 2, 3, 4
SPPC_SHIFT_E0, SPPC_SHIFT_RITZ = 0, 1

STATUS_NAMES = {0: "SPPC_OK", 1: "SPPC_E_ARG", 2: "SPPC_E_HIP", 3: "SPPC_E_NOMEM",
                4: "SPPC_E_SINGULAR_E0", 5: "SPPC_E_BREAKDOWN", 6: "SPPC_E_NOCONV", 7: "SPPC_E_NAN"}

EXPORTS = ("sppc_default_opts", "sppc_workspace_size", "sppc_setup", "sppc_spmm", "sppc_spmm_upper", "sppc_spmm_noalloc", "sppc_correct", "sppc_rayleigh_ritz",
           "sppc_solve", "sppc_get", "sppc_last_error", "sppc_setup_error", "sppc_destroy",
           "sppc_release_cached_memory", "sppc_set_memory_cache", "sppc_mpnn_set_weights", "sppc_mpnn_eval", "sppc_mpnn_train_step", "sppc_mpnn_target")
SPPC_MPNN_NPARAM = 289


class sppc_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr_dev", ctypes.c_void_p),
                ("col_dev", ctypes.c_void_p), ("val_dev", ctypes.c_void_p), ("val_type", ctypes.c_int)]


class sppc_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("p_switch", ctypes.c_int),
                ("max_cont", ctypes.c_int), ("m_max", ctypes.c_int), ("n_deflate", ctypes.c_int),
                ("tau_drop", ctypes.c_double), ("inner_tol", ctypes.c_double), ("h0_tol", ctypes.c_double),
                ("precision", ctypes.c_int), ("precond", ctypes.c_int), ("final_check", ctypes.c_int),
                ("verbose", ctypes.c_int), ("panel_width", ctypes.c_int), ("refine_precond", ctypes.c_int),
                ("precond_tol", ctypes.c_double), ("auto_switch", ctypes.c_int), ("corr_shift", ctypes.c_int), ("pair_index", ctypes.c_int),
                ("rmm_precond", ctypes.c_int)]


class sppc_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("cont_steps", ctypes.c_int), ("refine_steps", ctypes.c_int),
                ("mpnn_steps", ctypes.c_int), ("n_spmv", ctypes.c_int64),
                ("spmm_calls", ctypes.c_int64), ("spmm_cols", ctypes.c_int64),
                ("basis_size", ctypes.c_int), ("cg_iterations", ctypes.c_int), ("h0_iterations", ctypes.c_int),
                ("converged", ctypes.c_int), ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("t_spmm_ms", ctypes.c_double), ("t_small_ms", ctypes.c_double), ("t_ortho_ms", ctypes.c_double),
                ("t_rr_ms", ctypes.c_double), ("spmm_alg_bytes", ctypes.c_double), ("t_h0_ms", ctypes.c_double),
                ("mpnn_fallbacks", ctypes.c_int), ("workspace_peak", ctypes.c_int64),
                ("rmm_iterations", ctypes.c_int), ("rmm_handover", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SPPCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if it was not built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsppc.so is not built: run `python -m paper_2407_08901_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, c_int, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        L.sppc_default_opts.argtypes = [ctypes.POINTER(sppc_opts)]
        L.sppc_setup.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(sppc_csr), ctypes.POINTER(i64), c_int, c_int,
                                 c_int, ctypes.POINTER(sppc_opts), vp, ctypes.c_size_t, vp]
        L.sppc_workspace_size.argtypes = [ctypes.POINTER(sppc_csr), ctypes.POINTER(i64), c_int, c_int, c_int,
                                          ctypes.POINTER(sppc_opts), ctypes.POINTER(ctypes.c_size_t)]
        L.sppc_set_memory_cache.argtypes = [ctypes.c_size_t]
        L.sppc_set_memory_cache.restype = ctypes.c_size_t
        L.sppc_spmm.argtypes = [vp, vp, c_int, vp, c_int]
        L.sppc_spmm_noalloc.argtypes = [vp, vp, c_int, vp, c_int]
        L.sppc_spmm_upper.argtypes = [ctypes.POINTER(sppc_csr), vp, c_int, vp, c_int, vp]
        L.sppc_correct.argtypes = [vp, c_int, dp]
        L.sppc_rayleigh_ritz.argtypes = [vp, dp, dp, ctypes.POINTER(c_int)]
        L.sppc_solve.argtypes = [vp, dp, vp, dp, ctypes.POINTER(sppc_stats)]
        L.sppc_get.argtypes = [vp, c_int, vp, i64]
        L.sppc_last_error.argtypes = [vp]
        L.sppc_last_error.restype = ctypes.c_char_p
        L.sppc_setup_error.restype = ctypes.c_char_p
        L.sppc_destroy.argtypes = [vp]
        L.sppc_destroy.restype = None
        L.sppc_release_cached_memory.argtypes = []
        L.sppc_release_cached_memory.restype = ctypes.c_size_t
        fp = ctypes.POINTER(ctypes.c_float)
        L.sppc_mpnn_set_weights.argtypes = [vp, fp]
        L.sppc_mpnn_eval.argtypes = [vp, fp, c_int, vp, vp, dp, vp, c_int, vp, vp, dp, dp, c_int]
        L.sppc_mpnn_train_step.argtypes = [vp, vp, c_int, vp, vp, dp, vp, c_int, vp, ctypes.c_float, c_int, dp]
        L.sppc_mpnn_target.argtypes = [vp, c_int, vp, c_int, vp, vp]
        for name in ("sppc_default_opts", "sppc_workspace_size", "sppc_setup", "sppc_spmm", "sppc_spmm_upper", "sppc_spmm_noalloc", "sppc_correct", "sppc_rayleigh_ritz",
                     "sppc_solve", "sppc_get", "sppc_mpnn_set_weights", "sppc_mpnn_eval", "sppc_mpnn_train_step",
                     "sppc_mpnn_target"):
            getattr(L, name).restype = c_int
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != SPPC_OK:
        L = lib()
        msg = (L.sppc_last_error(ctx) if ctx else L.sppc_setup_error()) or b""
        raise SPPCError(status, msg.decode(errors="replace"))


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def sppc_default_opts(**kw) -> sppc_opts:
    o = sppc_opts()
    _check(lib().sppc_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


_LIVE = weakref.WeakSet()  # contexts not destroyed yet
_EXITING = False


@atexit.register
def _destroy_live_contexts():
    # Contexts still alive at interpreter exit are destroyed here, while the HIP runtime (and a
    # profiler's tool library) is still up: a destroy run later from garbage collection during
    # interpreter teardown would call hipStreamSynchronize/hipFree after they were finalised.
    global _EXITING
    for ctx in list(_LIVE):
        try:
            sppc_destroy(ctx)
        except Exception:
            pass
    _EXITING = True


class Context:
    """Owns an sppc_ctx and keeps the device arrays it borrows (and its workspace) alive."""

    def __init__(self, handle, n, k, keep, stream):
        self.handle = handle
        self.n = n
        self.k = k
        self._keep = keep
        self.stream = stream
        _LIVE.add(self)

    def __del__(self):
        if _EXITING:
            return
        try:
            sppc_destroy(self)
        except Exception:
            pass


def _csr(row_ptr, col, val):
    for t, dt in ((row_ptr, torch.int64), (col, torch.int32)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError("row_ptr must be int64, col int32; contiguous GPU tensors")
    if not val.is_cuda or val.dtype not in (torch.float64, torch.float32) or not val.is_contiguous():
        raise TypeError("val must be a contiguous float64/float32 GPU tensor")
    n = row_ptr.numel() - 1
    return n, sppc_csr(n, col.numel(), row_ptr.data_ptr(), col.data_ptr(), val.data_ptr(),
                       SPPC_F32 if val.dtype == torch.float32 else SPPC_F64)


def sppc_workspace_size(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, level_offsets: Sequence[int],
                        n_small_levels: int, k: int, opts: Optional[sppc_opts] = None) -> int:
    """Bytes of device workspace for sppc_setup + sppc_solve of this problem with these options."""
    n, H = _csr(row_ptr, col, val)
    lo = (ctypes.c_int64 * len(level_offsets))(*[int(x) for x in level_offsets])
    out = ctypes.c_size_t()
    _check(lib().sppc_workspace_size(ctypes.byref(H), lo, len(level_offsets) - 1, n_small_levels, k,
                                     ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)))
    return int(out.value)


def workspace_tensor(nbytes: int) -> torch.Tensor:
    """A device workspace of nbytes from PyTorch's allocator."""
    return torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")


def sppc_setup(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, level_offsets: Sequence[int],
               n_small_levels: int, k: int, opts: Optional[sppc_opts] = None, stream=None,
               workspace: Optional[torch.Tensor] = None) -> Context:
    """Upper-triangular CSR of H on the GPU (int64 row_ptr, int32 col, float64/float32 val).
    workspace: a uint8 GPU tensor of at least sppc_workspace_size bytes that every device array of
    the context comes from (None: the library allocates)."""
    n, H = _csr(row_ptr, col, val)
    wp, wb = None, 0
    if workspace is not None:
        if not workspace.is_cuda or not workspace.is_contiguous():
            raise TypeError("workspace must be a contiguous GPU tensor")
        wp, wb = ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
    lo = (ctypes.c_int64 * len(level_offsets))(*[int(x) for x in level_offsets])
    h = ctypes.c_void_p()
    st = stream if stream is not None else torch.cuda.current_stream()
    status = lib().sppc_setup(ctypes.byref(h), ctypes.byref(H), lo, len(level_offsets) - 1, n_small_levels, k,
                              ctypes.byref(opts) if opts is not None else None, wp, wb, _stream_handle(st))
    _check(status)
    return Context(h, n, k, (row_ptr, col, val, workspace), st)


def sppc_spmm(ctx: Context, X: torch.Tensor, Y: torch.Tensor) -> None:
    """Y = H X; X row-major n x b (float64 or float32), Y float64 n x b."""
    if X.dim() != 2 or Y.shape != X.shape or X.shape[0] != ctx.n or Y.dtype != torch.float64:
        raise ValueError("X, Y must be n x b, Y float64")
    if not (X.is_contiguous() and Y.is_contiguous() and X.is_cuda and Y.is_cuda):
        raise ValueError("X, Y must be contiguous GPU tensors")
    xt = SPPC_F32 if X.dtype == torch.float32 else SPPC_F64
    _check(lib().sppc_spmm(ctx.handle, ctypes.c_void_p(X.data_ptr()), xt, ctypes.c_void_p(Y.data_ptr()),
                           X.shape[1]), ctx.handle)


def sppc_spmm_upper(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, X: torch.Tensor,
                    Y: torch.Tensor, stream=None) -> None:
    """Y = H X from the upper-triangular CSR alone (no context); X row-major n x b (float64 or
    float32), Y float64 n x b."""
    n, H = _csr(row_ptr, col, val)
    if X.dim() != 2 or Y.shape != X.shape or X.shape[0] != n or Y.dtype != torch.float64:
        raise ValueError("X, Y must be n x b, Y float64")
    if not (X.is_contiguous() and Y.is_contiguous() and X.is_cuda and Y.is_cuda):
        raise ValueError("X, Y must be contiguous GPU tensors")
    xt = SPPC_F32 if X.dtype == torch.float32 else SPPC_F64
    _check(lib().sppc_spmm_upper(ctypes.byref(H), ctypes.c_void_p(X.data_ptr()), xt, ctypes.c_void_p(Y.data_ptr()),
                                 X.shape[1], _stream_handle(stream)))


def sppc_spmm_noalloc(ctx: Context, X: torch.Tensor, Y: torch.Tensor) -> None:
    """Y = H X as sppc_spmm, allocating nothing (the padded copy of X goes to the library's static
    device scratch)."""
    if X.dim() != 2 or Y.shape != X.shape or X.shape[0] != ctx.n or Y.dtype != torch.float64:
        raise ValueError("X, Y must be n x b, Y float64")
    if not (X.is_contiguous() and Y.is_contiguous() and X.is_cuda and Y.is_cuda):
        raise ValueError("X, Y must be contiguous GPU tensors")
    xt = SPPC_F32 if X.dtype == torch.float32 else SPPC_F64
    _check(lib().sppc_spmm_noalloc(ctx.handle, ctypes.c_void_p(X.data_ptr()), xt, ctypes.c_void_p(Y.data_ptr()),
                                   X.shape[1]), ctx.handle)


def sppc_correct(ctx: Context, kind: int = SPPC_CORR_PERTURBATIVE, shifts=None) -> None:
    """shifts: k per-pair shifts in place of E^(0) (perturbative corrections only), or None."""
    sh = None
    if shifts is not None:
        if len(shifts) != ctx.k:
            raise ValueError("one shift per wanted pair")
        sh = (ctypes.c_double * ctx.k)(*[float(x) for x in shifts])
    _check(lib().sppc_correct(ctx.handle, kind, sh), ctx.handle)


def sppc_rayleigh_ritz(ctx: Context):
    th = (ctypes.c_double * ctx.k)()
    rr = (ctypes.c_double * ctx.k)()
    added = ctypes.c_int()
    status = lib().sppc_rayleigh_ritz(ctx.handle, th, rr, ctypes.byref(added))
    if status not in (SPPC_OK, SPPC_E_BREAKDOWN):
        _check(status, ctx.handle)
    return list(th), list(rr), added.value


def sppc_solve(ctx: Context, want_vectors: bool = True):
    """Returns (evals list, evecs tensor n x k or None, rrn list, stats dict, status)."""
    ev = (ctypes.c_double * ctx.k)()
    rr = (ctypes.c_double * ctx.k)()
    st = sppc_stats()
    Z = torch.empty((ctx.n, ctx.k), dtype=torch.float64, device="cuda") if want_vectors else None
    status = lib().sppc_solve(ctx.handle, ev, ctypes.c_void_p(Z.data_ptr()) if Z is not None else None, rr,
                              ctypes.byref(st))
    if status not in (SPPC_OK, SPPC_E_NOCONV):
        _check(status, ctx.handle)
    return list(ev), Z, list(rr), st.as_dict(), status


def sppc_get(ctx: Context, what: int, count: int, device: bool = False):
    """Inspection copies (see sppc.h).  device=True for the device items (3, 4, 5, 9)."""
    if device:
        out = torch.empty(max(count, 1), dtype=torch.float64, device="cuda")
        _check(lib().sppc_get(ctx.handle, what, ctypes.c_void_p(out.data_ptr()), count), ctx.handle)
        return out[:count]
    buf = (ctypes.c_double * max(count, 1))()
    _check(lib().sppc_get(ctx.handle, what, buf, count), ctx.handle)
    return list(buf)[:count]


def _fptr(w):
    import numpy as np
    a = np.ascontiguousarray(w, dtype=np.float32)
    if a.size != SPPC_MPNN_NPARAM:
        raise ValueError("the network has %d parameters" % SPPC_MPNN_NPARAM)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def sppc_mpnn_set_weights(ctx: Context, w) -> None:
    a, p = _fptr(w)
    _check(lib().sppc_mpnn_set_weights(ctx.handle, p), ctx.handle)


def _basis(ctx: Context, Q: Optional[torch.Tensor]):
    if Q is None:
        return None, 0
    if Q.dim() != 2 or Q.shape[0] != ctx.n or Q.dtype != torch.float64 or not Q.is_contiguous():
        raise ValueError("Q must be a contiguous float64 n x m tensor")
    return _dptr(Q), Q.shape[1]


def sppc_mpnn_eval(ctx: Context, w, R: torch.Tensor, X: torch.Tensor, theta, E: Optional[torch.Tensor] = None,
                   want_output: bool = True, f64: bool = False, Q: Optional[torch.Tensor] = None):
    """Returns (T or None, loss list or None, grad list or None).  R, X, E: n x S float64 GPU;
    Q: optional n x m basis for the output projection."""
    a, p = _fptr(w)
    S = R.shape[1]
    for t in (R, X, E):
        if t is not None and (t.shape != (ctx.n, S) or t.dtype != torch.float64 or not t.is_contiguous()):
            raise ValueError("R, X, E must be contiguous float64 n x S")
    qp, m = _basis(ctx, Q)
    T = torch.empty_like(R) if want_output else None
    th = (ctypes.c_double * S)(*[float(x) for x in theta])
    loss = (ctypes.c_double * S)() if E is not None else None
    grad = (ctypes.c_double * SPPC_MPNN_NPARAM)() if E is not None else None
    _check(lib().sppc_mpnn_eval(ctx.handle, p, S, _dptr(R), _dptr(X), th, qp, m, _dptr(E), _dptr(T), loss, grad,
                                1 if f64 else 0), ctx.handle)
    return T, (list(loss) if loss is not None else None), (list(grad) if grad is not None else None)


def sppc_mpnn_train_step(ctx: Context, state: torch.Tensor, R, X, theta, E, lr: float, step: int,
                         Q: Optional[torch.Tensor] = None) -> float:
    """state: float32 GPU tensor [4 * 289] (weights, Adam moments, bfloat16 copy)."""
    S = R.shape[1]
    qp, m = _basis(ctx, Q)
    th = (ctypes.c_double * S)(*[float(x) for x in theta])
    loss = ctypes.c_double()
    _check(lib().sppc_mpnn_train_step(ctx.handle, ctypes.c_void_p(state.data_ptr()), S, _dptr(R), _dptr(X), th,
                                      qp, m, _dptr(E), ctypes.c_float(lr), step, ctypes.byref(loss)), ctx.handle)
    return loss.value


def sppc_mpnn_target(ctx: Context, Q: torch.Tensor, Psi: torch.Tensor) -> torch.Tensor:
    """E = (I - Q Q^T) Psi on the GPU."""
    qp, m = _basis(ctx, Q)
    E = torch.empty_like(Psi)
    _check(lib().sppc_mpnn_target(ctx.handle, Psi.shape[1], qp, m, _dptr(Psi), _dptr(E)), ctx.handle)
    return E


def sppc_destroy(ctx: Context) -> None:
    if ctx is not None and ctx.handle:
        lib().sppc_destroy(ctx.handle)
        ctx.handle = None


def sppc_set_memory_cache(bytes_per_device: int) -> int:
    """Enables (bytes > 0) or disables (0) the library's cache of freed device blocks; returns the
    previous limit."""
    return int(lib().sppc_set_memory_cache(int(bytes_per_device)))


def sppc_release_cached_memory() -> int:
    """Frees the library's cached device memory; returns the bytes freed."""
    return int(lib().sppc_release_cached_memory())


def upload(A, dtype=torch.float64, device="cuda"):
    """Upper CSR arrays (numpy) -> GPU tensors (row_ptr int64, col int32, val dtype)."""
    import numpy as np
    rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int64)).to(device)
    col = torch.from_numpy(np.ascontiguousarray(A.col, dtype=np.int32)).to(device)
    val = torch.from_numpy(np.ascontiguousarray(A.val)).to(device=device, dtype=dtype)
    return rp, col, val
