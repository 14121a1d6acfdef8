"""Python binding of libpasm (include/pasm.h): argument marshalling only.

Every computation of the eigensolver runs in the HIP library; this module
converts arguments, raises on error statuses and uses PyTorch only for device
memory (tensors whose pointers are passed to the library) and for the current
HIP stream.  If the library has not been built, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpasm.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "pasm.h")

PASM_OK, PASM_E_INVALID, PASM_E_NOMEM, PASM_E_DEVICE, PASM_E_STATE, PASM_E_NOTCONV, PASM_E_BREAKDOWN = range(7)
PASM_FP64, PASM_MIXED = 0, 1
PASM_JACOBI, PASM_CHEBYSHEV, PASM_LEARNED, PASM_CG = 0, 1, 2, 3
PASM_OP_STIFFNESS, PASM_OP_MASS = 0, 1


class PasmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pasm status {status}: {msg}")
        self.status = status


class pasm_domain(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int)]


class pasm_coefficients(ctypes.Structure):
    _fields_ = [("kappa", ctypes.POINTER(ctypes.c_double)),
                ("potential", ctypes.POINTER(ctypes.c_double)),
                ("n_elements", ctypes.c_size_t),
                ("tensor", ctypes.POINTER(ctypes.c_double))]


class pasm_instance(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("coef", pasm_coefficients)]


class pasm_learned_stats(ctypes.Structure):
    _fields_ = [("enabled", ctypes.c_int), ("train_steps", ctypes.c_int),
                ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("plain_rate", ctypes.c_double), ("learned_rate", ctypes.c_double),
                ("plain_cycle_ms", ctypes.c_double), ("learned_cycle_ms", ctypes.c_double),
                ("cycles_learned", ctypes.c_long), ("cycles_fallback", ctypes.c_long)]


class pasm_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("smoother", ctypes.c_int),
                ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("vcycles", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("tol", ctypes.c_double), ("omega", ctypes.c_double),
                ("cheb_alpha", ctypes.c_double), ("stream", ctypes.c_void_p),
                ("fused_smoothing", ctypes.c_int), ("exhaustive_selection", ctypes.c_int)]


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib() -> ctypes.CDLL:
    """Load libpasm.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1908_10251_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.pasm_default_options.argtypes = [ctypes.POINTER(pasm_options)]
    L.pasm_default_options.restype = None
    L.pasm_setup.argtypes = [ctypes.POINTER(_P), ctypes.POINTER(pasm_domain), ctypes.POINTER(pasm_coefficients),
                             ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.POINTER(pasm_options)]
    L.pasm_iterate.argtypes = [_P, _I]
    L.pasm_iterate_n.argtypes = [_P, ctypes.c_int, _I]
    L.pasm_solve.argtypes = [_P, _I]
    L.pasm_restart.argtypes = [_P]
    L.pasm_restart_nested.argtypes = [_P, ctypes.c_int]
    L.pasm_eigenpairs.argtypes = [_P, _D, _D, ctypes.c_size_t]
    L.pasm_eigenvectors_device.argtypes = [_P, _P, ctypes.c_size_t]
    L.pasm_set_state.argtypes = [_P, _D, _D, ctypes.c_size_t]
    L.pasm_last_selection.argtypes = [_P, _I, _D, _I]
    L.pasm_coarse_eigenpairs.argtypes = [_P, _D, _D]
    L.pasm_last_borders.argtypes = [_P, _D, _D, _D]
    L.pasm_num_dofs.argtypes = [_P]
    L.pasm_num_dofs.restype = ctypes.c_size_t
    L.pasm_coarse_dofs.argtypes = [_P]
    L.pasm_coarse_dofs.restype = ctypes.c_size_t
    L.pasm_num_levels.argtypes = [_P]
    L.pasm_destroy.argtypes = [_P]
    L.pasm_status_string.argtypes = [ctypes.c_int]
    L.pasm_status_string.restype = ctypes.c_char_p
    L.pasm_last_error.argtypes = [_P]
    L.pasm_last_error.restype = ctypes.c_char_p
    L.pasm_apply_operator.argtypes = [_P, ctypes.c_int, ctypes.c_int, _P, _P, ctypes.c_size_t, ctypes.c_int]
    L.pasm_vcycle.argtypes = [_P, _P, _P, ctypes.c_size_t, ctypes.c_int, ctypes.c_int]
    L.pasm_use_graph.argtypes = [_P, ctypes.c_int]
    L.pasm_graph_stats.argtypes = [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_long)]
    L.pasm_profile.argtypes = [_P, ctypes.c_int, ctypes.c_int]
    L.pasm_profile_read.argtypes = [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_long), _D, _D]
    _F = ctypes.POINTER(ctypes.c_float)
    L.pasm_learned_report.argtypes = [_P, ctypes.POINTER(pasm_learned_stats)]
    L.pasm_learned_weights.argtypes = [_P, _F]
    L.pasm_learned_ratios.argtypes = [_P, _D, ctypes.c_int]
    L.pasm_learned_ratios.restype = ctypes.c_int
    L.pasm_learned_set_weights.argtypes = [_P, _F]
    L.pasm_learned_train.argtypes = [_P, ctypes.c_int, _D]
    L.pasm_learned_set_threshold.argtypes = [_P, ctypes.c_double]
    L.pasm_learned_enable.argtypes = [_P, ctypes.c_int]
    L.pasm_learned_step.argtypes = [_P, ctypes.c_int, _P, _P, _P, ctypes.c_size_t, ctypes.c_int]
    L.pasm_learned_loss_grad.argtypes = [_P, ctypes.c_int, _P, ctypes.c_size_t, ctypes.c_int, _D, _D]
    L.pasm_learned_loss_grad_noalloc.argtypes = [_P, ctypes.c_int, _P, ctypes.c_size_t, ctypes.c_int, _D, _D]
    L.pasm_batch_setup.argtypes = [ctypes.POINTER(_P), ctypes.POINTER(pasm_domain), ctypes.POINTER(pasm_instance),
                                   ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.POINTER(pasm_options)]
    L.pasm_batch_iterate.argtypes = [_P, _I]
    L.pasm_batch_restart.argtypes = [_P]
    L.pasm_batch_solve.argtypes = [_P, _I]
    L.pasm_batch_eigenpairs.argtypes = [_P, ctypes.c_int, _D, _D, ctypes.c_size_t]
    L.pasm_batch_set_state.argtypes = [_P, ctypes.c_int, _D, _D, ctypes.c_size_t]
    L.pasm_batch_num_dofs.argtypes = [_P, ctypes.c_int]
    L.pasm_batch_num_dofs.restype = ctypes.c_size_t
    L.pasm_batch_num_levels.argtypes = [_P]
    L.pasm_batch_use_graph.argtypes = [_P, ctypes.c_int]
    L.pasm_batch_tuning.argtypes = [_P, _I, _D]
    L.pasm_batch_set_tiles.argtypes = [_P, _I]
    L.pasm_batch_profile.argtypes = [_P, ctypes.c_int, ctypes.c_int]
    L.pasm_batch_profile_read.argtypes = [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_long), _D, _D]
    L.pasm_batch_destroy.argtypes = [_P]
    L.pasm_batch_last_error.argtypes = [_P]
    L.pasm_batch_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int, ctx=None):
    if status != PASM_OK:
        L = lib()
        msg = (L.pasm_last_error(ctx) or b"").decode()
        raise PasmError(status, f"{L.pasm_status_string(status).decode()}: {msg}")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _torch_ptr(t) -> int:
    """Device pointer of a float64 CUDA tensor.  Torch's current stream is
    synchronised first: the library works on its own stream, and must not read
    the tensor before torch's pending writes to it have landed."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    torch.cuda.current_stream(t.device).synchronize()
    return t.data_ptr()


def current_stream_handle() -> Optional[int]:
    """The raw hipStream_t of torch's current stream (None without a GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:  # pragma: no cover
        pass
    return None


def pasm_default_options() -> pasm_options:
    o = pasm_options()
    lib().pasm_default_options(ctypes.byref(o))
    return o


def pasm_setup(dim: int, H: float, h: float, k: int, kappa: Optional[np.ndarray] = None,
               potential: Optional[np.ndarray] = None, options: Optional[pasm_options] = None,
               stream=None, tensor: Optional[np.ndarray] = None):
    """Create a context; returns the opaque handle (ctypes.c_void_p)."""
    L = lib()
    dom = pasm_domain(dim)
    coef = pasm_coefficients()
    keep = []
    n_el = 0
    if kappa is not None:
        kap = np.ascontiguousarray(kappa, dtype=np.float64)
        keep.append(kap)
        coef.kappa = _dptr(kap)
        n_el = kap.size
    if potential is not None:
        pot = np.ascontiguousarray(potential, dtype=np.float64)
        keep.append(pot)
        coef.potential = _dptr(pot)
        n_el = pot.size
    if tensor is not None:
        ten = np.ascontiguousarray(tensor, dtype=np.float64).reshape(-1)
        keep.append(ten)
        coef.tensor = _dptr(ten)
        n_el = ten.size // 6
    coef.n_elements = n_el
    opt = options if options is not None else pasm_default_options()
    if stream is not None:
        opt.stream = stream
    ctx = _P()
    st = L.pasm_setup(ctypes.byref(ctx), ctypes.byref(dom), ctypes.byref(coef), float(H), float(h), int(k),
                      ctypes.byref(opt))
    _check(st, None)
    return ctx


def pasm_iterate(ctx) -> bool:
    conv = ctypes.c_int(0)
    _check(lib().pasm_iterate(ctx, ctypes.byref(conv)), ctx)
    return bool(conv.value)


def pasm_iterate_n(ctx, n: int) -> bool:
    conv = ctypes.c_int(0)
    _check(lib().pasm_iterate_n(ctx, int(n), ctypes.byref(conv)), ctx)
    return bool(conv.value)


def pasm_restart(ctx) -> None:
    _check(lib().pasm_restart(ctx), ctx)


def pasm_restart_nested(ctx, varpi: int = 1) -> None:
    _check(lib().pasm_restart_nested(ctx, int(varpi)), ctx)


def pasm_solve(ctx, allow_notconv: bool = False) -> int:
    it = ctypes.c_int(0)
    st = lib().pasm_solve(ctx, ctypes.byref(it))
    if not (allow_notconv and st == PASM_E_NOTCONV):
        _check(st, ctx)
    return it.value


def pasm_num_dofs(ctx) -> int:
    return int(lib().pasm_num_dofs(ctx))


def pasm_coarse_dofs(ctx) -> int:
    return int(lib().pasm_coarse_dofs(ctx))


def pasm_num_levels(ctx) -> int:
    return int(lib().pasm_num_levels(ctx))


def pasm_eigenpairs(ctx, k: int, vectors: bool = True) -> Tuple[np.ndarray, Optional[np.ndarray]]:
    N = pasm_num_dofs(ctx)
    lam = np.empty(k)
    U = np.empty((k, N)) if vectors else None
    _check(lib().pasm_eigenpairs(ctx, _dptr(lam), _dptr(U) if vectors else None, N), ctx)
    return lam, U


def pasm_eigenvectors_device(ctx, U_dev) -> None:
    _check(lib().pasm_eigenvectors_device(ctx, _torch_ptr(U_dev), U_dev.shape[-1]), ctx)


def pasm_set_state(ctx, lam: np.ndarray, U: np.ndarray) -> None:
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    _check(lib().pasm_set_state(ctx, _dptr(lam), _dptr(U), U.shape[1]), ctx)


def pasm_last_selection(ctx, k: int):
    rank = np.empty(k, dtype=np.int32)
    score = np.empty(k)
    flags = np.empty(k, dtype=np.int32)
    _check(lib().pasm_last_selection(ctx, rank.ctypes.data_as(_I), _dptr(score), flags.ctypes.data_as(_I)), ctx)
    return rank, score, flags


def pasm_coarse_eigenpairs(ctx):
    N = pasm_coarse_dofs(ctx)
    theta = np.empty(N)
    Q = np.empty((N, N))           # row j = eigenvector j (column-major Q)
    _check(lib().pasm_coarse_eigenpairs(ctx, _dptr(theta), _dptr(Q)), ctx)
    return theta, Q.T.copy()


def pasm_last_borders(ctx, k: int):
    N = pasm_coarse_dofs(ctx)
    bz = np.empty((k, 2))
    p = np.empty((k, N))
    q = np.empty((k, N))
    _check(lib().pasm_last_borders(ctx, _dptr(bz), _dptr(p), _dptr(q)), ctx)
    return bz, p, q


def pasm_apply_operator(ctx, level: int, op: int, x, y) -> None:
    """y = A_level x or M_h x for torch float64 CUDA tensors of shape (nrhs, N_level)."""
    _check(lib().pasm_apply_operator(ctx, level, op, _torch_ptr(x), _torch_ptr(y), x.shape[1], x.shape[0]), ctx)


def pasm_vcycle(ctx, f, x, ncycles: int) -> None:
    _check(lib().pasm_vcycle(ctx, _torch_ptr(f), _torch_ptr(x), x.shape[1], x.shape[0], ncycles), ctx)


def pasm_use_graph(ctx, enable: bool) -> None:
    _check(lib().pasm_use_graph(ctx, int(enable)), ctx)


def pasm_graph_stats(ctx):
    """(enabled, graphs held, steps replayed from a graph)."""
    e, g, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_long()
    _check(lib().pasm_graph_stats(ctx, ctypes.byref(e), ctypes.byref(g), ctypes.byref(r)), ctx)
    return bool(e.value), g.value, r.value


def pasm_profile(ctx, kernel: int, enable: bool) -> None:
    _check(lib().pasm_profile(ctx, kernel, int(enable)), ctx)


def pasm_profile_read(ctx, kernel: int):
    n = ctypes.c_long(0)
    ms = ctypes.c_double(0)
    b = ctypes.c_double(0)
    _check(lib().pasm_profile_read(ctx, kernel, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)), ctx)
    return n.value, ms.value, b.value


def pasm_destroy(ctx) -> None:
    if ctx:
        _check(lib().pasm_destroy(ctx))


def options(precision: int = PASM_FP64, smoother: int = PASM_JACOBI, nu_pre: int = 2, nu_post: int = 2,
            vcycles: int = 2, max_iter: int = 50, tol: float = 1e-10, omega: float = 0.0,
            cheb_alpha: float = 0.0, fused: bool = True, exhaustive: bool = False) -> pasm_options:
    o = pasm_default_options()
    o.fused_smoothing = int(fused)
    o.exhaustive_selection = int(exhaustive)
    o.precision, o.smoother, o.nu_pre, o.nu_post = precision, smoother, nu_pre, nu_post
    o.vcycles, o.max_iter, o.tol, o.omega, o.cheb_alpha = vcycles, max_iter, tol, omega, cheb_alpha
    return o


def options_for(workload) -> pasm_options:
    """Options matching a `workloads.Workload` description."""
    sm = {"cheb": PASM_CHEBYSHEV, "jacobi": PASM_JACOBI, "learned": PASM_LEARNED, "cg": PASM_CG}[workload.smoother]
    return options(precision=PASM_MIXED if workload.precision == "mixed" else PASM_FP64,
                   smoother=sm,
                   nu_pre=workload.nu_pre, nu_post=workload.nu_post, vcycles=workload.vcycles,
                   tol=workload.tol)


class Solver:
    """Owning wrapper around a context."""

    def __init__(self, dim, H, h, k, kappa=None, potential=None, opts=None, stream=None, tensor=None):
        self.k = k
        self.ctx = pasm_setup(dim, H, h, k, kappa, potential, opts, stream, tensor)

    def iterate(self) -> bool:
        return pasm_iterate(self.ctx)

    def iterate_n(self, n: int) -> bool:
        return pasm_iterate_n(self.ctx, n)

    def solve(self, allow_notconv=False) -> int:
        return pasm_solve(self.ctx, allow_notconv)

    def eigenpairs(self, vectors=True):
        return pasm_eigenpairs(self.ctx, self.k, vectors)

    def close(self):
        if self.ctx:
            pasm_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# learned smoother
# ---------------------------------------------------------------------------
def pasm_learned_report(ctx) -> dict:
    st = pasm_learned_stats()
    _check(lib().pasm_learned_report(ctx, ctypes.byref(st)), ctx)
    return {f: getattr(st, f) for f, _ in pasm_learned_stats._fields_}


def pasm_learned_weights(ctx) -> np.ndarray:
    w = np.empty((2, 16, 27), dtype=np.float32)
    _check(lib().pasm_learned_weights(ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), ctx)
    return w


def pasm_learned_ratios(ctx, max_count: int = 4096) -> np.ndarray:
    """Recent per-cycle, per-right-hand-side residual reductions of learned V-cycles."""
    out = np.empty(max_count, dtype=np.float64)
    n = lib().pasm_learned_ratios(ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(max_count))
    if n < 0:
        raise PasmError(-1, "pasm_learned_ratios: invalid arguments")
    return out[:n].copy()


def pasm_learned_set_weights(ctx, w) -> None:
    w = np.ascontiguousarray(w, dtype=np.float32).reshape(2, 16, 27)
    _check(lib().pasm_learned_set_weights(ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), ctx)


def pasm_learned_set_threshold(ctx, rate: float) -> None:
    _check(lib().pasm_learned_set_threshold(ctx, float(rate)), ctx)


def pasm_learned_enable(ctx, enable: bool) -> None:
    _check(lib().pasm_learned_enable(ctx, int(enable)), ctx)


def pasm_learned_train(ctx, steps: int) -> np.ndarray:
    h = np.zeros(max(steps, 1))
    _check(lib().pasm_learned_train(ctx, steps, _dptr(h)), ctx)
    return h[:steps]


def pasm_learned_step(ctx, level: int, x, f, out) -> None:
    """out = x + N((f - A x)/D) for torch float64 CUDA tensors (nrhs, N_level)."""
    _check(lib().pasm_learned_step(ctx, level, _torch_ptr(x), _torch_ptr(f), _torch_ptr(out), x.shape[1],
                                   x.shape[0]), ctx)


def pasm_learned_loss_grad(ctx, level: int, r):
    """Training loss and gradient [2][16][27] of samples r (torch float64 CUDA, (ns, N_level))."""
    loss = ctypes.c_double(0)
    g = np.zeros((2, 16, 27))
    _check(lib().pasm_learned_loss_grad(ctx, level, _torch_ptr(r), r.shape[1], r.shape[0], ctypes.byref(loss),
                                        _dptr(g)), ctx)
    return loss.value, g


def pasm_learned_loss_grad_noalloc(ctx, level: int, r):
    """As pasm_learned_loss_grad, with the library's fixed scratch array instead
    of device allocations (raises PASM_E_INVALID beyond its size)."""
    loss = ctypes.c_double(0)
    g = np.zeros((2, 16, 27))
    _check(lib().pasm_learned_loss_grad_noalloc(ctx, level, _torch_ptr(r), r.shape[1], r.shape[0],
                                                ctypes.byref(loss), _dptr(g)), ctx)
    return loss.value, g


# ---------------------------------------------------------------------------
# batches of uneven instances
# ---------------------------------------------------------------------------
def _bcheck(status: int, b=None):
    if status != PASM_OK:
        L = lib()
        msg = (L.pasm_batch_last_error(b) or b"").decode()
        raise PasmError(status, f"{L.pasm_status_string(status).decode()}: {msg}")


def pasm_batch_setup(H: float, k: int, instances, options: Optional[pasm_options] = None, stream=None, dim: int = 2):
    """instances: sequence of (h, kappa or None, potential or None)."""
    L = lib()
    n = len(instances)
    arr = (pasm_instance * max(n, 1))()
    keep = []
    for i, (h, kap, pot) in enumerate(instances):
        arr[i].h = float(h)
        n_el = 0
        if kap is not None:
            a = np.ascontiguousarray(kap, dtype=np.float64)
            keep.append(a)
            arr[i].coef.kappa = _dptr(a)
            n_el = a.size
        if pot is not None:
            a = np.ascontiguousarray(pot, dtype=np.float64)
            keep.append(a)
            arr[i].coef.potential = _dptr(a)
            n_el = a.size
        arr[i].coef.n_elements = n_el
    opt = options if options is not None else pasm_default_options()
    if stream is not None:
        opt.stream = stream
    b = _P()
    st = L.pasm_batch_setup(ctypes.byref(b), ctypes.byref(pasm_domain(dim)), arr, n, float(H), int(k),
                            ctypes.byref(opt))
    _bcheck(st, None)
    return b


def pasm_batch_iterate(b) -> bool:
    conv = ctypes.c_int(0)
    _bcheck(lib().pasm_batch_iterate(b, ctypes.byref(conv)), b)
    return bool(conv.value)


def pasm_batch_restart(b) -> None:
    _bcheck(lib().pasm_batch_restart(b), b)


def pasm_batch_solve(b, allow_notconv: bool = False) -> int:
    it = ctypes.c_int(0)
    st = lib().pasm_batch_solve(b, ctypes.byref(it))
    if not (allow_notconv and st == PASM_E_NOTCONV):
        _bcheck(st, b)
    return it.value


def pasm_batch_num_dofs(b, member: int) -> int:
    return int(lib().pasm_batch_num_dofs(b, member))


def pasm_batch_num_levels(b) -> int:
    return int(lib().pasm_batch_num_levels(b))


def pasm_batch_eigenpairs(b, member: int, k: int, vectors: bool = True):
    N = pasm_batch_num_dofs(b, member)
    lam = np.empty(k)
    U = np.empty((k, N)) if vectors else None
    _bcheck(lib().pasm_batch_eigenpairs(b, member, _dptr(lam), _dptr(U) if vectors else None, N), b)
    return lam, U


def pasm_batch_set_state(b, member: int, lam: np.ndarray, U: np.ndarray) -> None:
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    _bcheck(lib().pasm_batch_set_state(b, member, _dptr(lam), _dptr(U), U.shape[1]), b)


def pasm_batch_use_graph(b, enable: bool) -> None:
    _bcheck(lib().pasm_batch_use_graph(b, int(enable)), b)


def pasm_batch_tuning(b):
    L = pasm_batch_num_levels(b)
    rows = np.zeros(L, dtype=np.int32)
    ms = np.zeros((L, 4))
    _bcheck(lib().pasm_batch_tuning(b, rows.ctypes.data_as(_I), _dptr(ms)), b)
    return rows, ms


def pasm_batch_set_tiles(b, rows) -> None:
    r = np.ascontiguousarray(rows, dtype=np.int32)
    _bcheck(lib().pasm_batch_set_tiles(b, r.ctypes.data_as(_I)), b)


def pasm_batch_profile(b, kernel: int, enable: bool) -> None:
    _bcheck(lib().pasm_batch_profile(b, kernel, int(enable)), b)


def pasm_batch_profile_read(b, kernel: int):
    n = ctypes.c_long(0)
    ms = ctypes.c_double(0)
    by = ctypes.c_double(0)
    _bcheck(lib().pasm_batch_profile_read(b, kernel, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)), b)
    return n.value, ms.value, by.value


def pasm_batch_destroy(b) -> None:
    if b:
        _bcheck(lib().pasm_batch_destroy(b))


class Batch:
    """Owning wrapper around a batch of instances (h, kappa, potential)."""

    def __init__(self, H, k, instances, opts=None, stream=None):
        self.k = k
        self.n = len(instances)
        self.b = pasm_batch_setup(H, k, instances, opts, stream)

    def iterate(self) -> bool:
        return pasm_batch_iterate(self.b)

    def solve(self, allow_notconv=False) -> int:
        return pasm_batch_solve(self.b, allow_notconv)

    def eigenpairs(self, member, vectors=True):
        return pasm_batch_eigenpairs(self.b, member, self.k, vectors)

    def eigenvalues(self) -> np.ndarray:
        return np.stack([self.eigenpairs(i, False)[0] for i in range(self.n)])

    def close(self):
        if self.b:
            pasm_batch_destroy(self.b)
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
