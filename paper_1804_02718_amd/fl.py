"""Thin ctypes binding of ``libfl.so`` (C-ABI in ``include/fl.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device vectors are torch CUDA tensors (torch supplies device memory
and streams); the functions below pass their data pointers and the current
stream to the C entry points of the same names.  The library is required:
importing works without it, but the first call raises ``FlLibraryMissing``.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfl.so")

FL_OK, FL_E_INVAL, FL_E_NOMEM, FL_E_DEVICE, FL_E_NOCONV, FL_E_BREAKDOWN, FL_E_UNSUPPORTED = range(7)
FL_FP64, FL_FP32 = 0, 1
SOLVERS = {"auto": 0, "cg64": 1, "refine": 2, "fpcg": 3, "tau": 4, "tau32": 5}

EXPORTED = ["fl_coeffs", "fl_apply", "fl_apply_profiled", "fl_variant_count", "fl_variant_info",
            "fl_select_variant", "fl_autotune", "fl_batch_create", "fl_batch_poisson_solve", "fl_batch_info",
            "fl_batch_destroy", "fl_poisson_solve", "fl_poisson_solve_ex", "fl_allen_cahn_step",
            "fl_allen_cahn_step_ex", "fl_op_destroy", "fl_op_describe", "fl_get_coeffs", "fl_get_symbol",
            "fl_status_string", "fl_last_error", "fl_unet_create", "fl_unet_destroy", "fl_unet_num_params",
            "fl_unet_step", "fl_unet_get_weights", "fl_unet_set_weights", "fl_unet_apply", "fl_set_preconditioner",
            "fl_gemm_test", "fl_unet_pack", "fl_unet_train", "fl_allen_cahn_step_gen",
            "fl_coeffs_gamma", "fl_coeffs_box", "fl_tau_apply", "fl_apply_noalloc", "fl_residual", "fl_tune", "fl_batch_stats"]


class FlLibraryMissing(RuntimeError):
    pass


class FlError(RuntimeError):
    def __init__(self, status, message, info=None):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, status), message))
        self.status = status
        self.info = info


_STATUS_NAMES = {0: "FL_OK", 1: "FL_E_INVAL", 2: "FL_E_NOMEM", 3: "FL_E_DEVICE", 4: "FL_E_NOCONV",
                 5: "FL_E_BREAKDOWN", 6: "FL_E_UNSUPPORTED"}


class fl_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("fell_back", ctypes.c_int),
                ("status", ctypes.c_int), ("relres", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fl_solve_opts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("max_iter", ctypes.c_int), ("use_x0", ctypes.c_int),
                ("check_every", ctypes.c_int), ("inner_tol", ctypes.c_double)]


class fl_op_desc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("N", ctypes.c_int), ("n", ctypes.c_int), ("P", ctypes.c_int),
                ("Q", ctypes.c_int), ("M", ctypes.c_int64), ("alpha", ctypes.c_double),
                ("h", ctypes.c_double), ("c", ctypes.c_double), ("a0", ctypes.c_double),
                ("gamma", ctypes.c_double), ("nk", ctypes.c_int * 3)]


_LIB = None


def load(path: str = LIB_PATH):
    """Load libfl.so and declare its signatures (raises FlLibraryMissing if absent)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise FlLibraryMissing("HIP library %s is not built (run __graft_entry__.build())" % path)
    lib = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    lib.fl_coeffs.argtypes = [ip, dp, dp, ip, ctypes.POINTER(vp)]
    lib.fl_coeffs_gamma.argtypes = [ip, dp, dp, dp, ip, ctypes.POINTER(vp)]
    lib.fl_coeffs_box.argtypes = [ip, dp, dp, dp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(vp)]
    lib.fl_apply.argtypes = [vp, vp, vp, ip, vp]
    lib.fl_apply_noalloc.argtypes = [vp, vp, vp, ip, vp]
    lib.fl_residual.argtypes = [vp, vp, vp, vp, vp]
    lib.fl_tau_apply.argtypes = [vp, vp, vp, dp, dp, vp]
    lib.fl_apply_profiled.argtypes = [vp, vp, vp, ip, ip, vp, ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_int)]
    lib.fl_variant_count.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int)]
    lib.fl_variant_info.argtypes = [vp, ip, ip, ctypes.POINTER(ctypes.c_int)]
    lib.fl_select_variant.argtypes = [vp, ip, ip]
    lib.fl_autotune.argtypes = [vp, ip, ip, vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)]
    lib.fl_batch_create.argtypes = [ip, ip, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(vp)]
    lib.fl_batch_poisson_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), dp, ip,
                                           ctypes.POINTER(fl_info), vp]
    lib.fl_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.fl_batch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.fl_tune.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int)]
    lib.fl_batch_destroy.argtypes = [vp]
    lib.fl_poisson_solve.argtypes = [vp, vp, dp, vp, ctypes.POINTER(fl_info), vp]
    lib.fl_poisson_solve_ex.argtypes = [vp, vp, dp, vp, ctypes.POINTER(fl_solve_opts), ctypes.POINTER(fl_info), vp]
    lib.fl_allen_cahn_step.argtypes = [vp, vp, dp, dp, ctypes.POINTER(fl_info), vp]
    lib.fl_allen_cahn_step_ex.argtypes = [vp, vp, dp, dp, dp, dp, ip, ctypes.POINTER(fl_info), vp]
    lib.fl_allen_cahn_step_gen.argtypes = [vp, vp, dp, dp, dp, dp, dp, dp, ip, ctypes.POINTER(fl_info), vp]
    lib.fl_op_destroy.argtypes = [vp]
    lib.fl_op_describe.argtypes = [vp, ctypes.POINTER(fl_op_desc)]
    lib.fl_get_coeffs.argtypes = [vp, vp]
    lib.fl_get_symbol.argtypes = [vp, vp]
    fp = ctypes.POINTER(ctypes.c_float)
    lib.fl_unet_create.argtypes = [ip, ip, ctypes.c_ulonglong, ip, ctypes.POINTER(vp)]
    lib.fl_unet_destroy.argtypes = [vp]
    lib.fl_unet_num_params.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong)]
    lib.fl_unet_step.argtypes = [vp, ip, vp, vp, vp, ctypes.c_float, fp, fp]
    lib.fl_unet_pack.argtypes = [vp, ip, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_double), ip,
                                 vp, vp]
    lib.fl_unet_train.argtypes = [vp, ctypes.c_long, vp, vp, ctypes.POINTER(vp), ip, ip, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_ulonglong, fp]
    lib.fl_unet_get_weights.argtypes = [vp, fp]
    lib.fl_unet_set_weights.argtypes = [vp, fp]
    lib.fl_unet_apply.argtypes = [vp, vp, ip, dp, vp, vp]
    lib.fl_set_preconditioner.argtypes = [vp, vp]
    lib.fl_gemm_test.argtypes = [ip, ip, ip, ip, ip, fp, fp, fp]
    lib.fl_status_string.argtypes = [ip]
    lib.fl_status_string.restype = ctypes.c_char_p
    lib.fl_last_error.argtypes = []
    lib.fl_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("fl_status_string", "fl_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


def _check(status, info=None):
    if status != FL_OK:
        raise FlError(status, load().fl_last_error().decode(), info)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t, dtype=None, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected dtype %s, got %s" % (dtype, t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("expected %d entries, got %d" % (numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# C entry points under their own names
# ---------------------------------------------------------------------------
def fl_coeffs(d: int, alpha: float, h: float, N: int) -> ctypes.c_void_p:
    op = ctypes.c_void_p()
    _check(load().fl_coeffs(int(d), float(alpha), float(h), int(N), ctypes.byref(op)))
    return op


def fl_coeffs_gamma(d: int, alpha: float, gamma: float, h: float, N: int) -> ctypes.c_void_p:
    op = ctypes.c_void_p()
    _check(load().fl_coeffs_gamma(int(d), float(alpha), float(gamma), float(h), int(N), ctypes.byref(op)))
    return op


def fl_coeffs_box(d: int, alpha: float, gamma: float, h: float, Nk) -> ctypes.c_void_p:
    """Operator on a box with Nk[k] intervals of width h along axis k (x first)."""
    Nk = [int(x) for x in Nk]
    if len(Nk) != d:
        raise ValueError("Nk needs %d entries" % d)
    op = ctypes.c_void_p()
    _check(load().fl_coeffs_box(int(d), float(alpha), float(gamma), float(h), (ctypes.c_int * d)(*Nk),
                                ctypes.byref(op)))
    return op


def box_intervals(sides, h):
    """Intervals per axis of a box of the given side lengths: the smallest N_k with N_k h >= side (Sec. 2)."""
    return [max(2, int(math.ceil(s / h * (1.0 - 1e-12)))) for s in sides]


def fl_op_describe(op) -> dict:
    desc = fl_op_desc()
    _check(load().fl_op_describe(op, ctypes.byref(desc)))
    out = {k: getattr(desc, k) for k, _ in desc._fields_}
    out["nk"] = list(out["nk"])[:desc.d]
    return out


def fl_apply(op, u, y, stream=None):
    import torch
    prec = FL_FP64 if u.dtype == torch.float64 else FL_FP32
    if u.dtype not in (torch.float32, torch.float64) or y.dtype != u.dtype:
        raise TypeError("u and y must both be float32 or both float64")
    _check(load().fl_apply(op, _ptr(u), _ptr(y), prec, _stream(stream)))
    return y


def fl_apply_noalloc(op, u, y, stream=None):
    """fl_apply with the spectra workspaces in the library's static per-GPU array (no allocation)."""
    import torch
    prec = FL_FP64 if u.dtype == torch.float64 else FL_FP32
    if u.dtype not in (torch.float32, torch.float64) or y.dtype != u.dtype:
        raise TypeError("u and y must both be float32 or both float64")
    _check(load().fl_apply_noalloc(op, _ptr(u), _ptr(y), prec, _stream(stream)))
    return y


def fl_residual(op, f, u, r, stream=None):
    """r = f - A u in FP64 (float64 device vectors; r may be f)."""
    import torch
    _check(load().fl_residual(op, _ptr(f, torch.float64), _ptr(u, torch.float64), _ptr(r, torch.float64),
                              _stream(stream)))
    return r


def fl_tau_apply(op, r, z, s0=0.0, s1=1.0, stream=None):
    """z = M^{-1} r, M the sine-transform (tau) preconditioner of s0 I + s1 A (float64 vectors)."""
    import torch
    _check(load().fl_tau_apply(op, _ptr(r, torch.float64), _ptr(z, torch.float64), float(s0), float(s1),
                               _stream(stream)))
    return z


def fl_apply_profiled(op, u, y, reps, stream=None):
    """Average per-pass milliseconds over `reps` matvecs (HIP events on the given stream)."""
    import torch
    prec = FL_FP64 if u.dtype == torch.float64 else FL_FP32
    ms = (ctypes.c_float * 8)()
    npass = ctypes.c_int()
    _check(load().fl_apply_profiled(op, _ptr(u), _ptr(y), prec, int(reps), _stream(stream), ms,
                                    ctypes.byref(npass)))
    return [ms[i] for i in range(npass.value)]


def _prec(prec):
    return {"fp64": FL_FP64, "fp32": FL_FP32}.get(prec, prec)


def fl_variant_count(op, prec) -> int:
    n = ctypes.c_int()
    _check(load().fl_variant_count(op, _prec(prec), ctypes.byref(n)))
    return n.value


def fl_variant_info(op, prec, k) -> dict:
    d = (ctypes.c_int * 5)()
    _check(load().fl_variant_info(op, _prec(prec), int(k), d))
    return {"ex": d[0], "ey": d[1], "tile": d[2], "row_pairs": d[3], "kind": d[4]}


def fl_select_variant(op, prec, k):
    _check(load().fl_select_variant(op, _prec(prec), int(k)))


def fl_autotune(op, prec, reps=20, stream=None):
    """Time every kernel variant, select the fastest; returns (best, [ms per variant])."""
    n = fl_variant_count(op, prec)
    ms = (ctypes.c_float * max(n, 1))()
    best = ctypes.c_int()
    _check(load().fl_autotune(op, _prec(prec), int(reps), _stream(stream), ctypes.byref(best), ms))
    return best.value, [ms[i] for i in range(n)]


def fl_poisson_solve(op, f, tol, u, stream=None):
    info = fl_info()
    st = load().fl_poisson_solve(op, _ptr(f), float(tol), _ptr(u), ctypes.byref(info), _stream(stream))
    _check(st, info.as_dict())
    return info.as_dict()


def fl_poisson_solve_ex(op, f, tol, u, solver="auto", max_iter=0, use_x0=False, check_every=0, inner_tol=0.0,
                        stream=None, raise_on_error=True):
    opts = fl_solve_opts(SOLVERS[solver] if isinstance(solver, str) else int(solver), int(max_iter),
                         int(bool(use_x0)), int(check_every), float(inner_tol))
    info = fl_info()
    st = load().fl_poisson_solve_ex(op, _ptr(f), float(tol), _ptr(u), ctypes.byref(opts), ctypes.byref(info),
                                    _stream(stream))
    if raise_on_error:
        _check(st, info.as_dict())
    return info.as_dict()


def fl_allen_cahn_step(op, u, tau, eps, stream=None):
    info = fl_info()
    st = load().fl_allen_cahn_step(op, _ptr(u), float(tau), float(eps), ctypes.byref(info), _stream(stream))
    _check(st, info.as_dict())
    return info.as_dict()


def fl_allen_cahn_step_ex(op, u, tau, eps, theta=0.5, tol=1e-8, solver="auto", stream=None):
    info = fl_info()
    st = load().fl_allen_cahn_step_ex(op, _ptr(u), float(tau), float(eps), float(theta), float(tol),
                                      SOLVERS[solver] if isinstance(solver, str) else int(solver),
                                      ctypes.byref(info), _stream(stream))
    _check(st, info.as_dict())
    return info.as_dict()


def fl_allen_cahn_step_gen(op, u, tau, kappa, gamma, shift, theta=0.5, tol=1e-8, solver="auto", stream=None):
    info = fl_info()
    st = load().fl_allen_cahn_step_gen(op, _ptr(u), float(tau), float(kappa), float(gamma), float(shift),
                                       float(theta), float(tol),
                                       SOLVERS[solver] if isinstance(solver, str) else int(solver),
                                       ctypes.byref(info), _stream(stream))
    _check(st, info.as_dict())
    return info.as_dict()


def fl_get_coeffs(op) -> np.ndarray:
    desc = fl_op_describe(op)
    a = np.zeros((desc["N"] + 1) ** desc["d"])
    _check(load().fl_get_coeffs(op, a.ctypes.data_as(ctypes.c_void_p)))
    return a.reshape((desc["N"] + 1,) * desc["d"])


def fl_get_symbol(op) -> np.ndarray:
    desc = fl_op_describe(op)
    lam = np.zeros(desc["Q"] ** desc["d"])
    _check(load().fl_get_symbol(op, lam.ctypes.data_as(ctypes.c_void_p)))
    return lam.reshape((desc["Q"],) * desc["d"])


def fl_op_destroy(op):
    if op:
        load().fl_op_destroy(op)


def fl_batch_create(d, Ns, alphas, hs):
    n = len(Ns)
    b = ctypes.c_void_p()
    _check(load().fl_batch_create(int(d), n, (ctypes.c_int * n)(*[int(x) for x in Ns]),
                                  (ctypes.c_double * n)(*[float(x) for x in alphas]),
                                  (ctypes.c_double * n)(*[float(x) for x in hs]), ctypes.byref(b)))
    return b


def fl_batch_poisson_solve(b, fs, us, tol, max_iter=0, stream=None, raise_on_error=True):
    n = len(fs)
    fp = (ctypes.c_void_p * n)(*[_ptr(x, numel=None).value for x in fs])
    up = (ctypes.c_void_p * n)(*[_ptr(x).value for x in us])
    infos = (fl_info * n)()
    st = load().fl_batch_poisson_solve(b, fp, up, float(tol), int(max_iter), infos, _stream(stream))
    out = [infos[i].as_dict() for i in range(n)]
    if raise_on_error:
        _check(st, out)
    return out


def fl_batch_info(b):
    nc, mb = ctypes.c_int(), ctypes.c_int()
    _check(load().fl_batch_info(b, ctypes.byref(nc), ctypes.byref(mb)))
    return {"classes": nc.value, "max_batch": mb.value}


def fl_batch_stats(b):
    """Host waits and graph replays of the last batched solve, and each class's variants."""
    nc = fl_batch_info(b)["classes"]
    hw, gl = ctypes.c_int(), ctypes.c_int()
    v32, v64 = (ctypes.c_int * nc)(), (ctypes.c_int * nc)()
    _check(load().fl_batch_stats(b, ctypes.byref(hw), ctypes.byref(gl), v32, v64))
    return {"host_waits": hw.value, "graph_launches": gl.value, "var32": list(v32), "var64": list(v64)}


def fl_tune(op, prec):
    """Select (and return) the cached, or newly timed, fastest variant for prec."""
    k = ctypes.c_int()
    _check(load().fl_tune(op, _prec(prec), ctypes.byref(k)))
    return k.value


def fl_batch_destroy(b):
    if b:
        load().fl_batch_destroy(b)


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def fl_unet_create(H, max_batch, seed, fp32_operands=False):
    u = ctypes.c_void_p()
    _check(load().fl_unet_create(int(H), int(max_batch), int(seed), int(bool(fp32_operands)), ctypes.byref(u)))
    return u


def fl_unet_destroy(u):
    if u:
        load().fl_unet_destroy(u)


def fl_unet_num_params(u) -> int:
    n = ctypes.c_longlong()
    _check(load().fl_unet_num_params(u, ctypes.byref(n)))
    return n.value


def fl_unet_step(u, x, t=None, y=None, lr=0.0, want_loss=False, want_grad=False):
    """x: device float32 [nb, H, H, 2]; t, y: device float32 [nb, H, H] or None.
    Returns (loss per sample or None, gradient or None) as numpy float32."""
    nb = x.shape[0]
    loss = np.zeros(nb, np.float32) if (want_loss and t is not None) else None
    grad = np.zeros(fl_unet_num_params(u), np.float32) if (want_grad and t is not None) else None
    _check(load().fl_unet_step(u, int(nb), _ptr(x), _ptr(t) if t is not None else None,
                               _ptr(y) if y is not None else None, float(lr),
                               _fptr(loss) if loss is not None else None, _fptr(grad) if grad is not None else None))
    return loss, grad


def fl_unet_pack(u, rs, sols, alphas, n, x, t=None):
    """Training samples from device pairs: rs, sols lists of float64 CUDA tensors (n*n each)."""
    k = len(rs)
    rp = (ctypes.c_void_p * k)(*[_ptr(r).value for r in rs])
    sp = (ctypes.c_void_p * k)(*[_ptr(s).value for s in sols]) if sols is not None else None
    al = (ctypes.c_double * k)(*[float(a) for a in alphas])
    _check(load().fl_unet_pack(u, k, rp, sp, al, int(n), _ptr(x), _ptr(t) if t is not None else None))


def fl_unet_train(u, x, t, epochs, batch, lr, lr_final=0.0, seed=0, ops=None):
    """Train on device samples x [count, H, H, 2], t [count, H, H]; returns the mean loss per epoch.
    ops: None (relative L2 loss) or one operator handle per sample (energy-norm loss; with t None
    the target-free residual loss ||A y - x0||^2 / ||x0||^2)."""
    losses = np.zeros(int(epochs), np.float32)
    count = int(x.shape[0])
    opa = None
    if ops is not None:
        if len(ops) != count:
            raise ValueError("one operator per sample")
        opa = (ctypes.c_void_p * count)(*[o.value if isinstance(o, ctypes.c_void_p) else o for o in ops])
    if t is None and ops is None:
        raise ValueError("targets or operators are needed")
    _check(load().fl_unet_train(u, count, _ptr(x), _ptr(t) if t is not None else None, opa, int(epochs),
                                int(batch), float(lr),
                                float(lr_final), int(seed), _fptr(losses)))
    return losses


def fl_unet_get_weights(u) -> np.ndarray:
    w = np.zeros(fl_unet_num_params(u), np.float32)
    _check(load().fl_unet_get_weights(u, _fptr(w)))
    return w


def fl_unet_set_weights(u, w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    if w.size != fl_unet_num_params(u):
        raise ValueError("expected %d weights" % fl_unet_num_params(u))
    _check(load().fl_unet_set_weights(u, _fptr(w)))


def fl_unet_apply(u, r, n, alpha, z, stream=None):
    _check(load().fl_unet_apply(u, _ptr(r), int(n), float(alpha), _ptr(z), _stream(stream)))
    return z


def fl_set_preconditioner(op, u):
    _check(load().fl_set_preconditioner(op, u))


def fl_gemm_test(A, B, kchunk=None, fp32_operands=False):
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    M, K = A.shape
    N = B.shape[0]
    C = np.zeros((M, N), np.float32)
    _check(load().fl_gemm_test(M, N, K, int(kchunk or K), int(bool(fp32_operands)), _fptr(A), _fptr(B), _fptr(C)))
    return C


class UNet:
    """The learned preconditioner network (one fl_unet)."""

    def __init__(self, H, max_batch=1, seed=0, fp32_operands=False):
        self._u = fl_unet_create(H, max_batch, seed, fp32_operands)
        self.H = H
        self.max_batch = max_batch

    @property
    def handle(self):
        return self._u

    def num_params(self):
        return fl_unet_num_params(self._u)

    def weights(self):
        return fl_unet_get_weights(self._u)

    def set_weights(self, w):
        fl_unet_set_weights(self._u, w)

    def forward(self, x):
        import torch
        y = torch.empty(x.shape[:3], dtype=torch.float32, device=x.device)
        fl_unet_step(self._u, x, None, y)
        return y

    def step(self, x, t, lr=0.0, want_grad=False, y=None):
        return fl_unet_step(self._u, x, t, y, lr, True, want_grad)

    def pack(self, rs, sols, alphas, n, x, t=None):
        fl_unet_pack(self._u, rs, sols, alphas, n, x, t)

    def train(self, x, t, epochs, batch, lr, lr_final=0.0, seed=0, ops=None):
        """ops: None, or per sample an Operator (or handle) for the energy-norm loss."""
        if ops is not None:
            ops = [o.handle if hasattr(o, "handle") else o for o in ops]
        return fl_unet_train(self._u, x, t, epochs, batch, lr, lr_final, seed, ops)

    def apply(self, r, n, alpha, z=None, stream=None):
        import torch
        if z is None:
            z = torch.empty_like(r)
        return fl_unet_apply(self._u, r, n, alpha, z, stream)

    def close(self):
        if getattr(self, "_u", None):
            fl_unet_destroy(self._u)
            self._u = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many Poisson problems of mixed (N, alpha) solved together (one fl_batch)."""

    def __init__(self, d, Ns, alphas, hs):
        self._b = fl_batch_create(d, Ns, alphas, hs)
        self.count = len(Ns)

    def solve(self, fs, us=None, tol=1e-8, max_iter=0, stream=None):
        import torch
        if us is None:
            us = [torch.zeros_like(f) for f in fs]
        return us, fl_batch_poisson_solve(self._b, fs, us, tol, max_iter, stream)

    def info(self):
        return fl_batch_info(self._b)

    def stats(self):
        return fl_batch_stats(self._b)

    def close(self):
        if getattr(self, "_b", None):
            fl_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# convenience wrapper owning one fl_op
# ---------------------------------------------------------------------------
class Operator:
    """The discrete fractional Laplacian on (a, a + N h)^d, zero outside (one fl_op).

    With ``Nk`` (intervals per axis, x first) it is the operator of the box
    prod_k (a_k, a_k + Nk[k] h): N = max(Nk) (``N`` may be None), and vectors
    hold prod_k (Nk[k] - 1) entries, x index fastest.
    """

    def __init__(self, d: int, alpha: float, h: float, N, gamma: float = 2.0, Nk=None):
        if Nk is not None:
            if N is not None and int(N) != max(int(x) for x in Nk):
                raise ValueError("N must equal max(Nk)")
            self._op = fl_coeffs_box(d, alpha, gamma, h, Nk)
        elif gamma == 2.0:
            self._op = fl_coeffs(d, alpha, h, N)
        else:
            self._op = fl_coeffs_gamma(d, alpha, gamma, h, N)
        self.desc = fl_op_describe(self._op)
        for k, v in self.desc.items():
            setattr(self, k, v)

    @property
    def handle(self):
        return self._op

    def apply(self, u, y=None, stream=None):
        import torch
        if u.numel() != self.M:
            raise ValueError("expected %d entries, got %d" % (self.M, u.numel()))
        if y is None:
            y = torch.empty_like(u)
        elif y.numel() != self.M:
            raise ValueError("expected %d entries, got %d" % (self.M, y.numel()))
        return fl_apply(self._op, u, y, stream)

    def residual(self, f, u, r=None, stream=None):
        """r = f - A u (float64); a new vector unless r is given (r may be f)."""
        import torch
        for t in (f, u):
            if t.numel() != self.M:
                raise ValueError("expected %d entries, got %d" % (self.M, t.numel()))
        if r is None:
            r = torch.empty_like(f)
        return fl_residual(self._op, f, u, r, stream)

    def tau_apply(self, r, z=None, s0=0.0, s1=1.0, stream=None):
        """The sine-transform preconditioner of s0 I + s1 A applied to r (float64)."""
        import torch
        if r.numel() != self.M:
            raise ValueError("expected %d entries, got %d" % (self.M, r.numel()))
        if z is None:
            z = torch.empty_like(r)
        elif z.numel() != self.M:
            raise ValueError("expected %d entries, got %d" % (self.M, z.numel()))
        return fl_tau_apply(self._op, r, z, s0, s1, stream)

    def poisson_solve(self, f, tol=1e-8, u=None, stream=None, **kw):
        import torch
        if u is None:
            u = torch.zeros_like(f)
        info = fl_poisson_solve_ex(self._op, f, tol, u, stream=stream, **kw)
        return u, info

    def allen_cahn_step(self, u, tau, eps, theta=0.5, tol=1e-8, solver="auto", stream=None):
        return fl_allen_cahn_step_ex(self._op, u, tau, eps, theta, tol, solver, stream)

    def allen_cahn_step_gen(self, u, tau, kappa, gamma, shift, theta=0.5, tol=1e-8, solver="auto", stream=None):
        return fl_allen_cahn_step_gen(self._op, u, tau, kappa, gamma, shift, theta, tol, solver, stream)

    def coeffs(self):
        return fl_get_coeffs(self._op)

    def set_preconditioner(self, net):
        """Attach a UNet (kept alive by this operator) for solver='fpcg'; None detaches."""
        fl_set_preconditioner(self._op, net.handle if net is not None else None)
        self._net = net

    def variants(self, prec):
        return [fl_variant_info(self._op, prec, k) for k in range(fl_variant_count(self._op, prec))]

    def select_variant(self, prec, k):
        fl_select_variant(self._op, prec, k)

    def tune(self, prec):
        """The variant for this operator's (d, FFT length, prec) from the on-disk tuning cache."""
        return fl_tune(self._op, prec)

    def autotune(self, prec, reps=20, stream=None):
        return fl_autotune(self._op, prec, reps, stream)

    def symbol(self):
        return fl_get_symbol(self._op)

    def close(self):
        if getattr(self, "_op", None):
            fl_op_destroy(self._op)
            self._op = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
