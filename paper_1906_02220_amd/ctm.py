"""Python binding of the C ABI in include/ctm.h (argument marshalling only).

Every function of the header is exposed under its own name with the same
arguments (numpy arrays for host buffers); the classes ``Context`` and
``Environment`` wrap them for convenience.  All computation happens in the
HIP library; if ``libctm.so`` is missing or cannot be loaded, importing the
library raises instead of falling back to anything else.

When torch is used in the same process, import torch before the library is
first loaded: torch ships its own HIP runtime, and loading it first makes the
library bind to that one instead of starting a second runtime beside it (with
which torch would then find no device).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctm.so")

CTM_OK = 0
CTM_ENOTCONV = 1
CTM_EINVAL = -1
CTM_ENOMEM = -2
CTM_EDEVICE = -3
CTM_ENUMERIC = -4

CTM_PREC_F64 = 0
CTM_PREC_F32 = 1
CTM_PREC_BF16X3 = 3
CTM_PREC_BF16X4 = 4

_STATUS_NAMES = {0: "CTM_OK", 1: "CTM_ENOTCONV", -1: "CTM_EINVAL", -2: "CTM_ENOMEM",
                 -3: "CTM_EDEVICE", -4: "CTM_ENUMERIC"}


class CtmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(code, code), msg))
        self.code = code


class ctm_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int),
                ("eps_cut", ctypes.c_double),
                ("svd_block", ctypes.c_int),
                ("svd_iters", ctypes.c_int),
                ("svd_iters_cold", ctypes.c_int),
                ("seed", ctypes.c_ulonglong),
                ("boundary", ctypes.POINTER(ctypes.c_double)),
                ("svd_oversample", ctypes.c_int),
                ("svd_tol", ctypes.c_double),
                ("move_order", ctypes.c_int * 4)]


class ctm_grad_info(ctypes.Structure):
    _fields_ = [("moves", ctypes.c_int),
                ("cg_iters_max", ctypes.c_int),
                ("cg_iters_total", ctypes.c_longlong),
                ("ms_forward", ctypes.c_double),
                ("ms_recompute", ctypes.c_double),
                ("ms_backward", ctypes.c_double),
                ("tape_bytes", ctypes.c_double),
                ("checkpoint_bytes", ctypes.c_double)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_LL = ctypes.POINTER(ctypes.c_longlong)

# name -> (restype, argtypes); mirrors include/ctm.h
SIGNATURES = {
    "ctm_opts_default": (None, [ctypes.POINTER(ctm_opts)]),
    "ctm_context_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P)]),
    "ctm_context_destroy": (None, [_P]),
    "ctm_last_error": (ctypes.c_char_p, [_P]),
    "ctm_context_set_stream": (ctypes.c_int, [_P, _P]),
    "ctm_context_set_graphs": (ctypes.c_int, [_P, ctypes.c_int]),
    "ctm_context_set_autotune": (ctypes.c_int, [_P, ctypes.c_int]),
    "ctm_env_init_tensor": (ctypes.c_int, [_P, _D, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctm_opts), ctypes.POINTER(_P)]),
    "ctm_env_init_purification": (ctypes.c_int, [_P, _D, _D, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int, ctypes.c_int,
                                                 ctypes.POINTER(ctm_opts), ctypes.POINTER(_P)]),
    "ctm_env_init_tensor_dev": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctm_opts), ctypes.POINTER(_P)]),
    "ctm_env_init_purification_dev": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int,
                                                     ctypes.c_int, ctypes.c_int,
                                                     ctypes.POINTER(ctm_opts), ctypes.POINTER(_P)]),
    "ctm_env_destroy": (None, [_P]),
    "ctm_sweep": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, _I, _D]),
    "ctm_sweep_batch": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, _I, _D]),
    "ctm_sweep_batch_grouped": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int,
                                               ctypes.c_double, _I, _D]),
    "ctm_move": (ctypes.c_int, [_P, ctypes.c_int]),
    "ctm_norm": (ctypes.c_int, [_P, _D]),
    "ctm_log_z": (ctypes.c_int, [_P, _D, _D]),
    "ctm_bond_metric": (ctypes.c_int, [_P, _D, ctypes.c_size_t]),
    "ctm_expect": (ctypes.c_int, [_P, _D, ctypes.c_int, _D]),
    "ctm_expect_noalloc": (ctypes.c_int, [_P, _D, ctypes.c_int, _D]),
    "ctm_expect_tensor": (ctypes.c_int, [_P, _D, _D]),
    "ctm_corner_spectra": (ctypes.c_int, [_P, _D, ctypes.c_size_t]),
    "ctm_env_get": (ctypes.c_int, [_P, _D, _D, _D]),
    "ctm_env_set": (ctypes.c_int, [_P, _D, _D, _D]),
    "ctm_env_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "ctm_env_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "ctm_env_dims": (ctypes.c_int, [_P, _I, _I, _I, _I]),
    "ctm_svd_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.POINTER(ctypes.c_longlong), _D]),
    "ctm_debug_poison_allocations": (ctypes.c_int, [ctypes.c_int, _I]),
    "ctm_debug_guard_violations": (ctypes.c_int, [ctypes.POINTER(ctypes.c_longlong)]),
    "ctm_grad_purification": (ctypes.c_int, [_P, _D, _D, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.POINTER(ctm_opts), ctypes.c_int,
                                             ctypes.c_int, _D, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_double, _D, _D, _D, _D,
                                             ctypes.POINTER(ctm_grad_info)]),
    "ctm_grad_tensor": (ctypes.c_int, [_P, _D, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctm_opts), ctypes.c_int, ctypes.c_int, _D,
                                       ctypes.c_double, ctypes.c_double, _D, _D, _D,
                                       ctypes.POINTER(ctm_grad_info)]),
    "ctm_grad_purification_dev": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int, ctypes.c_int,
                                                 ctypes.POINTER(ctm_opts), ctypes.c_int,
                                                 ctypes.c_int, _D, ctypes.c_int, ctypes.c_double,
                                                 ctypes.c_double, _D, _D, _P, _P,
                                                 ctypes.POINTER(ctm_grad_info)]),
    "ctm_grad_tensor_dev": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctm_opts), ctypes.c_int, ctypes.c_int,
                                           _D, ctypes.c_double, ctypes.c_double, _D, _D, _P,
                                           ctypes.POINTER(ctm_grad_info)]),
    "ctm_fu_bond_update": (ctypes.c_int, [_P, _D, _D, ctypes.c_int, ctypes.c_int, _D,
                                          ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctm_opts),
                                          ctypes.c_int, ctypes.c_int, _D, _D, _D]),
    "ctm_fu_trotter_step": (ctypes.c_int, [_P, _D, _D, ctypes.c_int, _D, ctypes.c_double,
                                           ctypes.c_int, ctypes.POINTER(ctm_opts), ctypes.c_int,
                                           ctypes.c_int, _D]),
    "ctm_transfer_spectrum": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, _D, _D, _D]),
    "ctm_timing_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "ctm_timing_reset": (ctypes.c_int, [_P]),
    "ctm_timing_get": (ctypes.c_int, [_P, ctypes.c_int, _LL, _D, _D]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libctm.so and declare every entry point; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libctm.so is not built (%s); run python -m paper_1906_02220_amd.build"
                          % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _on_gpu(x):
    """A torch tensor in GPU memory (checked without importing torch)."""
    return bool(getattr(x, "is_cuda", False))


def _gpu_f64(x):
    """Contiguous FP64 copy (or x itself) of a GPU tensor, with the producing
    stream drained so that the library's stream may read it."""
    import torch
    y = x.detach().to(dtype=torch.float64).contiguous()
    torch.cuda.current_stream(y.device).synchronize()
    return y


def _module_fn(name):
    def call(*args):
        return getattr(load_library(), name)(*args)
    call.__name__ = name
    call.__doc__ = "Direct call of %s (see include/ctm.h)." % name
    return call


for _name in SIGNATURES:
    globals()[_name] = _module_fn(_name)


def default_opts(**kw):
    o = ctm_opts()
    load_library().ctm_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "boundary":
            continue
        if k == "move_order":
            v = (ctypes.c_int * 4)(*[int(x) for x in v])
        setattr(o, k, v)
    return o


class Context:
    """One HIP device (must be gfx950) with its stream."""

    def __init__(self, device=0):
        lib = load_library()
        h = _P()
        rc = lib.ctm_context_create(device, ctypes.byref(h))
        if rc != CTM_OK:
            raise CtmError(rc, "ctm_context_create(%d) failed" % device)
        self.h = h
        self.lib = lib

    def check(self, rc, what):
        if rc < 0:
            raise CtmError(rc, "%s: %s" % (what, self.lib.ctm_last_error(self.h).decode()))
        return rc

    def set_stream(self, stream_ptr):
        self.check(self.lib.ctm_context_set_stream(self.h, _P(stream_ptr)), "set_stream")

    def graphs(self, on=True):
        """Replay warm sweeps of this context's environments from HIP graphs."""
        self.check(self.lib.ctm_context_set_graphs(self.h, 1 if on else 0), "set_graphs")

    def autotune(self, on=True):
        """Time the candidate tilings of each large product shape once and keep the fastest."""
        self.check(self.lib.ctm_context_set_autotune(self.h, 1 if on else 0), "set_autotune")

    def timing(self, on=True):
        self.check(self.lib.ctm_timing_enable(self.h, 1 if on else 0), "timing_enable")

    def timing_reset(self):
        self.check(self.lib.ctm_timing_reset(self.h), "timing_reset")

    def timing_get(self, cls):
        c = ctypes.c_longlong()
        ms = ctypes.c_double()
        fl = ctypes.c_double()
        self.check(self.lib.ctm_timing_get(self.h, cls, ctypes.byref(c), ctypes.byref(ms),
                                           ctypes.byref(fl)), "timing_get")
        return c.value, ms.value, fl.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.ctm_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sweep_batch(envs, max_sweeps, tol=0.0, grouped=False):
    """Sweeps of several environments at once: ctm_sweep_batch (environments
    on different contexts run concurrently) or, with grouped=True,
    ctm_sweep_batch_grouped (lock-step moves whose n x n x n products run as
    grouped launches).  Returns (rc, sweeps_done, delta) with one entry per
    environment."""
    envs = list(envs)
    n = len(envs)
    if n == 0:
        return CTM_OK, np.zeros(0, np.int32), np.zeros(0)
    arr = (_P * n)(*[e.h for e in envs])
    done = np.zeros(n, dtype=np.int32)
    delta = np.zeros(n)
    lib = load_library()
    name = "ctm_sweep_batch_grouped" if grouped else "ctm_sweep_batch"
    rc = getattr(lib, name)(arr, n, max_sweeps, tol, done.ctypes.data_as(_I),
                            delta.ctypes.data_as(_D))
    envs[0].ctx.check(rc, name)
    return rc, done, delta


def poison_allocations(on):
    """ctm_debug_poison_allocations: while on, every device buffer the library
    allocates starts as all-ones bytes (NaN doubles), so that reads of memory
    it never wrote show up in the results, and sits between guard bands that
    are checked when it is freed (guard_violations()).  Returns the previous
    state."""
    prev = ctypes.c_int()
    load_library().ctm_debug_poison_allocations(1 if on else 0, ctypes.byref(prev))
    return bool(prev.value)


def guard_violations():
    """ctm_debug_guard_violations: damaged guard bands of poisoned buffers
    found so far (each is a write past the end of a library buffer)."""
    n = ctypes.c_longlong()
    load_library().ctm_debug_guard_violations(ctypes.byref(n))
    return n.value


def _info_dict(info):
    return {name: getattr(info, name) for name, _ in ctm_grad_info._fields_}


def grad_purification(ctx, A, B, gamma, chi, sweeps, op=None, w_log_kappa=1.0, w_expect=0.0,
                      checkpoint_every=0, **kw):
    """ctm_grad_purification: gradient of w_log_kappa ln(kappa) + w_expect <op>
    after `sweeps` sweeps.  Returns (log_kappa, expect, dA, dB, info).  With
    A and B torch tensors in GPU memory the call goes through
    ctm_grad_purification_dev and dA, dB are FP64 torch tensors on that GPU;
    otherwise they are NumPy arrays."""
    if _on_gpu(A) and _on_gpu(B):
        return _grad_purification_dev(ctx, A, B, gamma, chi, sweeps, op, w_log_kappa, w_expect,
                                      checkpoint_every, **kw)
    A = _f64(A)
    B = _f64(B)
    if A.shape != B.shape or A.ndim != 5 or A.shape[:2] != (2, 2):
        raise ValueError("A and B must both have shape (2, 2, Dx, Dy, Dz)")
    dims = list(A.shape[2:])
    Dg = dims[gamma]
    rest = [dims[i] for i in range(3) if i != gamma]
    if rest[0] != rest[1]:
        raise ValueError("the two non-fused bonds must share one dimension D")
    o = default_opts(**kw)
    opp, op_dim = None, 0
    if op is not None:
        opp = _f64(op)
        op_dim = opp.shape[0]
    gA = np.zeros_like(A)
    gB = np.zeros_like(B)
    lk = ctypes.c_double()
    ex = ctypes.c_double()
    info = ctm_grad_info()
    rc = ctx.lib.ctm_grad_purification(ctx.h, _dptr(A), _dptr(B), rest[0], Dg, gamma, chi,
                                       ctypes.byref(o), sweeps, checkpoint_every,
                                       _dptr(opp) if opp is not None else None, op_dim,
                                       w_log_kappa, w_expect, ctypes.byref(lk), ctypes.byref(ex),
                                       _dptr(gA), _dptr(gB), ctypes.byref(info))
    ctx.check(rc, "ctm_grad_purification")
    return lk.value, ex.value, gA, gB, _info_dict(info)


def _grad_purification_dev(ctx, A, B, gamma, chi, sweeps, op, w_log_kappa, w_expect,
                           checkpoint_every, **kw):
    import torch
    A = _gpu_f64(A)
    B = _gpu_f64(B)
    if A.shape != B.shape or A.dim() != 5 or tuple(A.shape[:2]) != (2, 2):
        raise ValueError("A and B must both have shape (2, 2, Dx, Dy, Dz)")
    dims = list(A.shape[2:])
    Dg = dims[gamma]
    rest = [dims[i] for i in range(3) if i != gamma]
    if rest[0] != rest[1]:
        raise ValueError("the two non-fused bonds must share one dimension D")
    o = default_opts(**kw)
    opp, op_dim = None, 0
    if op is not None:
        opp = _f64(op.detach().cpu().numpy() if torch.is_tensor(op) else op)
        op_dim = opp.shape[0]
    gA = torch.empty_like(A)
    gB = torch.empty_like(B)
    lk = ctypes.c_double()
    ex = ctypes.c_double()
    info = ctm_grad_info()
    rc = ctx.lib.ctm_grad_purification_dev(
        ctx.h, _P(A.data_ptr()), _P(B.data_ptr()), rest[0], Dg, gamma, chi, ctypes.byref(o), sweeps,
        checkpoint_every, _dptr(opp) if opp is not None else None, op_dim, w_log_kappa, w_expect,
        ctypes.byref(lk), ctypes.byref(ex), _P(gA.data_ptr()), _P(gB.data_ptr()), ctypes.byref(info))
    ctx.check(rc, "ctm_grad_purification_dev")
    return lk.value, ex.value, gA, gB, _info_dict(info)


def grad_tensor(ctx, a, chi, sweeps, a_imp=None, w_log_kappa=1.0, w_expect=0.0,
                checkpoint_every=0, **kw):
    """ctm_grad_tensor: gradient of w_log_kappa ln(kappa) + w_expect <E,a_imp>/<E,a>
    with respect to the site tensor a.  Returns (log_kappa, expect, da, info).
    With a a torch tensor in GPU memory the call goes through
    ctm_grad_tensor_dev and da is an FP64 torch tensor on that GPU."""
    dev = _on_gpu(a)
    if dev:
        import torch
        a = _gpu_f64(a)
        if torch.is_tensor(a_imp):
            a_imp = a_imp.detach().cpu().numpy()
    else:
        a = _f64(a)
    d = a.shape[0]
    if tuple(a.shape) != (d, d, d, d):
        raise ValueError("a must have shape (d, d, d, d)")
    o = default_opts(**kw)
    ai = _f64(a_imp) if a_imp is not None else None
    lk = ctypes.c_double()
    ex = ctypes.c_double()
    info = ctm_grad_info()
    if dev:
        ga = torch.empty_like(a)
        rc = ctx.lib.ctm_grad_tensor_dev(ctx.h, _P(a.data_ptr()), d, chi, ctypes.byref(o), sweeps,
                                         checkpoint_every, _dptr(ai) if ai is not None else None,
                                         w_log_kappa, w_expect, ctypes.byref(lk), ctypes.byref(ex),
                                         _P(ga.data_ptr()), ctypes.byref(info))
        ctx.check(rc, "ctm_grad_tensor_dev")
        return lk.value, ex.value, ga, _info_dict(info)
    ga = np.zeros_like(a)
    lk = ctypes.c_double()
    ex = ctypes.c_double()
    info = ctm_grad_info()
    rc = ctx.lib.ctm_grad_tensor(ctx.h, _dptr(a), d, chi, ctypes.byref(o), sweeps,
                                 checkpoint_every, _dptr(ai) if ai is not None else None,
                                 w_log_kappa, w_expect, ctypes.byref(lk), ctypes.byref(ex),
                                 _dptr(ga), ctypes.byref(info))
    ctx.check(rc, "ctm_grad_tensor")
    return lk.value, ex.value, ga, _info_dict(info)


def fu_bond_update(ctx, A, B, gamma, H, tau, chi, sweeps, als_iters, **kw):
    """ctm_fu_bond_update: returns (A'', B'', errors) for A, B of shape
    (2, 2, D, D, D)."""
    A = _f64(A)
    B = _f64(B)
    D = A.shape[2]
    if A.shape != (2, 2, D, D, D) or B.shape != A.shape:
        raise ValueError("A and B must both have shape (2, 2, D, D, D)")
    Hc = _f64(H)
    o = default_opts(**kw)
    A2 = np.zeros_like(A)
    B2 = np.zeros_like(B)
    errs = np.zeros(als_iters + 1)
    rc = ctx.lib.ctm_fu_bond_update(ctx.h, _dptr(A), _dptr(B), D, gamma, _dptr(Hc), tau, chi,
                                    ctypes.byref(o), sweeps, als_iters, _dptr(A2), _dptr(B2),
                                    _dptr(errs))
    ctx.check(rc, "ctm_fu_bond_update")
    return A2, B2, errs


def fu_trotter_step(ctx, A, B, H3, dbeta, chi, sweeps, als_iters, **kw):
    """ctm_fu_trotter_step: returns (A, B, errors[5, als_iters + 1]) after one
    second-order Trotter step with bond terms H3 = (H_x, H_y, H_z)."""
    A = _f64(A).copy()
    B = _f64(B).copy()
    D = A.shape[2]
    if A.shape != (2, 2, D, D, D) or B.shape != A.shape:
        raise ValueError("A and B must both have shape (2, 2, D, D, D)")
    Hs = _f64(np.stack([np.asarray(h, dtype=np.float64) for h in H3]))
    o = default_opts(**kw)
    errs = np.zeros((5, als_iters + 1))
    rc = ctx.lib.ctm_fu_trotter_step(ctx.h, _dptr(A), _dptr(B), D, _dptr(Hs), dbeta, chi,
                                     ctypes.byref(o), sweeps, als_iters, _dptr(errs))
    ctx.check(rc, "ctm_fu_trotter_step")
    return A, B, errs


class Environment:
    """CTMRG environment owned by the library."""

    def __init__(self, ctx, handle, keep=()):
        self.ctx = ctx
        self.h = handle
        self._keep = keep
        chi = ctypes.c_int()
        d = ctypes.c_int()
        D = ctypes.c_int()
        sw = ctypes.c_int()
        ctx.lib.ctm_env_dims(self.h, ctypes.byref(chi), ctypes.byref(d), ctypes.byref(D),
                             ctypes.byref(sw))
        self.chi, self.d, self.D = chi.value, d.value, D.value

    @staticmethod
    def _opts(boundary, kw):
        o = default_opts(**kw)
        keep = ()
        if boundary is not None:
            bb = _f64(boundary)
            o.boundary = _dptr(bb)
            keep = (bb,)
        return o, keep

    @classmethod
    def from_tensor(cls, ctx, a, chi, boundary=None, **kw):
        """a: (d, d, d, d) array, or a torch tensor on the GPU (read in place
        through ctm_env_init_tensor_dev)."""
        dev = _on_gpu(a)
        a = _gpu_f64(a) if dev else _f64(a)
        d = a.shape[0]
        if tuple(a.shape) != (d, d, d, d):
            raise ValueError("a must have shape (d, d, d, d)")
        o, keep = cls._opts(boundary, kw)
        h = _P()
        if dev:
            rc = ctx.lib.ctm_env_init_tensor_dev(ctx.h, _P(a.data_ptr()), d, chi, ctypes.byref(o),
                                                 ctypes.byref(h))
            ctx.check(rc, "ctm_env_init_tensor_dev")
        else:
            ctx.check(ctx.lib.ctm_env_init_tensor(ctx.h, _dptr(a), d, chi, ctypes.byref(o),
                                                  ctypes.byref(h)), "ctm_env_init_tensor")
        return cls(ctx, h, keep)

    @classmethod
    def from_purification(cls, ctx, A, B, gamma, chi, boundary=None, **kw):
        """A, B: (2, 2, Dx, Dy, Dz) arrays, or torch tensors on the GPU (read in
        place through ctm_env_init_purification_dev)."""
        dev = _on_gpu(A)
        if dev != _on_gpu(B):
            raise ValueError("A and B must both be host arrays or both GPU tensors")
        A, B = (_gpu_f64(A), _gpu_f64(B)) if dev else (_f64(A), _f64(B))
        if tuple(A.shape) != tuple(B.shape) or A.ndim != 5 or tuple(A.shape[:2]) != (2, 2):
            raise ValueError("A and B must both have shape (2, 2, Dx, Dy, Dz)")
        if gamma not in (0, 1, 2):
            raise ValueError("gamma must be 0 (x), 1 (y) or 2 (z)")
        dims = list(A.shape[2:])
        Dg = dims[gamma]
        rest = [dims[i] for i in range(3) if i != gamma]
        if rest[0] != rest[1]:
            raise ValueError("the two non-fused bonds must share one dimension D")
        o, keep = cls._opts(boundary, kw)
        h = _P()
        if dev:
            rc = ctx.lib.ctm_env_init_purification_dev(ctx.h, _P(A.data_ptr()), _P(B.data_ptr()),
                                                       rest[0], Dg, gamma, chi, ctypes.byref(o),
                                                       ctypes.byref(h))
            ctx.check(rc, "ctm_env_init_purification_dev")
        else:
            ctx.check(ctx.lib.ctm_env_init_purification(ctx.h, _dptr(A), _dptr(B), rest[0], Dg,
                                                        gamma, chi, ctypes.byref(o),
                                                        ctypes.byref(h)),
                      "ctm_env_init_purification")
        return cls(ctx, h, keep)

    def sweep(self, max_sweeps, tol=0.0):
        done = ctypes.c_int()
        delta = ctypes.c_double()
        rc = self.ctx.check(self.ctx.lib.ctm_sweep(self.h, max_sweeps, tol, ctypes.byref(done),
                                                   ctypes.byref(delta)), "ctm_sweep")
        return rc, done.value, delta.value

    def move(self, direction):
        self.ctx.check(self.ctx.lib.ctm_move(self.h, direction), "ctm_move")

    def norm(self):
        k = ctypes.c_double()
        self.ctx.check(self.ctx.lib.ctm_norm(self.h, ctypes.byref(k)), "ctm_norm")
        return k.value

    def log_z(self):
        la = ctypes.c_double()
        sg = ctypes.c_double()
        self.ctx.check(self.ctx.lib.ctm_log_z(self.h, ctypes.byref(la), ctypes.byref(sg)),
                       "ctm_log_z")
        return la.value, sg.value

    def bond_metric(self):
        n = self.d ** 4
        out = np.empty(n)
        self.ctx.check(self.ctx.lib.ctm_bond_metric(self.h, _dptr(out), n), "ctm_bond_metric")
        if self.D > 0:
            return out.reshape((self.D,) * 8)
        return out.reshape((self.d,) * 4)

    def expect(self, op):
        op = _f64(op)
        dim = op.shape[0]
        v = ctypes.c_double()
        self.ctx.check(self.ctx.lib.ctm_expect(self.h, _dptr(op), dim, ctypes.byref(v)),
                       "ctm_expect")
        return v.value

    def expect_tensor(self, a_imp):
        a_imp = _f64(a_imp)
        v = ctypes.c_double()
        self.ctx.check(self.ctx.lib.ctm_expect_tensor(self.h, _dptr(a_imp), ctypes.byref(v)),
                       "ctm_expect_tensor")
        return v.value

    def transfer_spectrum(self, direction=0, site=True, nev=4, krylov=40):
        """Leading transfer-matrix eigenvalues (complex, by decreasing
        magnitude) and the correlation length (ctm_transfer_spectrum)."""
        re = np.zeros(nev)
        im = np.zeros(nev)
        xi = ctypes.c_double()
        self.ctx.check(self.ctx.lib.ctm_transfer_spectrum(self.h, direction, 1 if site else 0, nev,
                                                          krylov, _dptr(re), _dptr(im),
                                                          ctypes.byref(xi)),
                       "ctm_transfer_spectrum")
        return re + 1j * im, xi.value

    def svd_stats(self):
        """(truncated SVDs by subspace iteration, their iterations, residual
        max_i ||M u_i - s_i v_i|| / s_1 of the last move's kept triplets)."""
        calls, iters, res = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_double()
        self.ctx.check(self.ctx.lib.ctm_svd_stats(self.h, ctypes.byref(calls), ctypes.byref(iters),
                                                  ctypes.byref(res)), "ctm_svd_stats")
        return calls.value, iters.value, res.value

    def corner_spectra(self):
        out = np.empty(4 * self.chi)
        self.ctx.check(self.ctx.lib.ctm_corner_spectra(self.h, _dptr(out), out.size),
                       "ctm_corner_spectra")
        return out.reshape(4, self.chi)

    def get(self):
        C = np.empty((4, self.chi, self.chi))
        T = np.empty((4, self.chi, self.d, self.chi))
        L = np.empty(8)
        self.ctx.check(self.ctx.lib.ctm_env_get(self.h, _dptr(C), _dptr(T), _dptr(L)),
                       "ctm_env_get")
        return C, T, L

    def set(self, C, T, L):
        C, T, L = _f64(C), _f64(T), _f64(L)
        self.ctx.check(self.ctx.lib.ctm_env_set(self.h, _dptr(C), _dptr(T), _dptr(L)),
                       "ctm_env_set")

    def save(self, path):
        self.ctx.check(self.ctx.lib.ctm_env_save(self.h, path.encode()), "ctm_env_save")

    def load(self, path):
        self.ctx.check(self.ctx.lib.ctm_env_load(self.h, path.encode()), "ctm_env_load")

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.ctm_env_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
