"""MI355X-native modular polynomial multiplication (NTT / TFT convolution over Z/pZ).

Thin ctypes binding over the C ABI of ``libpolymul.so`` (declared in
``include/polymul.h``).  PyTorch supplies device memory and the current HIP
stream; every step of every product runs in the library's HIP kernels.  If
the library has not been built the calls raise: there is no fallback.

    import torch, paper_1609_01010_amd as pm
    a = torch.randint(0, 998244353, (1024,), dtype=torch.int64).to(torch.uint32).cuda()
    c = pm.poly_mul(a, a, 998244353)          # 2047 coefficients, uint32
"""

from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolymul.so")

PRIMES = (998244353, 2013265921, 469762049, 167772161)

PM_OK, PM_EINVAL, PM_EUNSUPPORTED, PM_ETOOLARGE, PM_ENOTREDUCED, PM_ENOMEM, PM_EDEVICE = range(7)
CTX_SINGLE, CTX_BATCH = 0, 1  # tuning contexts: a product alone, one of a batch
POLICY_DEFAULT, POLICY_EXHAUSTIVE, POLICY_LEARNED = range(3)
# plan kinds: defining sum, one work-group in LDS, four-step, general radix (q 2^k)
PLAN_DIRECT, PLAN_LDS, PLAN_FOURSTEP, PLAN_MIXED = range(4)


class PolymulError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _status_str(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")


class Plan(ctypes.Structure):
    """Mirror of pm_plan."""

    _fields_ = [
        ("kind", ctypes.c_int32),
        ("log_l", ctypes.c_int32),
        ("log_ra", ctypes.c_int32),
        ("log_rb", ctypes.c_int32),
        ("log_c", ctypes.c_int32),
        ("ma", ctypes.c_int32),
        ("lq", ctypes.c_int32),
        ("lnt", ctypes.c_int32),
        ("q", ctypes.c_int32),
    ]

    def as_tuple(self):
        return tuple(getattr(self, f) for f, _ in self._fields_)

    def __repr__(self):
        return "Plan(" + ", ".join(f"{f}={getattr(self, f)}" for f, _ in self._fields_) + ")"


class Problem(ctypes.Structure):
    """Mirror of pm_problem."""

    _fields_ = [
        ("a", ctypes.c_void_p),
        ("len_a", ctypes.c_size_t),
        ("b", ctypes.c_void_p),
        ("len_b", ctypes.c_size_t),
        ("p", ctypes.c_uint32),
        ("c", ctypes.c_void_p),
    ]


_lib = None
_lock = threading.Lock()

# exported functions: name -> (restype, argtypes)
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_u32 = ctypes.c_uint32
_int = ctypes.c_int
SIGNATURES = {
    "pm_status_str": (ctypes.c_char_p, [_int]),
    "pm_init": (_int, []),
    "pm_poly_mul": (_int, [_vp, _sz, _vp, _sz, _u32, _vp, _vp]),
    "pm_poly_mul_noalloc": (_int, [_vp, _sz, _vp, _sz, _u32, _vp, _vp]),
    "pm_poly_mul_batch": (_int, [ctypes.POINTER(Problem), _sz, _vp]),
    "pm_batch_plans_used": (_int, [_vp, ctypes.POINTER(Plan), _sz]),
    "pm_cyclic_mul": (_int, [_vp, _sz, _vp, _sz, _sz, _u32, _vp, _vp]),
    "pm_poly_mul_mixed": (_int, [_vp, _sz, _vp, _sz, _u32, _u32, _vp, _vp]),
    "pm_workspace_query": (_int, [_sz, _sz, _u32, ctypes.POINTER(ctypes.c_size_t)]),
    "pm_batch_workspace_query": (_int, [ctypes.POINTER(Problem), _sz, ctypes.POINTER(ctypes.c_size_t)]),
    "pm_int_mul_workspace_query": (_int, [_sz, _sz, ctypes.POINTER(ctypes.c_size_t)]),
    "pm_set_workspace": (_int, [_vp, _vp, _sz]),
    "pm_poly_mul_multi": (_int, [_vp, ctypes.POINTER(_sz), _vp, ctypes.POINTER(_sz), _int, _u32, _vp, _vp]),
    "pm_negacyclic_mul": (_int, [_vp, _sz, _vp, _sz, _sz, _u32, _vp, _vp]),
    "pm_int_mul": (_int, [_vp, _sz, _vp, _sz, _vp, _vp]),
    "pm_int_mul_digits": (_int, [_vp, _sz, _vp, _sz, ctypes.c_int, _vp, _vp]),
    "pm_int_mul_digits_workspace_query": (_int, [_sz, _sz, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "pm_ntt": (_int, [_vp, _vp, _sz, _u32, _int, _vp]),
    "pm_tft": (_int, [_vp, _sz, _sz, _sz, _u32, _vp, _vp]),
    "pm_itft": (_int, [_vp, _sz, _sz, _u32, _vp, _vp]),
    "pm_itft_granularity": (_sz, [_sz]),
    "pm_stream_check": (_int, [_vp]),
    "pm_set_policy": (_int, [_int]),
    "pm_get_policy": (_int, []),
    "pm_config_from_env": (_int, []),
    "pm_plan_for": (_int, [_sz, _u32, ctypes.POINTER(Plan)]),
    "pm_plan_for_ctx": (_int, [_sz, _u32, _int, ctypes.POINTER(Plan)]),
    "pm_poly_mul_plan": (_int, [_vp, _sz, _vp, _sz, _u32, _vp, ctypes.POINTER(Plan), _vp]),
    "pm_plan_candidates": (_sz, [_sz, _u32, ctypes.POINTER(Plan), _sz]),
    "pm_plan_cache_put": (_int, [_sz, _u32, ctypes.POINTER(Plan)]),
    "pm_plan_cache_clear": (None, []),
    "pm_tune": (_int, [ctypes.POINTER(_sz), _sz, _u32, _int, _vp]),
    "pm_tune_ctx": (_int, [ctypes.POINTER(_sz), _sz, _u32, _int, _int, _vp]),
    "pm_time_plan": (_int, [_sz, _u32, ctypes.POINTER(Plan), _int, ctypes.POINTER(ctypes.c_double)]),
    "pm_time_plan_ctx": (_int, [_sz, _u32, ctypes.POINTER(Plan), _int, _int, ctypes.POINTER(ctypes.c_double)]),
    "pm_tune_db_size": (_sz, []),
    "pm_tune_db_get": (_int, [_sz, ctypes.POINTER(_sz), ctypes.POINTER(_u32), ctypes.POINTER(Plan),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_int)]),
    "pm_tune_db_add": (_int, [_sz, _u32, ctypes.POINTER(Plan), ctypes.c_double, _int]),
    "pm_tune_db_clear": (None, []),
    "pm_tune_db_save": (_int, [ctypes.c_char_p]),
    "pm_tune_db_load": (_int, [ctypes.c_char_p]),
    "pm_model_features": (_int, [_sz, _u32, ctypes.POINTER(Plan), _int, ctypes.POINTER(ctypes.c_float)]),
    "pm_model_train": (_int, [ctypes.POINTER(ctypes.c_float), _int, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]),
    "pm_model_get": (_int, [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                            ctypes.POINTER(ctypes.c_float)]),
    "pm_model_set": (_int, [ctypes.POINTER(ctypes.c_float), ctypes.c_float, ctypes.c_float]),
    "pm_model_predict": (_int, [_sz, _u32, ctypes.POINTER(Plan), _sz, _int, ctypes.POINTER(ctypes.c_double)]),
    "pm_model_save": (_int, [ctypes.c_char_p]),
    "pm_model_load": (_int, [ctypes.c_char_p]),
    "pm_mlp_num_params": (_sz, []),
    "pm_mlp_forward": (_int, [ctypes.POINTER(ctypes.c_float)] * 2 + [_int, ctypes.POINTER(ctypes.c_float)]),
    "pm_mlp_loss_grad": (_int, [ctypes.POINTER(ctypes.c_float)] * 3 + [_int] + [ctypes.POINTER(ctypes.c_float)] * 2),
    "pm_mlp_adam": (_int, [ctypes.POINTER(ctypes.c_float)] * 4 + [_int, ctypes.c_float]),
    "pm_mlp_train": (_int, [ctypes.POINTER(ctypes.c_float)] * 3 + [_int, _int, ctypes.c_float,
                                                                   ctypes.POINTER(ctypes.c_float)]),
    "pm_trace_enable": (None, [_int]),
    "pm_trace_reset": (None, []),
    "pm_trace_query": (_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "pm_trace_names": (_sz, [ctypes.c_char_p, _sz]),
}


def lib():
    """Load libpolymul.so (raises if it has not been built)."""
    global _lib
    L = _lib
    if L is not None:  # loaded: no lock on the per-call path
        return L
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(
                    "libpolymul.so is not built; run `python -m paper_1609_01010_amd.build` "
                    "(there is no non-HIP fallback)"
                )
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _status_str(st: int) -> str:
    try:
        return lib().pm_status_str(st).decode()
    except ImportError:
        return "status %d" % st


def _check(st: int, what: str = ""):
    if st != PM_OK:
        raise PolymulError(st, what)


def _torch():
    import torch

    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# products

def poly_mul(a, b, p: int, out=None, plan: Plan | None = None, stream=None):
    """c_k = sum_{i+j=k} a_i b_j mod p for uint32 device tensors a, b."""
    torch = _torch()
    la, lb = a.numel(), b.numel()
    if out is None:
        out = torch.empty(max(la + lb - 1, 1), dtype=torch.uint32, device=a.device)
    args = (_dev_ptr(a, torch.uint32, "a"), la, _dev_ptr(b, torch.uint32, "b"), lb, p, _dev_ptr(out, torch.uint32, "out"))
    if plan is None:
        _check(lib().pm_poly_mul(*args, _stream(stream)), "pm_poly_mul")
    else:
        _check(lib().pm_poly_mul_plan(*args, ctypes.byref(plan), _stream(stream)), "pm_poly_mul_plan")
    return out


def init():
    """Build the twiddle tables of the four primes on the current device and
    find the allocation-free product's scratch array there."""
    _check(lib().pm_init(), "pm_init")


def poly_mul_noalloc(a, b, p: int, out, stream=None):
    """pm_poly_mul with every intermediate in the library's static scratch
    array (nothing allocated; init() first; out is required)."""
    torch = _torch()
    la, lb = a.numel(), b.numel()
    _check(lib().pm_poly_mul_noalloc(_dev_ptr(a, torch.uint32, "a"), la, _dev_ptr(b, torch.uint32, "b"), lb, p,
                                     _dev_ptr(out, torch.uint32, "out"), _stream(stream)), "pm_poly_mul_noalloc")
    return out


def poly_mul_multi(a, b, p: int, out=None, stream=None):
    """Dense multivariate product by Kronecker substitution.  a, b: uint32 device
    tensors with one dimension per variable (1 + the degree in it); returns the
    product, of shape a.shape[i] + b.shape[i] - 1."""
    torch = _torch()
    nv = a.dim()
    if b.dim() != nv:
        raise ValueError("a and b need the same number of variables")
    shape = tuple(x + y - 1 for x, y in zip(a.shape, b.shape))
    if out is None:
        out = torch.empty(shape, dtype=torch.uint32, device=a.device)
    da = (_sz * max(nv, 1))(*a.shape)
    db = (_sz * max(nv, 1))(*b.shape)
    _check(lib().pm_poly_mul_multi(_dev_ptr(a, torch.uint32, "a"), da, _dev_ptr(b, torch.uint32, "b"), db, nv, p,
                                   _dev_ptr(out, torch.uint32, "out"), _stream(stream)), "pm_poly_mul_multi")
    return out


def _ring_mul(fn, a, b, n: int, p: int, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(n, dtype=torch.uint32, device=a.device)
    _check(getattr(lib(), fn)(_dev_ptr(a, torch.uint32, "a"), a.numel(), _dev_ptr(b, torch.uint32, "b"), b.numel(), n,
                              p, _dev_ptr(out, torch.uint32, "out"), _stream(stream)), fn)
    return out


def cyclic_mul(a, b, n: int, p: int, out=None, stream=None):
    """a b mod (x^n - 1) mod p (the circular convolution); n a power of two."""
    return _ring_mul("pm_cyclic_mul", a, b, n, p, out, stream)


def negacyclic_mul(a, b, n: int, p: int, out=None, stream=None):
    """a b mod (x^n + 1) mod p (the nega-circular convolution); n a power of two."""
    return _ring_mul("pm_negacyclic_mul", a, b, n, p, out, stream)


def poly_mul_mixed(a, b, p: int, q: int, out=None, stream=None):
    """a * b mod p through a circular convolution of length q 2^k >= la + lb - 1
    (q odd, dividing p - 1)."""
    torch = _torch()
    lc = a.numel() + b.numel() - 1
    if out is None:
        out = torch.empty(lc, dtype=torch.uint32, device=a.device)
    _check(lib().pm_poly_mul_mixed(_dev_ptr(a, torch.uint32, "a"), a.numel(), _dev_ptr(b, torch.uint32, "b"),
                                   b.numel(), p, q, _dev_ptr(out, torch.uint32, "out"), _stream(stream)),
           "pm_poly_mul_mixed")
    return out


def workspace_query(len_a: int, len_b: int, p: int) -> int:
    """Workspace bytes of a product of these lengths under the current plans."""
    n = ctypes.c_size_t(0)
    _check(lib().pm_workspace_query(len_a, len_b, p, ctypes.byref(n)), "pm_workspace_query")
    return n.value


def int_mul_workspace_query(na: int, nb: int, digits=None) -> int:
    n = ctypes.c_size_t(0)
    if digits is None:
        _check(lib().pm_int_mul_workspace_query(na, nb, ctypes.byref(n)), "pm_int_mul_workspace_query")
    else:
        _check(lib().pm_int_mul_digits_workspace_query(na, nb, int(digits), ctypes.byref(n)),
               "pm_int_mul_digits_workspace_query")
    return n.value


def batch_workspace_query(problems) -> int:
    """problems: list of (a, b, p) uint32 device tensors."""
    arr = (Problem * max(len(problems), 1))()
    for i, (a, b, p) in enumerate(problems):
        arr[i].a, arr[i].len_a, arr[i].b, arr[i].len_b, arr[i].p = a.data_ptr(), a.numel(), b.data_ptr(), b.numel(), p
        arr[i].c = a.data_ptr()  # not written: the query only validates and sizes
    n = ctypes.c_size_t(0)
    _check(lib().pm_batch_workspace_query(arr, len(problems), ctypes.byref(n)), "pm_batch_workspace_query")
    return n.value


def set_workspace(buf, stream=None):
    """Use the device tensor buf as the stream's workspace (None: the library's own)."""
    if buf is None:
        _check(lib().pm_set_workspace(_stream(stream), None, 0), "pm_set_workspace")
    else:
        _check(lib().pm_set_workspace(_stream(stream), ctypes.c_void_p(buf.data_ptr()),
                                      buf.numel() * buf.element_size()), "pm_set_workspace")


class PreparedBatch:
    """A batch whose argument array is marshalled once: run() is one C call.

    problems: list of (a, b, p) uint32 device tensors; outs: optional outputs.
    The library recognises a repeated batch shape and only patches pointers,
    so repeated run() calls cost one descriptor upload and one graph launch."""

    def __init__(self, problems, outs=None):
        torch = _torch()
        self.n = len(problems)
        self.arr = (Problem * max(self.n, 1))()
        self.outs = []
        self._keep = []
        for i, (a, b, p) in enumerate(problems):
            la, lb = a.numel(), b.numel()
            c = outs[i] if outs is not None else torch.empty(la + lb - 1, dtype=torch.uint32, device=a.device)
            self.arr[i].a = _dev_ptr(a, torch.uint32, "a").value
            self.arr[i].len_a = la
            self.arr[i].b = _dev_ptr(b, torch.uint32, "b").value
            self.arr[i].len_b = lb
            self.arr[i].p = p
            self.arr[i].c = _dev_ptr(c, torch.uint32, "c").value
            self.outs.append(c)
            self._keep.append((a, b))

    def run(self, stream=None):
        _check(lib().pm_poly_mul_batch(self.arr, self.n, _stream(stream)), "pm_poly_mul_batch")
        return self.outs


def batch_plans_used(count: int, stream=None):
    """The plans the last batch of `count` problems on the stream used, in problem order."""
    arr = (Plan * max(count, 1))()
    _check(lib().pm_batch_plans_used(_stream(stream), arr, count), "pm_batch_plans_used")
    return [arr[i] for i in range(count)]


def poly_mul_batch(problems, outs=None, stream=None):
    """problems: list of (a, b, p); returns the list of products (one graph launch)."""
    return PreparedBatch(problems, outs).run(stream)


def int_mul(a, b, out=None, stream=None, digits=None):
    """Product of two little-endian 16-bit-limb integers (uint16 tensors): na + nb limbs.

    digits: None (pm_int_mul: 32-bit digits where the plans allow, else the
    limbs), or 0, 16 or 32 (pm_int_mul_digits)."""
    torch = _torch()
    na, nb = a.numel(), b.numel()
    if out is None:
        out = torch.empty(na + nb, dtype=torch.uint16, device=a.device)
    pa, pb, po = _dev_ptr(a, torch.uint16, "a"), _dev_ptr(b, torch.uint16, "b"), _dev_ptr(out, torch.uint16, "out")
    if digits is None:
        _check(lib().pm_int_mul(pa, na, pb, nb, po, _stream(stream)), "pm_int_mul")
    else:
        _check(lib().pm_int_mul_digits(pa, na, pb, nb, int(digits), po, _stream(stream)), "pm_int_mul_digits")
    return out


# ---------------------------------------------------------------------------
# transform hooks

def ntt(x, p: int, inverse: bool = False, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty_like(x)
    _check(lib().pm_ntt(_dev_ptr(x, torch.uint32, "x"), _dev_ptr(out, torch.uint32, "out"), x.numel(), p,
                        1 if inverse else 0, _stream(stream)), "pm_ntt")
    return out


def tft(x, L: int, n: int, p: int, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(n, dtype=torch.uint32, device=x.device)
    _check(lib().pm_tft(_dev_ptr(x, torch.uint32, "x"), x.numel(), L, n, p, _dev_ptr(out, torch.uint32, "out"),
                        _stream(stream)), "pm_tft")
    return out


def itft(v, L: int, p: int, out=None, stream=None):
    torch = _torch()
    n = v.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.uint32, device=v.device)
    _check(lib().pm_itft(_dev_ptr(v, torch.uint32, "v"), L, n, p, _dev_ptr(out, torch.uint32, "out"),
                         _stream(stream)), "pm_itft")
    return out


def itft_granularity(L: int) -> int:
    return int(lib().pm_itft_granularity(L))


def stream_check(stream=None) -> int:
    """Synchronise and return the deferred device status (0 = ok)."""
    return int(lib().pm_stream_check(_stream(stream)))


# ---------------------------------------------------------------------------
# plans

def set_policy(policy: int):
    _check(lib().pm_set_policy(policy), "pm_set_policy")


def get_policy() -> int:
    return int(lib().pm_get_policy())


def config_from_env():
    """Apply PM_PLAN_POLICY, PM_TUNE_DB and PM_MLP_WEIGHTS (host only)."""
    _check(lib().pm_config_from_env(), "pm_config_from_env")


def plan_for(lc: int, p: int, context: int = 0) -> Plan:
    P = Plan()
    _check(lib().pm_plan_for_ctx(lc, p, context, ctypes.byref(P)), "pm_plan_for_ctx")
    return P


def plan_candidates(lc: int, p: int, general_radix: bool = True):
    """The tuner's plans for (lc, p); general_radix=False keeps the
    power-of-two plans (kinds 0-2), the ones the batch executor and the cost
    model take."""
    n = lib().pm_plan_candidates(lc, p, None, 0)
    arr = (Plan * max(n, 1))()
    lib().pm_plan_candidates(lc, p, arr, n)
    return [arr[i] for i in range(n) if general_radix or arr[i].kind != PLAN_MIXED]


def plan_cache_put(lc: int, p: int, plan: Plan):
    _check(lib().pm_plan_cache_put(lc, p, ctypes.byref(plan)), "pm_plan_cache_put")


def plan_cache_clear():
    lib().pm_plan_cache_clear()


# ---------------------------------------------------------------------------
# tracing: per-kernel durations from HIP events recorded on the launch stream

def trace_enable(on: bool = True):
    lib().pm_trace_enable(1 if on else 0)


def trace_reset():
    lib().pm_trace_reset()


def trace_query(kernel: str):
    """(total milliseconds, number of launches) of a library kernel since the reset."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().pm_trace_query(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)), "pm_trace_query")
    return ms.value, n.value


def trace_names():
    need = lib().pm_trace_names(None, 0)
    buf = ctypes.create_string_buffer(need)
    lib().pm_trace_names(buf, need)
    return [x for x in buf.value.decode().split("\n") if x]


# ---------------------------------------------------------------------------
# the autotuner and the learned cost model

def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _f32(a):
    import numpy as np

    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def tune(lcs, p: int, reps: int = 5, stream=None, context: int = 0):
    """Time every candidate plan of each output length (context CTX_SINGLE: one
    product; CTX_BATCH: time per product of a batch); fills the database and
    the plan cache of that context."""
    arr = (ctypes.c_size_t * len(lcs))(*[int(x) for x in lcs])
    _check(lib().pm_tune_ctx(arr, len(lcs), p, reps, context, _stream(stream) if stream is not None else None),
           "pm_tune_ctx")


def time_plan(lc: int, p: int, plan: Plan, reps: int = 5, context: int = 0) -> float:
    us = ctypes.c_double()
    _check(lib().pm_time_plan_ctx(lc, p, ctypes.byref(plan), reps, context, ctypes.byref(us)), "pm_time_plan_ctx")
    return us.value


def tune_db_rows(context: int = 0):
    """[(lc, p, Plan, us)] of the timing database rows of one context."""
    out = []
    for i in range(lib().pm_tune_db_size()):
        lc = ctypes.c_size_t()
        p = ctypes.c_uint32()
        P = Plan()
        us = ctypes.c_double()
        cx = ctypes.c_int()
        _check(lib().pm_tune_db_get(i, ctypes.byref(lc), ctypes.byref(p), ctypes.byref(P), ctypes.byref(us),
                                    ctypes.byref(cx)))
        if cx.value == context:
            out.append((lc.value, p.value, P, us.value))
    return out


def tune_db_add(lc: int, p: int, plan: Plan, us: float, context: int = 0):
    _check(lib().pm_tune_db_add(lc, p, ctypes.byref(plan), us, context), "pm_tune_db_add")


def tune_db_clear():
    lib().pm_tune_db_clear()


def tune_db_save(path: str):
    _check(lib().pm_tune_db_save(path.encode()), "pm_tune_db_save")


def tune_db_load(path: str):
    _check(lib().pm_tune_db_load(path.encode()), "pm_tune_db_load")


def mlp_num_params() -> int:
    return int(lib().pm_mlp_num_params())


def model_features(lc: int, p: int, plan: Plan, context: int = 0):
    import numpy as np

    from .inputs import MLP_F

    f = np.zeros(MLP_F, dtype=np.float32)
    _check(lib().pm_model_features(lc, p, ctypes.byref(plan), context, _fptr(f)), "pm_model_features")
    return f


def model_train(init=None, steps: int = 2000, lr: float = 3e-3):
    """Train on the timing database (device kernels); returns the loss per step."""
    import numpy as np

    losses = np.zeros(steps, dtype=np.float32)
    ip = _fptr(_f32(init)) if init is not None else None
    if init is not None:
        keep = _f32(init)
        ip = _fptr(keep)
    _check(lib().pm_model_train(ip, steps, lr, _fptr(losses)), "pm_model_train")
    return losses


def model_get():
    import numpy as np

    w = np.zeros(mlp_num_params(), dtype=np.float32)
    mean = ctypes.c_float()
    sd = ctypes.c_float()
    _check(lib().pm_model_get(_fptr(w), ctypes.byref(mean), ctypes.byref(sd)), "pm_model_get")
    return w, mean.value, sd.value


def model_set(w, mean: float, sd: float):
    w = _f32(w)
    _check(lib().pm_model_set(_fptr(w), mean, sd), "pm_model_set")


def model_predict(lc: int, p: int, plans, context: int = 0):
    import numpy as np

    arr = (Plan * len(plans))(*plans)
    out = np.zeros(len(plans), dtype=np.float64)
    _check(lib().pm_model_predict(lc, p, arr, len(plans), context,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "pm_model_predict")
    return out


def model_save(path: str):
    _check(lib().pm_model_save(path.encode()), "pm_model_save")


def model_load(path: str):
    _check(lib().pm_model_load(path.encode()), "pm_model_load")


def mlp_forward(params, X):
    import numpy as np

    params, X = _f32(params), _f32(X)
    y = np.zeros(X.shape[0], dtype=np.float32)
    _check(lib().pm_mlp_forward(_fptr(params), _fptr(X), X.shape[0], _fptr(y)), "pm_mlp_forward")
    return y


def mlp_loss_grad(params, X, t):
    import numpy as np

    params, X, t = _f32(params), _f32(X), _f32(t)
    g = np.zeros(mlp_num_params(), dtype=np.float32)
    loss = np.zeros(1, dtype=np.float32)
    _check(lib().pm_mlp_loss_grad(_fptr(params), _fptr(X), _fptr(t), X.shape[0], _fptr(loss), _fptr(g)),
           "pm_mlp_loss_grad")
    return float(loss[0]), g


def mlp_adam(params, grads, m, v, step: int, lr: float):
    """One Adam step; returns new (params, m, v)."""
    params, grads, m, v = (_f32(x).copy() for x in (params, grads, m, v))
    _check(lib().pm_mlp_adam(_fptr(params), _fptr(grads), _fptr(m), _fptr(v), step, lr), "pm_mlp_adam")
    return params, m, v


def mlp_train(params, X, t, steps: int, lr: float):
    import numpy as np

    params, X, t = _f32(params).copy(), _f32(X), _f32(t)
    losses = np.zeros(steps, dtype=np.float32)
    _check(lib().pm_mlp_train(_fptr(params), _fptr(X), _fptr(t), X.shape[0], steps, lr, _fptr(losses)),
           "pm_mlp_train")
    return params, losses
