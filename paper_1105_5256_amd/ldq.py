"""ctypes binding of libldq (include/ldq.h): argument marshalling only.

Every computation happens in the HIP library; this module converts Python /
numpy / torch arguments into the C ABI's plain pointers and sizes, raises
``LdqError`` on a non-OK status and wraps handles so they are released.
If the shared library has not been built the import of the functions fails
loudly; there is no fallback.
"""
import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldq.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ldq.h")

LDQ_OK, LDQ_E_INVALID, LDQ_E_NOT_SPD, LDQ_E_NO_CONVERGENCE = 0, 1, 2, 3
LDQ_E_ENCLOSURE, LDQ_E_DEVICE, LDQ_E_NO_MEMORY, LDQ_E_UNSUPPORTED = 4, 5, 6, 7
LDQ_SHIFTED_LAPLACIAN, LDQ_SQUARED_SHIFTED_LAPLACIAN = 1, 2
LDQ_FLAG_DEVICE_PTR = 1
LDQ_FP64, LDQ_MIXED = 0, 1
LDQ_COLOUR_AUTO, LDQ_COLOUR_MODULAR, LDQ_COLOUR_GREEDY, LDQ_COLOUR_USER, LDQ_COLOUR_IDENTITY = 0, 1, 2, 3, 4
LDQ_COLOUR_RADEMACHER = 5
LDQ_LAUNCH_AUTO, LDQ_LAUNCH_GRAPH, LDQ_LAUNCH_DIRECT = 0, 1, 2


class ldq_options(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int),
        ("colouring", ctypes.c_int),
        ("user_colours", ctypes.POINTER(ctypes.c_int32)),
        ("priority", ctypes.POINTER(ctypes.c_int32)),
        ("nshifts", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("grad_tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("lambda_min", ctypes.c_double),
        ("lambda_max", ctypes.c_double),
        ("probe_block", ctypes.c_int),
        ("check_every", ctypes.c_int),
        ("launch_mode", ctypes.c_int),
        ("tile_rows", ctypes.c_int),
        ("lanes", ctypes.c_int),
        ("nrandom", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("consistent_grad", ctypes.c_int),
    ]


class ldq_info(ctypes.Structure):
    _fields_ = [
        ("ncolours", ctypes.c_int32),
        ("iters_max", ctypes.c_int32),
        ("iters_total", ctypes.c_int64),
        ("lambda_min", ctypes.c_double),
        ("lambda_max", ctypes.c_double),
        ("max_rel_residual", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("loop_seconds", ctypes.c_double),
        ("passes", ctypes.c_int64),
        ("probe_passes", ctypes.c_int64),
        ("bytes_model", ctypes.c_double),
        ("enclosure_violations", ctypes.c_int32),
        ("lanes", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32),
        ("std_error", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class LdqError(RuntimeError):
    def __init__(self, status, func, detail):
        self.status = status
        super().__init__(f"{func}: {_status_name(status)}: {detail}")


_P = ctypes.c_void_p
_SIGNATURES = {
    "ldq_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ldq_last_error": (ctypes.c_char_p, []),
    "ldq_create": (ctypes.c_int, [ctypes.c_int, _P, ctypes.POINTER(_P)]),
    "ldq_destroy": (None, [_P]),
    "ldq_set_stream": (ctypes.c_int, [_P, _P]),
    "ldq_op_lattice": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                      ctypes.c_double, _P, ctypes.c_double, ctypes.c_uint, ctypes.POINTER(_P)]),
    "ldq_op_csr": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P, _P, ctypes.c_uint,
                                  ctypes.POINTER(_P)]),
    "ldq_op_diag": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_uint, ctypes.POINTER(_P)]),
    "ldq_op_add_obs": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P, ctypes.c_double]),
    "ldq_op_obs_gram": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P, ctypes.POINTER(_P)]),
    "ldq_op_size": (ctypes.c_int64, [_P]),
    "ldq_op_destroy": (None, [_P]),
    "ldq_options_default": (None, [ctypes.POINTER(ldq_options)]),
    "ldq_colouring": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _P,
                                     ctypes.POINTER(ctypes.c_int32)]),
    "ldq_spectrum_bounds": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]),
    "ldq_shifts": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, _P]),
    "ldq_logdet": (ctypes.c_int, [_P, _P, ctypes.POINTER(ldq_options), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ldq_info)]),
    "ldq_logdet_grad": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, ctypes.POINTER(ldq_options),
                                       ctypes.POINTER(ctypes.c_double), _P, ctypes.POINTER(ldq_info)]),
    "ldq_probe_terms": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int)]),
    "ldq_logm_apply": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P]),
    "ldq_solve": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P]),
    "ldq_logdet_batched": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int, _P, ctypes.POINTER(ldq_options),
                                          _P, _P, _P]),
}

_lib = None


def header_functions():
    """Names of the functions declared in include/ldq.h."""
    with open(HEADER_PATH) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\**\s*(ldq_\w+)\s*\(", text, re.M)))


def load():
    """Load libldq.so (built in-tree by build_lib.py); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _status_name(status):
    return load().ldq_status_string(status).decode()


def _check(status, func):
    if status != LDQ_OK:
        raise LdqError(status, func, load().ldq_last_error().decode())


def _ptr(a):
    """Data pointer of a numpy array or a torch tensor (host or device)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _is_device(a):
    return hasattr(a, "is_cuda") and a.is_cuda


# ------------------------------------------------------------------ wrappers
def ldq_create(device=0, stream=None):
    """Create a context on `device`; `stream` is a raw hipStream_t (int) or None."""
    h = ctypes.c_void_p()
    _check(load().ldq_create(device, ctypes.c_void_p(stream) if stream else None, ctypes.byref(h)), "ldq_create")
    return h


def ldq_destroy(ctx):
    load().ldq_destroy(ctx)


def ldq_set_stream(ctx, stream):
    _check(load().ldq_set_stream(ctx, ctypes.c_void_p(stream) if stream else None), "ldq_set_stream")


def ldq_op_lattice(ctx, shape, kind, kappa2=0.0, kappa2_field=None, scale=1.0):
    shp = (ctypes.c_int64 * len(shape))(*[int(m) for m in shape])
    flags = LDQ_FLAG_DEVICE_PTR if _is_device(kappa2_field) else 0
    if kappa2_field is not None and not _is_device(kappa2_field):
        kappa2_field = np.ascontiguousarray(kappa2_field, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(load().ldq_op_lattice(ctx, len(shape), shp, kind, float(kappa2), _ptr(kappa2_field), float(scale),
                                 flags, ctypes.byref(h)), "ldq_op_lattice")
    return h


def ldq_op_csr(ctx, n, rowptr, colind, val):
    dev = _is_device(val)
    if not dev:
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(load().ldq_op_csr(ctx, int(n), int(len(colind)), _ptr(rowptr), _ptr(colind), _ptr(val),
                             LDQ_FLAG_DEVICE_PTR if dev else 0, ctypes.byref(h)), "ldq_op_csr")
    return h


def ldq_op_diag(ctx, d):
    dev = _is_device(d)
    if not dev:
        d = np.ascontiguousarray(d, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(load().ldq_op_diag(ctx, int(len(d)), _ptr(d), LDQ_FLAG_DEVICE_PTR if dev else 0, ctypes.byref(h)),
           "ldq_op_diag")
    return h


def ldq_op_add_obs(op, corner, weight, tau):
    corner = np.ascontiguousarray(corner, dtype=np.int32)
    weight = np.ascontiguousarray(weight, dtype=np.float64)
    _check(load().ldq_op_add_obs(op, int(corner.shape[0]), _ptr(corner), _ptr(weight), float(tau)),
           "ldq_op_add_obs")


def ldq_op_obs_gram(ctx, like, corner, weight):
    corner = np.ascontiguousarray(corner, dtype=np.int32)
    weight = np.ascontiguousarray(weight, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(load().ldq_op_obs_gram(ctx, like, int(corner.shape[0]), _ptr(corner), _ptr(weight), ctypes.byref(h)),
           "ldq_op_obs_gram")
    return h


def ldq_op_size(op):
    return int(load().ldq_op_size(op))


def ldq_op_destroy(op):
    load().ldq_op_destroy(op)


def ldq_options_default(**overrides):
    """An ldq_options with the library defaults, then `overrides` applied.
    user_colours / priority may be numpy int32 arrays (kept alive on the struct)."""
    o = ldq_options()
    load().ldq_options_default(ctypes.byref(o))
    keep = []
    for key, val in overrides.items():
        if key in ("user_colours", "priority"):
            if val is None:
                setattr(o, key, None)
                continue
            arr = np.ascontiguousarray(val, dtype=np.int32)
            keep.append(arr)
            setattr(o, key, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        else:
            setattr(o, key, val)
    o._keep = keep
    return o


def ldq_colouring(ctx, Q, k, method, priority=None):
    n = ldq_op_size(Q)
    out = np.empty(n, dtype=np.int32)
    nc = ctypes.c_int32()
    prio = None if priority is None else np.ascontiguousarray(priority, dtype=np.int32)
    _check(load().ldq_colouring(ctx, Q, int(k), int(method), _ptr(prio), _ptr(out), ctypes.byref(nc)),
           "ldq_colouring")
    return out, int(nc.value)


def ldq_spectrum_bounds(ctx, Q):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(load().ldq_spectrum_bounds(ctx, Q, ctypes.byref(lo), ctypes.byref(hi)), "ldq_spectrum_bounds")
    return lo.value, hi.value


def ldq_shifts(ctx, lmin, lmax, nshifts):
    s = np.empty(2 * nshifts)
    c = np.empty(2 * nshifts)
    _check(load().ldq_shifts(ctx, float(lmin), float(lmax), int(nshifts), _ptr(s), _ptr(c)), "ldq_shifts")
    return s[0::2] + 1j * s[1::2], c[0::2] + 1j * c[1::2]


def ldq_logdet(ctx, Q, opts=None):
    """Returns (logdet, info dict)."""
    opts = opts if opts is not None else ldq_options_default()
    val = ctypes.c_double()
    info = ldq_info()
    _check(load().ldq_logdet(ctx, Q, ctypes.byref(opts), ctypes.byref(val), ctypes.byref(info)), "ldq_logdet")
    return val.value, info.as_dict()


def ldq_logdet_grad(ctx, Q, dQ, opts=None):
    """Returns (logdet, grad (numpy), info dict) for derivative operators dQ (list of handles)."""
    opts = opts if opts is not None else ldq_options_default()
    arr = (ctypes.c_void_p * max(1, len(dQ)))(*[d.value for d in dQ])
    val = ctypes.c_double()
    grad = np.zeros(max(1, len(dQ)))
    info = ldq_info()
    _check(load().ldq_logdet_grad(ctx, Q, len(dQ), ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(opts),
                                  ctypes.byref(val), _ptr(grad), ctypes.byref(info)), "ldq_logdet_grad")
    return val.value, grad[:len(dQ)], info.as_dict()


def ldq_probe_terms(ctx):
    """Per-probe terms of the last call: array (nprobes, 1 + nparams)."""
    cnt, npar = ctypes.c_int64(), ctypes.c_int()
    _check(load().ldq_probe_terms(ctx, None, 0, ctypes.byref(cnt), ctypes.byref(npar)), "ldq_probe_terms")
    out = np.empty(cnt.value * (1 + npar.value))
    _check(load().ldq_probe_terms(ctx, _ptr(out), len(out), ctypes.byref(cnt), ctypes.byref(npar)),
           "ldq_probe_terms")
    return out.reshape(cnt.value, 1 + npar.value)


def ldq_logm_apply(ctx, Q, V, opts=None):
    """f_N(Q) V for the rows of V (a torch float64 CUDA tensor, nvec x n, contiguous):
    returns (Y of the same shape on the same device, info dict of the first solve)."""
    import torch
    if V.dim() == 1:
        V = V[None]
    if V.dtype != torch.float64 or not V.is_cuda or not V.is_contiguous():
        raise ValueError("V must be a contiguous float64 CUDA tensor")
    Y = torch.empty_like(V)
    opts = opts if opts is not None else ldq_options_default()
    info = ldq_info()
    _check(load().ldq_logm_apply(ctx, Q, V.shape[0], ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                 ctypes.byref(opts), ctypes.byref(info)), "ldq_logm_apply")
    return Y, info.as_dict()


def ldq_solve(ctx, Q, B, opts=None):
    """Q^{-1} B for the rows of B (a torch float64 CUDA tensor, nvec x n, contiguous):
    returns (X of the same shape on the same device, info dict of the first solve)."""
    import torch
    if B.dim() == 1:
        B = B[None]
    if B.dtype != torch.float64 or not B.is_cuda or not B.is_contiguous():
        raise ValueError("B must be a contiguous float64 CUDA tensor")
    X = torch.empty_like(B)
    opts = opts if opts is not None else ldq_options_default()
    info = ldq_info()
    _check(load().ldq_solve(ctx, Q, B.shape[0], ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                            ctypes.byref(opts), ctypes.byref(info)), "ldq_solve")
    return X, info.as_dict()


def ldq_logdet_batched(ctx, Qs, dQs=None, opts=None):
    """Qs: list of operator handles; dQs: list (per field) of lists of handles or None.
    Returns (logdet (nfields,), grad (nfields, nparams), list of info dicts)."""
    opts = opts if opts is not None else ldq_options_default()
    nf = len(Qs)
    npar = len(dQs[0]) if dQs else 0
    qarr = (ctypes.c_void_p * max(1, nf))(*[q.value for q in Qs])
    darr = (ctypes.c_void_p * max(1, nf * npar))(*[d.value for row in (dQs or []) for d in row])
    logdet = np.zeros(max(1, nf))
    grad = np.zeros(max(1, nf * npar))
    infos = (ldq_info * max(1, nf))()
    _check(load().ldq_logdet_batched(ctx, nf, ctypes.cast(qarr, ctypes.c_void_p), npar,
                                     ctypes.cast(darr, ctypes.c_void_p) if npar else None, ctypes.byref(opts),
                                     _ptr(logdet), _ptr(grad) if npar else None,
                                     ctypes.cast(infos, ctypes.c_void_p)), "ldq_logdet_batched")
    return logdet[:nf], grad[:nf * npar].reshape(nf, npar), [infos[i].as_dict() for i in range(nf)]


# --------------------------------------------------------------- conveniences
class Context:
    """Owns an ldq context bound to torch's current stream on `device`."""

    def __init__(self, device=0, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        self.handle = ldq_create(device, stream)
        self._ops = []

    def op(self, handle):
        self._ops.append(handle)
        return handle

    def close(self):
        for h in self._ops:
            ldq_op_destroy(h)
        self._ops = []
        if self.handle is not None:
            ldq_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
