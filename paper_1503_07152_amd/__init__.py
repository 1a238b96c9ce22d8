"""Python binding of libhbspeel (randomized HODLR / HBS compression on MI355X).

Argument marshalling only: every step of compression and apply runs in the
HIP kernels of ``libhbspeel.so`` behind the C ABI of ``include/hbspeel.h``.
PyTorch supplies device memory and the current stream.  Matrices cross the
boundary column-major; helpers here make column-major ("Fortran") tensors.

If the shared library is missing this module raises at import: there is no
fallback path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np
import torch

__all__ = [
    "HM_F64", "HM_F32", "HM_BF16", "lib", "HMError", "fortran", "to_fortran",
    "Options", "KernelOperator", "DenseOperator", "HBSOperator", "HBSProductOperator",
    "CallbackOperator", "Frontal", "FrontalOperator", "frontal_create",
    "HBS", "HODLR", "hm_gauss", "hm_operator_apply", "hbs_compress", "hbs_compress_adaptive",
    "hodlr_compress", "hbs_compress_batched", "autotune", "hbs_factor", "HBSFactor",
    "hss_apply", "hss_apply_adjoint", "hss_apply_noalloc", "hss_apply_backward", "hodlr_apply",
    "hm_hbs_from_generators", "hbs_from_tensors", "HBSApply", "hbs_apply", "use_torch_allocator",
]

HM_OK, HM_WARN_RANK_SATURATED = 0, 1
HM_F64, HM_F32, HM_BF16 = 0, 1, 2
HM_OP_CALLBACK, HM_OP_KERNEL, HM_OP_DENSE, HM_OP_HBS, HM_OP_HBS_PRODUCT = 0, 1, 2, 3, 4
HM_OP_FRONTAL = 5
HM_KERNEL_LOG, HM_KERNEL_NEAR = 0, 1
HM_FLAG_ORTHONORMAL, HM_FLAG_PERSISTENT_ID, HM_FLAG_LOW_MEMORY_PLAN = 1, 2, 4
HM_MAX_SAMPLES = 48

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhbspeel.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(
        f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
        " (there is no CPU fallback)")
lib = C.CDLL(_LIB_PATH)

MATVEC = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                     C.c_void_p, C.c_int64, C.c_int32, C.c_void_p)


class _Operator(C.Structure):
    _fields_ = [("kind", C.c_int32), ("sample_dtype", C.c_int32), ("fn", MATVEC),
                ("user", C.c_void_p), ("points", C.c_void_p), ("kernel_id", C.c_int32),
                ("kparam", C.c_double), ("dense", C.c_void_p), ("ld", C.c_int64),
                ("hbs", C.c_void_p), ("hbs2", C.c_void_p), ("frontal", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("n", C.c_int64), ("leaf_size", C.c_int64), ("rank", C.c_int32),
                ("oversample", C.c_int32), ("tol", C.c_double), ("seed", C.c_uint64),
                ("flags", C.c_int32), ("store_dtype", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("leaf_size", C.c_int64), ("levels", C.c_int32),
                ("rank_pad", C.c_int32), ("max_rank", C.c_int32), ("min_rank", C.c_int32),
                ("is_id", C.c_int32), ("dtype", C.c_int32), ("storage_reals", C.c_int64),
                ("sample_columns", C.c_int64), ("operator_calls", C.c_int32),
                ("saturated", C.c_int32), ("t_compress_ms", C.c_double),
                ("t_operator_ms", C.c_double), ("jacobi_sweeps", C.c_int32),
                ("adapt_rounds", C.c_int32), ("err_estimate", C.c_double)]


class _Views(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("rank_pad", C.c_int32), ("levels", C.c_int32),
                ("nmax", C.c_int32), ("n", C.c_int64), ("nodes", C.c_int64),
                ("U", C.c_void_p), ("V", C.c_void_p), ("Ut", C.c_void_p), ("Vt", C.c_void_p),
                ("B", C.c_void_p), ("D", C.c_void_p)]


class _Tune(C.Structure):
    _fields_ = [("gfirst", C.c_int32), ("ride", C.c_int32), ("ksplit", C.c_int32),
                ("candidates", C.c_int32), ("t_default_ms", C.c_double),
                ("t_best_ms", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

_P, _I64, _I32 = C.c_void_p, C.c_int64, C.c_int32
_SIGS = {
    "hm_last_error": (C.c_char_p, []),
    "hm_version": (C.c_char_p, []),
    "hm_gauss": (C.c_int, [C.c_uint64, _I32, _I32, _I64, _I64, _I32, _P, _I64, _P]),
    "hm_operator_apply": (C.c_int, [C.POINTER(_Operator), _I64, _I32, _I64, _P, _I64, _P, _I64,
                                    _P]),
    "hbs_compress": (C.c_int, [C.POINTER(_Options), C.POINTER(_Operator), _P, C.POINTER(_P)]),
    "hbs_compress_adaptive": (C.c_int, [C.POINTER(_Options), C.POINTER(_Operator), C.c_double,
                                        _P, C.POINTER(_P)]),
    "hodlr_compress": (C.c_int, [C.POINTER(_Options), C.POINTER(_Operator), _P, C.POINTER(_P)]),
    "hbs_compress_batched": (C.c_int, [_I32, C.POINTER(_Options), C.POINTER(_Operator), _P,
                                       C.POINTER(_P)]),
    "hss_apply": (C.c_int, [_P, _I64, _P, _I64, _P, _I64, _P]),
    "hss_apply_adjoint": (C.c_int, [_P, _I64, _P, _I64, _P, _I64, _P]),
    "hss_apply_noalloc": (C.c_int, [_P, _I64, _P, _I64, _P, _I64, _P]),
    "hss_apply_backward": (C.c_int, [_P, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P, _P, _P, _P,
                                     _P, _P]),
    "hodlr_apply": (C.c_int, [_P, _I32, _I64, _P, _I64, _P, _I64, _P]),
    "hm_hbs_from_generators": (C.c_int, [_I64, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P, _P,
                                         C.POINTER(_P)]),
    "hm_hbs_convert": (C.c_int, [_P, _I32, _P, C.POINTER(_P)]),
    "hm_hbs_info": (C.c_int, [_P, C.POINTER(_Info)]),
    "hm_hbs_generators": (C.c_int, [_P, C.POINTER(_Views)]),
    "hm_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, _P]),
    "hm_release_cached_memory": (C.c_int, []),
    "hm_autotune": (C.c_int, [C.POINTER(_Options), C.POINTER(_Operator), C.c_int32, _P,
                              C.POINTER(_Tune)]),
    "hm_hodlr_info": (C.c_int, [_P, C.POINTER(_Info)]),
    "hm_hbs_export": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "hm_hodlr_export": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "hm_hbs_free": (None, [_P]),
    "hbs_factor": (C.c_int, [_P, _P, C.POINTER(_P)]),
    "hbs_solve": (C.c_int, [_P, _I64, _P, _I64, _P, _I64, _P]),
    "hm_hbs_factor_free": (None, [_P]),
    "hm_hodlr_free": (None, [_P]),
    "hm_frontal_create": (C.c_int, [_I64, _I32, _P, _P, _P, C.POINTER(_P)]),
    "hm_frontal_apply": (C.c_int, [_P, _I64, _P, _I64, _P, _I64, _P]),
    "hm_frontal_free": (None, [_P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class HMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hbspeel error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc < 0:
        raise HMError(rc, lib.hm_last_error().decode())
    return rc


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def fortran(rows, cols, dtype=torch.float64, device="cuda"):
    """An uninitialised rows x cols tensor in column-major layout (ld = rows)."""
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def to_fortran(x, dtype=None, device="cuda"):
    """Column-major device copy of a 2-D array (numpy or torch); 1-D becomes n x 1."""
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    if x.dim() == 1:
        x = x[:, None]
    dtype = dtype or x.dtype
    out = fortran(x.shape[0], x.shape[1], dtype, device)
    out.copy_(x)
    return out


def _device_fortran(x, dtype):
    """``x`` itself when it already is a column-major device tensor of
    ``dtype``, else a column-major device copy."""
    if isinstance(x, torch.Tensor) and x.dim() == 2 and x.stride(0) == 1 and x.dtype == dtype \
            and x.is_cuda:
        return x
    return to_fortran(x, dtype)


def _ld(t):
    """Leading dimension of a column-major 2-D tensor."""
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError("expected a column-major 2-D tensor (see fortran())")
    return max(t.stride(1), t.shape[0])


class Options:
    def __init__(self, n, leaf_size, rank, oversample=10, tol=0.0, seed=0, orthonormal=False,
                 store_dtype=HM_F64, persistent_id=False, low_memory_plan=False):
        flags = (HM_FLAG_ORTHONORMAL if orthonormal else 0) | \
            (HM_FLAG_PERSISTENT_ID if persistent_id else 0) | \
            (HM_FLAG_LOW_MEMORY_PLAN if low_memory_plan else 0)
        self.c = _Options(n, leaf_size, rank, oversample, tol, seed, flags, store_dtype)


class KernelOperator:
    """Built-in kernel matrix on 2-D points: ``'log'`` (log|x-y|, 1 on the
    diagonal) or ``'near'`` (1/(|x-y| + delta)); sampled in ``sample_dtype``."""

    def __init__(self, points, kernel="near", kparam=1e-3, sample_dtype=HM_F64):
        pts = points if isinstance(points, torch.Tensor) else torch.from_numpy(np.asarray(points))
        self.points = pts.to(device="cuda", dtype=torch.float64).contiguous()
        self.c = _Operator()
        self.c.kind = HM_OP_KERNEL
        self.c.sample_dtype = sample_dtype
        self.c.points = self.points.data_ptr()
        self.c.kernel_id = HM_KERNEL_LOG if kernel == "log" else HM_KERNEL_NEAR
        self.c.kparam = kparam


class DenseOperator:
    def __init__(self, A):
        self.A = to_fortran(A, torch.float64)
        self.c = _Operator()
        self.c.kind = HM_OP_DENSE
        self.c.dense = self.A.data_ptr()
        self.c.ld = _ld(self.A)


class HBSOperator:
    def __init__(self, h):
        self.h = h
        self.c = _Operator()
        self.c.kind = HM_OP_HBS
        self.c.hbs = h.handle


class HBSProductOperator:
    """The product ``h1 @ h2`` of two FP64 HBS handles as a black box (Sec. 5.2:
    recompressing a product of compressed operators); each factor is applied
    in O(N k)."""

    def __init__(self, h1, h2):
        self.h1, self.h2 = h1, h2
        self.c = _Operator()
        self.c.kind = HM_OP_HBS_PRODUCT
        self.c.hbs = h1.handle
        self.c.hbs2 = h2.handle


class _DevArray:
    """Raw device buffer seen by torch through __cuda_array_interface__."""

    def __init__(self, ptr, rows, cols, ld, typestr="<f8"):
        self.__cuda_array_interface__ = {
            "shape": (cols, ld), "typestr": typestr, "data": (ptr, False), "version": 2,
            "strides": None}


# element types of the callback's X and Y per sample dtype (BF16 bit
# patterns travel as int16 and are viewed as bfloat16)
_CB_TYPES = {HM_F64: ("<f8", "<f8", None), HM_F32: ("<f4", "<f4", None),
             HM_BF16: ("<i2", "<f4", torch.bfloat16)}


class CallbackOperator:
    """User black box: ``fn(adjoint: bool, X, Y)`` with X, Y n x c column-major
    device tensors that alias library buffers; must write ``Y = A X`` (or
    ``A^* X``) on the current stream and return None (or 0).  ``sample_dtype``
    sets their types: HM_F64 (float64 / float64), HM_F32 (float32 / float32),
    HM_BF16 (X bfloat16, Y float32)."""

    def __init__(self, fn, sample_dtype=HM_F64):
        self.fn = fn

        def tramp(user, adjoint, n, ncols, X, ldx, Y, ldy, dtype, stream):
            try:
                tx, ty, view = _CB_TYPES[dtype]
                Xt = torch.as_tensor(_DevArray(X, n, ncols, ldx, tx), device="cuda").t()[:n]
                if view is not None:
                    Xt = Xt.view(view)
                Yt = torch.as_tensor(_DevArray(Y, n, ncols, ldy, ty), device="cuda").t()[:n]
                rc = self.fn(bool(adjoint), Xt, Yt)
                return int(rc or 0)
            except Exception:  # noqa: BLE001 -- a failing callback aborts the compression
                return 1

        self._tramp = MATVEC(tramp)
        self.c = _Operator()
        self.c.kind = HM_OP_CALLBACK
        self.c.sample_dtype = sample_dtype
        self.c.fn = self._tramp


def _info(fn, handle):
    inf = _Info()
    _check(fn(handle, C.byref(inf)))
    return {k: getattr(inf, k) for k, _ in _Info._fields_}


class _DeviceArray:
    """A device array of a handle's memory, handed to torch through the CUDA
    array interface (zero-copy); holds the handle so the memory outlives the
    tensor."""

    def __init__(self, owner, ptr, shape, strides, dtype):
        self.owner = owner
        typestr = "<f8" if dtype == torch.float64 else "<f4"
        es = 8 if dtype == torch.float64 else 4
        self.__cuda_array_interface__ = {
            "shape": tuple(shape), "typestr": typestr, "data": (ptr, False), "version": 2,
            "strides": tuple(st * es for st in strides)}


def _alias(owner, ptr, shape, strides, dtype):
    return torch.as_tensor(_DeviceArray(owner, ptr, shape, strides, dtype), device="cuda")


_ALLOC_STATE = {"hooks": None, "exiting": False}


def use_torch_allocator(enable=True):
    """Route every device allocation of the library (handle memory, per-call
    scratch) through torch's caching allocator (``hm_set_allocator``), or back
    to hipMalloc / hipFree.  Memory is allocated and returned on the stream
    of the call that needs it; buffers keep the allocator that made them."""
    if not enable:
        _check(lib.hm_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return

    # the callbacks bind what they use: module globals are cleared during
    # interpreter shutdown
    def alloc(ctx, nbytes, stream, _alloc=torch.cuda.caching_allocator_alloc):
        try:
            return _alloc(int(nbytes), stream=int(stream or 0))
        except Exception:   # reported to the library as an allocation failure
            return None

    def free(ctx, ptr, stream, _st=_ALLOC_STATE, _delete=torch.cuda.caching_allocator_delete):
        if _st["exiting"]:
            return   # torch may already be torn down; the process is ending
        try:
            _delete(int(ptr))
        except Exception:
            pass

    hooks = (ALLOC_FN(alloc), FREE_FN(free))
    _check(lib.hm_set_allocator(hooks[0], hooks[1], None))
    # every buffer made through these hooks calls them when it is freed, so
    # the thunks must outlive every buffer: one extra reference that is
    # never dropped keeps them alive until the process ends, whatever order
    # shutdown clears modules in
    C.pythonapi.Py_IncRef(C.py_object(hooks))
    _ALLOC_STATE["hooks"] = hooks


# Handles still alive when the interpreter exits are freed by an exit handler,
# while torch (and its caching allocator, if it backs the library) is whole;
# this handler is registered after torch's and so runs before them.
_LIVE = weakref.WeakSet()


def _release_at_exit():
    for obj in list(_LIVE):
        obj._release()
    _ALLOC_STATE["exiting"] = True


atexit.register(_release_at_exit)


class HBS:
    """An HBS handle owned by the library."""

    def __init__(self, handle, status=HM_OK):
        self.handle = handle
        self.status = status
        _LIVE.add(self)

    # bound at class creation: module globals may already be cleared when
    # the last handles are collected at interpreter exit
    _free = lib.hm_hbs_free

    def _release(self):
        if getattr(self, "handle", None):
            type(self)._free(self.handle)
            self.handle = None

    __del__ = _release

    def info(self):
        return _info(lib.hm_hbs_info, self.handle)

    def export(self, stream=None):
        """Generators in the flat layout (torch tensors on the device, heap-
        indexed blocks) plus host ranks and skeletons."""
        inf = self.info()
        n, R, L = inf["n"], inf["rank_pad"], inf["levels"]
        nn = 2 ** (L + 1)
        dt = torch.float64 if inf["dtype"] == HM_F64 else torch.float32
        leafmax = self._nmax(n, inf["leaf_size"], L)
        out = dict(U=fortran(n, R, dt), V=fortran(n, R, dt),
                   Ut=torch.zeros((nn, R, 2 * R), dtype=dt, device="cuda"),
                   Vt=torch.zeros((nn, R, 2 * R), dtype=dt, device="cuda"),
                   B=torch.zeros((nn, R, R), dtype=dt, device="cuda"),
                   D=fortran(n, leafmax, dt))
        ru = np.zeros(nn, dtype=np.int32)
        rv = np.zeros(nn, dtype=np.int32)
        si = np.full(nn * R, -1, dtype=np.int32)
        so = np.full(nn * R, -1, dtype=np.int32)
        ip = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(lib.hm_hbs_export(self.handle, _ptr(out["U"]), _ptr(out["V"]), _ptr(out["Ut"]),
                                 _ptr(out["Vt"]), _ptr(out["B"]), _ptr(out["D"]), ip(ru), ip(rv),
                                 ip(si), ip(so), _stream(stream)))
        torch.cuda.synchronize()
        # per-node blocks are column-major: block t viewed as (cols, rows) -> transpose
        out["Ut"] = out["Ut"].transpose(1, 2)
        out["Vt"] = out["Vt"].transpose(1, 2)
        out["B"] = out["B"].transpose(1, 2)
        out.update(rank_u=ru, rank_v=rv, skel_in=si.reshape(nn, R), skel_out=so.reshape(nn, R),
                   n=n, R=R, L=L, leaf=inf["leaf_size"], is_id=inf["is_id"])
        return out

    def generators(self):
        """Zero-copy device views of the handle's generators (``hm_hbs_generators``):
        U, V (n, R); Ut, Vt (nodes, 2R, R) and B (nodes, R, R), node with heap
        number t at index t - 1; D (n, nmax).  Read-only; each tensor keeps the
        handle alive."""
        v = _Views()
        _check(lib.hm_hbs_generators(self.handle, C.byref(v)))
        dt = torch.float64 if v.dtype == HM_F64 else torch.float32
        n, R, nn = v.n, v.rank_pad, v.nodes
        return dict(
            U=_alias(self, v.U, (n, R), (1, n), dt), V=_alias(self, v.V, (n, R), (1, n), dt),
            Ut=_alias(self, v.Ut, (nn, 2 * R, R), (2 * R * R, 1, 2 * R), dt),
            Vt=_alias(self, v.Vt, (nn, 2 * R, R), (2 * R * R, 1, 2 * R), dt),
            B=_alias(self, v.B, (nn, R, R), (R * R, 1, R), dt),
            D=_alias(self, v.D, (n, v.nmax), (1, n), dt),
            n=n, R=R, L=v.levels, nodes=nn)

    def convert(self, dtype, stream=None):
        """Copy with the generators stored in ``dtype`` (HM_F64 / HM_F32)."""
        h = C.c_void_p()
        _check(lib.hm_hbs_convert(self.handle, dtype, _stream(stream), C.byref(h)))
        return HBS(h)

    @staticmethod
    def _nmax(n, leaf, L):
        return -(-n // (2 ** L))

    def apply(self, x, adjoint=False, stream=None):
        return (hss_apply_adjoint if adjoint else hss_apply)(self, x, stream=stream)


class HBSFactor:
    """A factorisation of the inverse of an HBS matrix (``hbs_factor``);
    ``solve(b)`` returns ``A_H^-1 b`` (FP64)."""

    def __init__(self, handle):
        self.handle = handle
        _LIVE.add(self)

    _free = lib.hm_hbs_factor_free

    def _release(self):
        if getattr(self, "handle", None):
            type(self)._free(self.handle)
            self.handle = None

    __del__ = _release

    def solve(self, b, stream=None):
        bf = to_fortran(b, torch.float64)
        x = fortran(bf.shape[0], bf.shape[1])
        _check(lib.hbs_solve(self.handle, bf.shape[1], _ptr(bf), _ld(bf), _ptr(x), _ld(x),
                             _stream(stream)))
        return x


def hbs_factor(h, stream=None) -> HBSFactor:
    f = C.c_void_p()
    _check(lib.hbs_factor(h.handle, _stream(stream), C.byref(f)))
    return HBSFactor(f)


class Frontal:
    """The frontal matrix of nested dissection (Sec. 5.4) of a conduction grid
    with bar conductivities ``ch`` (height x (width-1)) and ``cv``
    ((height-1) x width), factored on the device (``hm_frontal_create``);
    ``apply(x)`` returns ``A x`` (FP64)."""

    def __init__(self, handle, height):
        self.handle = handle
        self.n = height
        _LIVE.add(self)

    _free = lib.hm_frontal_free

    def _release(self):
        if getattr(self, "handle", None):
            type(self)._free(self.handle)
            self.handle = None

    __del__ = _release

    def apply(self, x, stream=None):
        xf = to_fortran(x, torch.float64)
        y = fortran(xf.shape[0], xf.shape[1])
        _check(lib.hm_frontal_apply(self.handle, xf.shape[1], _ptr(xf), _ld(xf), _ptr(y), _ld(y),
                                    _stream(stream)))
        return y


def frontal_create(ch, cv, stream=None) -> Frontal:
    ch = torch.as_tensor(ch, dtype=torch.float64).to("cuda").contiguous()
    height, wm1 = ch.shape
    cvp = None
    if height > 1:
        cv = torch.as_tensor(cv, dtype=torch.float64).to("cuda").contiguous()
        if tuple(cv.shape) != (height - 1, wm1 + 1):
            raise ValueError(f"cv has shape {tuple(cv.shape)}, expected {(height - 1, wm1 + 1)}")
        cvp = cv.data_ptr()
    f = C.c_void_p()
    _check(lib.hm_frontal_create(height, wm1 + 1, ch.data_ptr(), cvp, _stream(stream),
                                 C.byref(f)))
    return Frontal(f, height)


class FrontalOperator:
    """A ``Frontal`` handle as the black box of a compression (symmetric)."""

    def __init__(self, f):
        self.f = f
        self.c = _Operator()
        self.c.kind = HM_OP_FRONTAL
        self.c.frontal = f.handle


class HODLR:
    def __init__(self, handle, status=HM_OK):
        self.handle = handle
        self.status = status
        _LIVE.add(self)

    # bound at class creation: module globals may already be cleared when
    # the last handles are collected at interpreter exit
    _free = lib.hm_hodlr_free

    def _release(self):
        if getattr(self, "handle", None):
            type(self)._free(self.handle)
            self.handle = None

    __del__ = _release

    def info(self):
        return _info(lib.hm_hodlr_info, self.handle)

    def apply(self, x, adjoint=False, stream=None):
        return hodlr_apply(self, x, adjoint=adjoint, stream=stream)

    def export(self, stream=None):
        inf = self.info()
        n, R, L = inf["n"], inf["rank_pad"], inf["levels"]
        nn = 2 ** (L + 1)
        U = torch.zeros((max(L, 1), R, n), dtype=torch.float64, device="cuda")
        V = torch.zeros_like(U)
        s = torch.zeros((nn, R), dtype=torch.float64, device="cuda")
        D = fortran(n, HBS._nmax(n, inf["leaf_size"], L))
        rk = np.zeros(nn, dtype=np.int32)
        _check(lib.hm_hodlr_export(self.handle, _ptr(U), _ptr(V), _ptr(s), _ptr(D),
                                   rk.ctypes.data_as(C.c_void_p), _stream(stream)))
        torch.cuda.synchronize()
        return dict(U=U.transpose(1, 2), V=V.transpose(1, 2), s=s, D=D, rank=rk, n=n, R=R, L=L)


def hm_gauss(seed, level, phase, row0, nrows, ncols, out=None, stream=None):
    """Rows row0.. of the counter-based Gaussian stream (n x ncols, column-major)."""
    if out is None:
        out = fortran(nrows, ncols)
    _check(lib.hm_gauss(seed, level, phase, row0, nrows, ncols, _ptr(out), _ld(out),
                        _stream(stream)))
    return out


def hm_operator_apply(op, x, adjoint=False, stream=None):
    """Y = A X (or A^* X) through a built-in or callback operator, enqueued on
    `stream` (torch's current stream by default) without waiting for it."""
    xf = to_fortran(x, torch.float64)
    y = fortran(xf.shape[0], xf.shape[1])
    if stream is not None:
        # the temporaries belong to the current stream; keep them until the
        # work on `stream` is done
        xf.record_stream(stream)
        y.record_stream(stream)
    _check(lib.hm_operator_apply(C.byref(op.c), xf.shape[0], 1 if adjoint else 0, xf.shape[1],
                                 _ptr(xf), _ld(xf), _ptr(y), _ld(y), _stream(stream)))
    return y


def hbs_compress(opts: Options, op, stream=None) -> HBS:
    h = C.c_void_p()
    rc = _check(lib.hbs_compress(C.byref(opts.c), C.byref(op.c), _stream(stream), C.byref(h)))
    return HBS(h, rc)


def hbs_compress_adaptive(opts: Options, op, e_target, stream=None) -> HBS:
    """Adaptive sampling: doubles the rank cap (from opts' rank) while a node
    saturates or the posterior estimate E exceeds ``e_target``."""
    h = C.c_void_p()
    rc = _check(lib.hbs_compress_adaptive(C.byref(opts.c), C.byref(op.c), e_target,
                                          _stream(stream), C.byref(h)))
    return HBS(h, rc)


def autotune(opts: Options, op, reps=2, stream=None):
    """Pick the fastest compression schedule for this workload shape (kept for
    later ``hbs_compress`` calls of the shape); returns the choice and times."""
    t = _Tune()
    _check(lib.hm_autotune(C.byref(opts.c), C.byref(op.c), reps, _stream(stream), C.byref(t)))
    return {k: getattr(t, k) for k, _ in _Tune._fields_}


def hodlr_compress(opts: Options, op, stream=None) -> HODLR:
    h = C.c_void_p()
    rc = _check(lib.hodlr_compress(C.byref(opts.c), C.byref(op.c), _stream(stream), C.byref(h)))
    return HODLR(h, rc)


def hbs_compress_batched(opts_list, ops_list, stream=None):
    cnt = len(opts_list)
    O = (_Options * cnt)(*[o.c for o in opts_list])
    P = (_Operator * cnt)(*[o.c for o in ops_list])
    H = (C.c_void_p * cnt)()
    rc = _check(lib.hbs_compress_batched(cnt, O, P, _stream(stream), H))
    return [HBS(C.c_void_p(H[i]), rc) for i in range(cnt)]


def _apply(fn, h, x, stream):
    dt = torch.float64 if h.info()["dtype"] == HM_F64 else torch.float32
    xf = _device_fortran(x, dt)
    y = fortran(xf.shape[0], xf.shape[1], dt)
    _check(fn(h.handle, xf.shape[1], _ptr(xf), _ld(xf), _ptr(y), _ld(y), _stream(stream)))
    return y


def hss_apply(h: HBS, x, stream=None):
    return _apply(lib.hss_apply, h, x, stream)


def hss_apply_adjoint(h: HBS, x, stream=None):
    return _apply(lib.hss_apply_adjoint, h, x, stream)


def hss_apply_noalloc(h: HBS, x, out, stream=None):
    """``out = A_H x`` without any device allocation by the library (its
    scratch is a fixed per-GPU array; overlapping calls on one GPU race).
    ``x`` and ``out``: column-major device tensors of the handle's dtype."""
    _check(lib.hss_apply_noalloc(h.handle, x.shape[1], _ptr(x), _ld(x), _ptr(out), _ld(out),
                                 _stream(stream)))
    return out


def hss_apply_backward(h: HBS, x, gy, want_generators=True, stream=None):
    """gx = A_H^* gy and the generator gradients of <gy, A_H x> (flat layout)."""
    inf = h.info()
    dt = torch.float64 if inf["dtype"] == HM_F64 else torch.float32
    n, R, L = inf["n"], inf["rank_pad"], inf["levels"]
    nn = 2 ** (L + 1)
    xf = _device_fortran(x, dt)
    gyf = _device_fortran(gy, dt)
    gx = fortran(n, xf.shape[1], dt)
    g = None
    if want_generators:
        # the library writes every entry (zeroing the blocks no node owns)
        g = dict(U=fortran(n, R, dt), V=fortran(n, R, dt),
                 Ut=torch.empty((nn, R, 2 * R), dtype=dt, device="cuda"),
                 Vt=torch.empty((nn, R, 2 * R), dtype=dt, device="cuda"),
                 B=torch.empty((nn, R, R), dtype=dt, device="cuda"),
                 D=fortran(n, HBS._nmax(n, inf["leaf_size"], L), dt))
    gp = (lambda k: _ptr(g[k]) if g else None)
    _check(lib.hss_apply_backward(h.handle, xf.shape[1], _ptr(xf), _ld(xf), _ptr(gyf), _ld(gyf),
                                  _ptr(gx), _ld(gx), gp("U"), gp("V"), gp("Ut"), gp("Vt"),
                                  gp("B"), gp("D"), _stream(stream)))
    if g:
        for k in ("Ut", "Vt", "B"):
            g[k] = g[k].transpose(1, 2)
    return gx, g


def hodlr_apply(h: HODLR, x, adjoint=False, stream=None):
    xf = to_fortran(x, torch.float64)
    y = fortran(xf.shape[0], xf.shape[1])
    _check(lib.hodlr_apply(h.handle, 1 if adjoint else 0, xf.shape[1], _ptr(xf), _ld(xf), _ptr(y),
                           _ld(y), _stream(stream)))
    return y


def hm_hbs_from_generators(g: dict, dtype=HM_F64, stream=None) -> HBS:
    """HBS handle from generators in the flat layout of ``workloads.synthetic_hbs``
    (numpy, row-major per-node blocks); uploads column-major copies."""
    tdt = torch.float64 if dtype == HM_F64 else torch.float32
    n, leaf, k = g["n"], g["leaf"], g["k"]
    U = to_fortran(g["U"], tdt)
    V = to_fortran(g["V"], tdt)
    blk = lambda a: torch.from_numpy(np.ascontiguousarray(np.swapaxes(a, 1, 2))).to(
        device="cuda", dtype=tdt).contiguous()
    Ut, Vt, B = blk(g["Ut"]), blk(g["Vt"]), blk(g["B"])
    D = to_fortran(g["D"], tdt)
    h = C.c_void_p()
    _check(lib.hm_hbs_from_generators(n, leaf, k, dtype, _ptr(U), _ptr(V), _ptr(Ut), _ptr(Vt),
                                      _ptr(B), _ptr(D), _stream(stream), C.byref(h)))
    torch.cuda.synchronize()
    return HBS(h)


def hbs_from_tensors(n, leaf, U, V, Ut, Vt, B, D, stream=None) -> HBS:
    """HBS handle from device generator tensors in the flat layout (U, V:
    (n, k); Ut, Vt: (nn, 2k, k); B: (nn, k, k); D: (n, nmax)); FP64 or FP32
    by U's dtype.  The library copies the data."""
    k = U.shape[1]
    dt = HM_F64 if U.dtype == torch.float64 else HM_F32
    tdt = U.dtype
    Uf, Vf, Df = to_fortran(U, tdt), to_fortran(V, tdt), to_fortran(D, tdt)
    blk = lambda a: a.detach().to(device="cuda", dtype=tdt).transpose(1, 2).contiguous()
    Utb, Vtb, Bb = blk(Ut), blk(Vt), blk(B)
    h = C.c_void_p()
    _check(lib.hm_hbs_from_generators(n, leaf, k, dt, _ptr(Uf), _ptr(Vf), _ptr(Utb), _ptr(Vtb),
                                      _ptr(Bb), _ptr(Df), _stream(stream), C.byref(h)))
    return HBS(h)


class HBSApply(torch.autograd.Function):
    """y = A_H(U, V, Ut, Vt, B, D) x with the library's forward (Fig. 7 + D)
    and hand-written backward (gradients w.r.t. x and every generator)."""

    @staticmethod
    def forward(ctx, x, U, V, Ut, Vt, B, D, n, leaf):
        h = hbs_from_tensors(n, leaf, U, V, Ut, Vt, B, D)
        xf = to_fortran(x, U.dtype)
        ctx.h = h
        ctx.save_for_backward(xf)
        return hss_apply(h, xf)

    @staticmethod
    def backward(ctx, gy):
        (xf,) = ctx.saved_tensors
        gx, g = hss_apply_backward(ctx.h, xf, gy)
        return gx, g["U"], g["V"], g["Ut"], g["Vt"], g["B"], g["D"], None, None


def hbs_apply(x, U, V, Ut, Vt, B, D, n, leaf):
    """Differentiable compressed apply (see HBSApply)."""
    return HBSApply.apply(x, U, V, Ut, Vt, B, D, n, leaf)
