"""Python binding of libme.so (argument marshalling only).

Every step of the matrix-element evaluation runs in the HIP kernels behind
the C ABI declared in ``include/me.h``; this module converts torch tensors to
device pointers and the current HIP stream to a handle.  If the shared
library is missing the import of the binding fails: there is no fallback.

Functions with the C names (``me_init``, ``me_eval``, ...) mirror the ABI one
to one; ``MatrixElement`` wraps a context for convenience.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libme.so")

DEFAULT_COUPLINGS = (0.118, 132.507, 1.16639e-5)   # alpha_s, 1/alpha, G_F
DEFAULT_MASSES = (91.188, 2.4414, 173.0, 1.4915)    # M_Z, W_Z, M_top, W_top

ME_OK, ME_EINVAL, ME_EPROCESS, ME_EDEVICE, ME_ENOMEM, ME_ESTATE = 0, -1, -2, -3, -4, -5
ME_FP64, ME_MIXED = 0, 1

NPART = {"ee_mumu": 4, "gg_tt": 4, "gg_ttg": 5, "gg_ttgg": 6, "gg_ttggg": 7}

_lib = None


class MEError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status}): {last_error()}")


def lib():
    """Load libme.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2503_21935_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback implementation")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    L.me_init.argtypes = [ctypes.c_char_p, dp, ctypes.c_int, dp, ctypes.c_int, ctypes.POINTER(vp)]
    L.me_eval.argtypes = [vp, vp, i64, vp, vp]
    L.me_eval_helicities.argtypes = [vp, vp, i64, vp, vp, vp]
    L.me_info.argtypes = [vp, ip, ip, ip, ip, ip, dp]
    L.me_good_helicities.argtypes = [vp, ip, ip]
    L.me_free.argtypes = [vp]
    L.me_strerror.argtypes = [ctypes.c_int]
    L.me_strerror.restype = ctypes.c_char_p
    L.me_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().me_strerror(status).decode()


def last_error() -> str:
    return lib().me_last_error().decode()


def _check(status, where):
    if status != ME_OK:
        raise MEError(status, where)


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype_name, what):
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what} must live on the GPU")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"{what} must be {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------
# C-named wrappers
# --------------------------------------------------------------------------

def me_init(process: str, couplings=DEFAULT_COUPLINGS, masses=DEFAULT_MASSES) -> ctypes.c_void_p:
    c = (ctypes.c_double * len(couplings))(*couplings)
    m = (ctypes.c_double * len(masses))(*masses)
    ctx = ctypes.c_void_p()
    _check(lib().me_init(process.encode(), c, len(couplings), m, len(masses), ctypes.byref(ctx)), "me_init")
    return ctx


def me_eval(ctx, momenta, nevt: int, out_me2, stream=None) -> None:
    _check(lib().me_eval(ctx, _dev_ptr(momenta, "float64", "momenta"), int(nevt),
                         _dev_ptr(out_me2, "float64", "out_me2"), _stream_handle(stream)), "me_eval")


def me_eval_helicities(ctx, momenta, nevt: int, out_me2, out_qhel, stream=None) -> None:
    _check(lib().me_eval_helicities(ctx, _dev_ptr(momenta, "float64", "momenta"), int(nevt),
                                    _dev_ptr(out_me2, "float64", "out_me2"),
                                    _dev_ptr(out_qhel, "float64", "out_qhel"), _stream_handle(stream)),
           "me_eval_helicities")


def me_info(ctx) -> dict:
    v = [ctypes.c_int() for _ in range(5)]
    f = ctypes.c_double()
    _check(lib().me_info(ctx, *[ctypes.byref(x) for x in v], ctypes.byref(f)), "me_info")
    keys = ["npart", "ndiag", "ncol", "nhel", "nhel_good"]
    out = {k: x.value for k, x in zip(keys, v)}
    out["flops_per_event"] = f.value
    return out


def me_good_helicities(ctx) -> list:
    cnt = ctypes.c_int()
    _check(lib().me_good_helicities(ctx, None, ctypes.byref(cnt)), "me_good_helicities")
    buf = (ctypes.c_int * max(1, cnt.value))()
    _check(lib().me_good_helicities(ctx, buf, ctypes.byref(cnt)), "me_good_helicities")
    return list(buf[:cnt.value])


def me_free(ctx) -> None:
    _check(lib().me_free(ctx), "me_free")


# --------------------------------------------------------------------------
# Convenience wrapper
# --------------------------------------------------------------------------

class MatrixElement:
    """One process on the current GPU.  ``eval`` takes float64 momenta
    [nevt][npart][4] on the device and returns |M|^2 [nevt] (float64)."""

    def __init__(self, process: str, couplings=DEFAULT_COUPLINGS, masses=DEFAULT_MASSES):
        self.process = process
        self.ctx = me_init(process, couplings, masses)
        self._info = me_info(self.ctx)

    @property
    def npart(self):
        return self._info["npart"]

    def info(self) -> dict:
        return dict(self._info)

    def good_helicities(self) -> list:
        return me_good_helicities(self.ctx)

    def _check_mom(self, momenta):
        if momenta.dim() != 3 or momenta.shape[1] != self.npart or momenta.shape[2] != 4:
            raise ValueError(f"momenta must be [nevt][{self.npart}][4], got {tuple(momenta.shape)}")

    def eval(self, momenta, out=None, stream=None):
        import torch

        self._check_mom(momenta)
        n = momenta.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        me_eval(self.ctx, momenta, n, out, stream)
        return out

    def eval_helicities(self, momenta, stream=None):
        import torch

        self._check_mom(momenta)
        n = momenta.shape[0]
        out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        q = torch.zeros(n, self._info["nhel"], dtype=torch.float64, device=momenta.device)
        me_eval_helicities(self.ctx, momenta, n, out, q, stream)
        return out, q

    def close(self):
        if self.ctx is not None:
            me_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
