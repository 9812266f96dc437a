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
ME_COLOUR_VALU, ME_COLOUR_MFMA = 0, 1

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
    L.me_flops.argtypes = [vp, dp, dp, dp]
    L.me_channels.argtypes = [vp, ip]
    L.me_channel_desc.argtypes = [vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_int]
    L.me_eval_multichannel.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.me_set_precision.argtypes = [vp, ctypes.c_int, ctypes.c_double]
    L.me_set_helicity_lanes.argtypes = [vp, ctypes.c_int]
    L.me_set_colour_form.argtypes = [vp, ctypes.c_int]
    L.me_eval_mixed_diag.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.me_fallback_count.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.me_eval_mixed_noalloc.argtypes = [vp, vp, i64, vp, vp]
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


def _opt_ptr(t, dtype_name, what):
    return None if t is None else _dev_ptr(t, dtype_name, what)


def _need(t, n, what):
    """Refuse a buffer with fewer than n elements (a kernel would write or read
    past its end)."""
    if t is not None and t.numel() < n:
        raise ValueError(f"{what} holds {t.numel()} elements, the call touches {n}")


def _nevt(nevt):
    # a negative count is passed on: the library refuses it with ME_EINVAL
    return int(nevt)


def _ctx_sizes(ctx):
    """(npart, nhel) of a context, from me_info."""
    npart, nhel = ctypes.c_int(), ctypes.c_int()
    _check(lib().me_info(ctx, ctypes.byref(npart), None, None, ctypes.byref(nhel), None, None), "me_info")
    return npart.value, nhel.value


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
    nevt = _nevt(nevt)
    npart, _ = _ctx_sizes(ctx)
    _need(momenta, nevt * npart * 4, "momenta")
    _need(out_me2, nevt, "out_me2")
    _check(lib().me_eval(ctx, _dev_ptr(momenta, "float64", "momenta"), int(nevt),
                         _dev_ptr(out_me2, "float64", "out_me2"), _stream_handle(stream)), "me_eval")


def me_eval_helicities(ctx, momenta, nevt: int, out_me2, out_qhel, stream=None) -> None:
    nevt = _nevt(nevt)
    npart, nhel = _ctx_sizes(ctx)
    _need(momenta, nevt * npart * 4, "momenta")
    _need(out_me2, nevt, "out_me2")
    _need(out_qhel, nevt * nhel, "out_qhel")
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
    a, c, x = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().me_flops(ctx, ctypes.byref(a), ctypes.byref(c), ctypes.byref(x)), "me_flops")
    out["flops_amp_per_hel"] = a.value
    out["flops_colour_per_hel"] = c.value
    out["flops_executed_per_hel"] = x.value
    return out


def me_good_helicities(ctx) -> list:
    cnt = ctypes.c_int()
    _check(lib().me_good_helicities(ctx, None, ctypes.byref(cnt)), "me_good_helicities")
    buf = (ctypes.c_int * max(1, cnt.value))()
    _check(lib().me_good_helicities(ctx, buf, ctypes.byref(cnt)), "me_good_helicities")
    return list(buf[:cnt.value])


def me_channels(ctx) -> list:
    """Descriptors of the process's channels (empty without a multi-channel form)."""
    n = ctypes.c_int()
    _check(lib().me_channels(ctx, ctypes.byref(n)), "me_channels")
    out = []
    buf = ctypes.create_string_buffer(256)
    for i in range(n.value):
        _check(lib().me_channel_desc(ctx, i, buf, 256), "me_channel_desc")
        out.append(buf.value.decode())
    return out


def me_eval_multichannel(ctx, momenta, chan, nevt: int, out_me2, out_alpha, stream=None) -> None:
    nevt = _nevt(nevt)
    npart, _ = _ctx_sizes(ctx)
    _need(momenta, nevt * npart * 4, "momenta")
    for t, what in ((chan, "chan"), (out_me2, "out_me2"), (out_alpha, "out_alpha")):
        _need(t, nevt, what)
    _check(lib().me_eval_multichannel(ctx, _dev_ptr(momenta, "float64", "momenta"), _dev_ptr(chan, "int32", "chan"),
                                      nevt, _dev_ptr(out_me2, "float64", "out_me2"),
                                      _dev_ptr(out_alpha, "float64", "out_alpha"), _stream_handle(stream)),
           "me_eval_multichannel")


def me_set_precision(ctx, mode: int, rel_tol: float = 1e-5) -> None:
    _check(lib().me_set_precision(ctx, int(mode), float(rel_tol)), "me_set_precision")


def me_set_helicity_lanes(ctx, lanes: int) -> None:
    _check(lib().me_set_helicity_lanes(ctx, int(lanes)), "me_set_helicity_lanes")


def me_set_colour_form(ctx, form: int) -> None:
    _check(lib().me_set_colour_form(ctx, int(form)), "me_set_colour_form")


def me_eval_mixed_diag(ctx, momenta, nevt: int, out_me2, out_err, out_flag, stream=None) -> None:
    nevt = _nevt(nevt)
    npart, _ = _ctx_sizes(ctx)
    _need(momenta, nevt * npart * 4, "momenta")
    for t, what in ((out_me2, "out_me2"), (out_err, "out_err"), (out_flag, "out_flag")):
        _need(t, nevt, what)
    _check(lib().me_eval_mixed_diag(ctx, _dev_ptr(momenta, "float64", "momenta"), int(nevt),
                                    _dev_ptr(out_me2, "float64", "out_me2"), _dev_ptr(out_err, "float32", "out_err"),
                                    _dev_ptr(out_flag, "uint8", "out_flag"), _stream_handle(stream)),
           "me_eval_mixed_diag")


def me_eval_mixed_noalloc(ctx, momenta, nevt: int, out_me2, stream=None) -> None:
    nevt = _nevt(nevt)
    npart, _ = _ctx_sizes(ctx)
    _need(momenta, nevt * npart * 4, "momenta")
    _need(out_me2, nevt, "out_me2")
    _check(lib().me_eval_mixed_noalloc(ctx, _dev_ptr(momenta, "float64", "momenta"), int(nevt),
                                       _dev_ptr(out_me2, "float64", "out_me2"), _stream_handle(stream)),
           "me_eval_mixed_noalloc")


def me_fallback_count(ctx) -> int:
    c = ctypes.c_int64()
    _check(lib().me_fallback_count(ctx, ctypes.byref(c)), "me_fallback_count")
    return c.value


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

    def set_precision(self, mode, rel_tol=1e-5):
        me_set_precision(self.ctx, mode, rel_tol)

    def set_helicity_lanes(self, lanes):
        me_set_helicity_lanes(self.ctx, lanes)

    def set_colour_form(self, form):
        me_set_colour_form(self.ctx, form)

    def channels(self) -> list:
        return me_channels(self.ctx)

    def eval_multichannel(self, momenta, chan, stream=None):
        """(|M|^2, single-diagram weight of each event's channel)."""
        import torch

        self._check_mom(momenta)
        n = momenta.shape[0]
        out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        alpha = torch.empty(n, dtype=torch.float64, device=momenta.device)
        me_eval_multichannel(self.ctx, momenta, chan, n, out, alpha, stream)
        return out, alpha

    def eval_mixed_diag(self, momenta, stream=None):
        """Mixed form without the float64 rerun: (me2, error estimate, flag)."""
        import torch

        self._check_mom(momenta)
        n = momenta.shape[0]
        out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        err = torch.empty(n, dtype=torch.float32, device=momenta.device)
        flag = torch.empty(n, dtype=torch.uint8, device=momenta.device)
        me_eval_mixed_diag(self.ctx, momenta, n, out, err, flag, stream)
        return out, err, flag

    def fallback_count(self) -> int:
        return me_fallback_count(self.ctx)

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


# --------------------------------------------------------------------------
# Phase-space sampling (include/ps.h)
# --------------------------------------------------------------------------

def ps_rambo(roots, masses, seed, first_event, nevt, momenta, weights=None, stream=None) -> None:
    L = lib()
    if not getattr(L, "_ps_ready", False):
        L.ps_rambo.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_uint64,
                               ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L._ps_ready = True
    nf = len(masses)
    nevt = _nevt(nevt)
    _need(momenta, nevt * (nf + 2) * 4, "momenta")
    _need(weights, nevt, "weights")
    m = (ctypes.c_double * max(1, nf))(*masses)
    _check(L.ps_rambo(float(roots), m, nf, int(seed), int(first_event), nevt,
                      _dev_ptr(momenta, "float64", "momenta"), _opt_ptr(weights, "float64", "weights"),
                      _stream_handle(stream)), "ps_rambo")


def ps_multichannel(roots, nfinal, pair, window, mz, wz, alpha, seed, first_event, nevt, momenta, weights=None,
                    channels=None, stream=None) -> None:
    L = lib()
    if not getattr(L, "_ps_mc_ready", False):
        d, vp = ctypes.c_double, ctypes.c_void_p
        L.ps_multichannel.argtypes = [d, ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d, d, d,
                                      ctypes.POINTER(d), ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, vp, vp,
                                      vp, vp]
        L._ps_mc_ready = True
    nevt = _nevt(nevt)
    _need(momenta, nevt * (nfinal + 2) * 4, "momenta")
    _need(weights, nevt, "weights")
    _need(channels, nevt, "channels")
    a = (ctypes.c_double * 3)(*[float(v) for v in alpha])
    _check(L.ps_multichannel(float(roots), int(nfinal), int(pair[0]), int(pair[1]), float(window[0]),
                             float(window[1]), float(mz), float(wz), a, int(seed), int(first_event), nevt,
                             _dev_ptr(momenta, "float64", "momenta"), _opt_ptr(weights, "float64", "weights"),
                             _opt_ptr(channels, "int32", "channels"), _stream_handle(stream)), "ps_multichannel")


def multichannel(roots, nfinal, pair, window, mz, wz, alpha, seed, n, first_event=0, device="cuda", stream=None):
    """Multi-channel phase-space points for a final state with a lepton pair
    (flat, Breit-Wigner and 1/M^2 channels on the pair mass), generated on the
    GPU: (momenta [n][nfinal + 2][4], weights [n], channels [n])."""
    import torch

    mom = torch.empty((n, nfinal + 2, 4), dtype=torch.float64, device=device)
    wt = torch.empty(n, dtype=torch.float64, device=device)
    ch = torch.empty(n, dtype=torch.int32, device=device)
    ps_multichannel(roots, nfinal, pair, window, mz, wz, alpha, seed, first_event, n, mom, wt, ch, stream)
    return mom, wt, ch


def rambo(roots, masses, seed, n, first_event=0, device="cuda", stream=None):
    """Flat phase-space points generated on the GPU: (momenta [n][nf + 2][4],
    weights [n]) as float64 device tensors."""
    import torch

    mom = torch.empty((n, len(masses) + 2, 4), dtype=torch.float64, device=device)
    wt = torch.empty(n, dtype=torch.float64, device=device)
    ps_rambo(roots, masses, seed, first_event, n, mom, wt, stream)
    return mom, wt


# --------------------------------------------------------------------------
# Surrogate network and two-stage unweighting (include/mlp.h)
# --------------------------------------------------------------------------

def _mlp_sigs(L):
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    if getattr(L, "_mlp_ready", False):
        return L
    L.mlp_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(vp)]
    L.mlp_n_params.argtypes = [vp, ctypes.POINTER(i64)]
    L.mlp_dims.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                           ctypes.POINTER(ctypes.c_int)]
    L.mlp_get_params.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i64]
    L.mlp_set_params.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i64]
    L.mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    L.mlp_train_step.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, vp, vp]
    L.mlp_train_steps.argtypes = [vp, vp, vp, vp, i64, i64, vp, vp, vp]
    L.mlp_backward.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
    L.mlp_free.argtypes = [vp]
    L.mlp_set_fused_step.argtypes = [vp, ctypes.c_int]
    L.me_features.argtypes = [vp, i64, ctypes.c_int, vp, vp]
    L.unweight_two_stage.argtypes = [vp, vp, vp, vp, i64, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, vp, vp, vp, vp]
    L._mlp_ready = True
    return L


def mlp_create(n_in=24, width=256, depth=4, seed=1004):
    h = ctypes.c_void_p()
    _check(_mlp_sigs(lib()).mlp_create(n_in, width, depth, seed, ctypes.byref(h)), "mlp_create")
    return h


def mlp_n_params(h) -> int:
    n = ctypes.c_int64()
    _check(_mlp_sigs(lib()).mlp_n_params(h, ctypes.byref(n)), "mlp_n_params")
    return n.value


def mlp_dims(h):
    """(n_in, width, depth) of a network."""
    v = [ctypes.c_int() for _ in range(3)]
    _check(_mlp_sigs(lib()).mlp_dims(h, *[ctypes.byref(x) for x in v]), "mlp_dims")
    return tuple(x.value for x in v)


def _batch_checks(h, x, t, idx, n):
    n = int(n)
    if idx is not None:
        _need(idx, n, "idx")
    else:
        n_in = mlp_dims(h)[0]
        _need(x, n * n_in, "x")
        _need(t, n, "t")
    return n


def mlp_get_params(h):
    import numpy as np

    n = mlp_n_params(h)
    out = np.empty(n, dtype=np.float32)
    _check(lib().mlp_get_params(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n), "mlp_get_params")
    return out


def mlp_set_params(h, params) -> None:
    import numpy as np

    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(_mlp_sigs(lib()).mlp_set_params(h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
           "mlp_set_params")


def mlp_forward(h, x, n, y, stream=None) -> None:
    n = _nevt(n)
    _need(x, n * mlp_dims(h)[0], "x")
    _need(y, n, "y")
    _check(_mlp_sigs(lib()).mlp_forward(h, _dev_ptr(x, "float32", "x"), int(n), _dev_ptr(y, "float32", "y"),
                                        _stream_handle(stream)), "mlp_forward")


def mlp_train_step(h, x, t, idx, n, lr, loss=None, stream=None) -> None:
    n = _batch_checks(h, x, t, idx, n)
    _need(loss, 1, "loss")
    _check(_mlp_sigs(lib()).mlp_train_step(h, _dev_ptr(x, "float32", "x"), _dev_ptr(t, "float32", "t"),
                                           _opt_ptr(idx, "int32", "idx"), int(n), float(lr),
                                           _opt_ptr(loss, "float32", "loss"), _stream_handle(stream)),
           "mlp_train_step")


def mlp_train_steps(h, x, t, idx, n, lr, loss=None, stream=None) -> None:
    """len(lr) consecutive Adam steps of batch n: step s on rows idx[s n:(s+1) n]
    (idx None: rows s n ..); lr a device float32 tensor of per-step rates; loss
    None or a device float32 tensor of one entry per step."""
    n = int(n)
    nsteps = _nevt(lr.numel())
    if idx is not None:
        _need(idx, n * nsteps, "idx")
    else:
        _need(x, n * nsteps * mlp_dims(h)[0], "x")
        _need(t, n * nsteps, "t")
    _need(loss, nsteps, "loss")
    _check(_mlp_sigs(lib()).mlp_train_steps(h, _dev_ptr(x, "float32", "x"), _dev_ptr(t, "float32", "t"),
                                            _opt_ptr(idx, "int32", "idx"), n, nsteps,
                                            _dev_ptr(lr, "float32", "lr"), _opt_ptr(loss, "float32", "loss"),
                                            _stream_handle(stream)), "mlp_train_steps")


def mlp_backward(h, x, t, idx, n, grad, loss=None, stream=None) -> None:
    n = _batch_checks(h, x, t, idx, n)
    _need(grad, mlp_n_params(h), "grad")
    _need(loss, 1, "loss")
    _check(_mlp_sigs(lib()).mlp_backward(h, _dev_ptr(x, "float32", "x"), _dev_ptr(t, "float32", "t"),
                                         _opt_ptr(idx, "int32", "idx"), int(n), _dev_ptr(grad, "float32", "grad"),
                                         _opt_ptr(loss, "float32", "loss"), _stream_handle(stream)), "mlp_backward")


def mlp_set_fused_step(h, on: bool) -> None:
    _check(_mlp_sigs(lib()).mlp_set_fused_step(h, int(bool(on))), "mlp_set_fused_step")


def mlp_free(h) -> None:
    _check(_mlp_sigs(lib()).mlp_free(h), "mlp_free")


def me_features(momenta, n, npart, x, stream=None) -> None:
    n = _nevt(n)
    _need(momenta, n * int(npart) * 4, "momenta")
    _need(x, n * int(npart) * 4, "x")
    _check(_mlp_sigs(lib()).me_features(_dev_ptr(momenta, "float64", "momenta"), int(n), int(npart),
                                        _dev_ptr(x, "float32", "x"), _stream_handle(stream)), "me_features")


def unweight_two_stage(ctx, mlp, momenta, w_ps, n, uniforms, y_mu, y_sigma, s_max, r_max, out_idx, out_w,
                       out_count, stream=None) -> None:
    n = _nevt(n)
    npart, _ = _ctx_sizes(ctx)
    _need(momenta, n * npart * 4, "momenta")
    _need(w_ps, n, "w_ps")
    _need(uniforms, 2 * n, "uniforms")
    _need(out_idx, n, "out_idx")
    _need(out_w, n, "out_w")
    _need(out_count, 2, "out_count")
    _check(_mlp_sigs(lib()).unweight_two_stage(
        ctx, mlp, _dev_ptr(momenta, "float64", "momenta"), _dev_ptr(w_ps, "float64", "w_ps"), int(n),
        _dev_ptr(uniforms, "float64", "uniforms"), float(y_mu), float(y_sigma), float(s_max), float(r_max),
        _dev_ptr(out_idx, "int32", "out_idx"), _dev_ptr(out_w, "float64", "out_w"),
        _dev_ptr(out_count, "int32", "out_count"), _stream_handle(stream)), "unweight_two_stage")


class Surrogate:
    """The network on the current GPU (wraps an mlp handle)."""

    def __init__(self, n_in=24, width=256, depth=4, seed=1004):
        self.n_in, self.width, self.depth = n_in, width, depth
        self.h = mlp_create(n_in, width, depth, seed)

    @property
    def n_params(self):
        return mlp_n_params(self.h)

    def get_params(self):
        return mlp_get_params(self.h)

    def set_params(self, p):
        mlp_set_params(self.h, p)

    def forward(self, x, stream=None):
        import torch

        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        mlp_forward(self.h, x, x.shape[0], y, stream)
        return y

    def train_step(self, x, t, idx, lr, loss=None, stream=None):
        n = idx.shape[0] if idx is not None else x.shape[0]
        mlp_train_step(self.h, x, t, idx, n, lr, loss, stream)

    def train_steps(self, x, t, idx, n, lr, loss=None, stream=None):
        """len(lr) steps of batch n in one call (see mlp_train_steps)."""
        mlp_train_steps(self.h, x, t, idx, n, lr, loss, stream)

    def set_fused_step(self, on):
        mlp_set_fused_step(self.h, on)

    def backward(self, x, t, idx=None, stream=None):
        import torch

        n = idx.shape[0] if idx is not None else x.shape[0]
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        mlp_backward(self.h, x, t, idx, n, g, loss, stream)
        return g, loss

    def close(self):
        if self.h is not None:
            mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(momenta, stream=None):
    """Network inputs [n][4 npart] float32 from float64 momenta [n][npart][4]."""
    import torch

    n, npart = momenta.shape[0], momenta.shape[1]
    x = torch.empty(n, 4 * npart, dtype=torch.float32, device=momenta.device)
    me_features(momenta, n, npart, x, stream)
    return x
