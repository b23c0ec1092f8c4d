"""ctypes binding of include/bound.h: the same entry points, argument marshalling only.

Every function takes torch tensors (device memory from PyTorch) and hands their data
pointers and the current HIP stream to libbound.so; all arithmetic runs in the
library's gfx950 kernels.  The library must be built in-tree (``build.py``); there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbound.so")

BOUND_OK, BOUND_E_ARG, BOUND_E_SHAPE, BOUND_E_NOMEM, BOUND_E_HIP, BOUND_E_STATE = 0, -1, -2, -3, -4, -5
BOUND_E_NUMERIC = -6
BOUND_LINEAR, BOUND_CONV2D = 0, 1
BOUND_SAVE_FOR_GRAD, BOUND_NO_SLACK, BOUND_BOTH_SIDES, BOUND_RECOMPUTE = 1, 2, 4, 8
BOUND_OPT_GEMM_ONLY = 1
BOUND_OPT_DIRECT_DMA = 2
BOUND_OPT_CHECK = 4
BOUND_OPT_DETERMINISTIC = 8
BOUND_STOP_RELU, BOUND_STOP_LINEAR = 1, 2

EXPORTED = ("bound_init", "bound_dims", "bound_backward", "bound_concretize", "bound_grad",
            "bound_adam", "bound_sample_bounds", "bound_autotune", "bound_autotune_report", "bound_set_options", "bound_set_plan",
            "bound_profile", "bound_profile_read", "bound_destroy",
            "bound_bab_init", "bound_bab_pick_out", "bound_bab_samples", "bound_bab_search_summary",
            "bound_bab_split", "bound_bab_update_best", "bound_bab_prune", "bound_bab_prune_noalloc",
            "bound_sample_bounds_merge", "bound_bab_cem_start", "bound_bab_cem_samples",
            "bound_bab_cem_refit", "bound_grad_adam", "bound_bab_destroy", "bound_last_error")

_p = ctypes.c_void_p


class BoundLayer(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("in_c", ctypes.c_int32), ("in_h", ctypes.c_int32),
                ("in_w", ctypes.c_int32), ("out_c", ctypes.c_int32), ("out_h", ctypes.c_int32),
                ("out_w", ctypes.c_int32), ("kh", ctypes.c_int32), ("kw", ctypes.c_int32),
                ("stride", ctypes.c_int32), ("pad", ctypes.c_int32), ("weight", _p), ("bias", _p)]


class BoundPass(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("rows", ctypes.c_int32), ("target", ctypes.c_int32),
                ("n_bounds", ctypes.c_int32), ("spec", _p), ("lo", _p), ("hi", _p),
                ("bound_of", _p), ("alpha", _p), ("split_off", _p), ("split_idx", _p),
                ("split_sign", _p), ("nnz", ctypes.c_int32), ("beta", _p), ("x_lo", _p),
                ("x_hi", _p), ("flags", ctypes.c_int32), ("stop_layer", ctypes.c_int32),
                ("stop_mode", ctypes.c_int32)]


class BoundOut(ctypes.Structure):
    _fields_ = [("lower", _p), ("upper", _p), ("ld", ctypes.c_int64), ("coeff", _p),
                ("offset", _p), ("offset_mag", _p), ("best", _p),
                ("pass_id", ctypes.POINTER(ctypes.c_int64)), ("best_upper", _p)]


class BoundAdamStep(ctypes.Structure):
    _fields_ = [("alpha", _p), ("m", _p), ("v", _p), ("step", ctypes.c_int32), ("lr", ctypes.c_float),
                ("b1", ctypes.c_float), ("b2", ctypes.c_float), ("eps", ctypes.c_float),
                ("grad_scale", ctypes.c_float), ("clip_lo", ctypes.c_float), ("clip_hi", ctypes.c_float)]


class BoundError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_LIB = None


def lib():
    """Load libbound.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        L.bound_init.argtypes = [ctypes.POINTER(BoundLayer), ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int64, ctypes.c_int64, _p, ctypes.POINTER(_p)]
        L.bound_dims.argtypes = [_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int32)]
        L.bound_backward.argtypes = [_p, ctypes.POINTER(BoundPass), ctypes.POINTER(BoundOut), _p]
        L.bound_concretize.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _p, _p, _p,
                                       _p, _p, ctypes.c_int32, _p, _p]
        L.bound_grad.argtypes = [_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, _p, _p, _p, _p]
        L.bound_grad_adam.argtypes = [_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, _p, ctypes.POINTER(BoundAdamStep), _p, _p]
        L.bound_sample_bounds.argtypes = [_p, ctypes.c_int32, ctypes.c_int32, _p, _p, _p, _p, _p]
        L.bound_sample_bounds_merge.argtypes = [_p, ctypes.c_int32, ctypes.c_int32, _p, _p, _p, _p, _p]
        L.bound_adam.argtypes = [ctypes.c_int64, _p, _p, _p, _p, ctypes.c_int32, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, _p]
        L.bound_autotune.argtypes = [_p, ctypes.POINTER(BoundPass), ctypes.POINTER(BoundOut), _p, _p]
        L.bound_autotune_report.argtypes = [_p, ctypes.c_char_p, ctypes.c_int32]
        L.bound_autotune_report.restype = ctypes.c_int32
        L.bound_set_options.argtypes = [_p, ctypes.c_int32]
        L.bound_set_plan.argtypes = [_p, ctypes.c_char, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32]
        L.bound_profile.argtypes = [_p, ctypes.c_int32]
        L.bound_profile_read.argtypes = [_p, ctypes.c_int32, ctypes.c_char_p,
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int32)]
        L.bound_profile_read.restype = ctypes.c_int32
        L.bound_destroy.argtypes = [_p]
        L.bound_destroy.restype = None
        i32, f32 = ctypes.c_int32, ctypes.c_float
        L.bound_bab_init.argtypes = [i32, i32, i32, ctypes.POINTER(_p)]
        L.bound_bab_destroy.argtypes = [_p]
        L.bound_bab_destroy.restype = None
        L.bound_bab_pick_out.argtypes = [_p, i32, _p, _p, _p, i32, f32, f32, _p, _p, _p]
        L.bound_bab_samples.argtypes = [_p, i32, i32, _p, _p, _p, _p, _p]
        L.bound_bab_search_summary.argtypes = [_p, i32, i32, _p, _p, i32, _p, _p, _p]
        L.bound_bab_split.argtypes = [_p, i32, _p, _p, _p, i32, _p, _p, _p, _p]
        L.bound_bab_update_best.argtypes = [_p, i32, _p, _p, i32, _p, _p, _p]
        L.bound_bab_prune.argtypes = [_p, i32, _p, _p, _p, _p, _p]
        L.bound_bab_prune_noalloc.argtypes = [i32, _p, _p, _p, _p, _p]
        L.bound_bab_cem_start.argtypes = [_p, i32, _p, _p, _p, i32, _p, _p, _p]
        L.bound_bab_cem_samples.argtypes = [_p, i32, i32, _p, _p, _p, _p, _p, _p, _p, i32, i32, _p]
        L.bound_bab_cem_refit.argtypes = [_p, i32, i32, _p, _p, i32, f32, _p, _p, _p, i32, i32, _p]
        L.bound_last_error.restype = ctypes.c_char_p
        for name in EXPORTED[:-1]:
            if name not in ("bound_profile_read", "bound_autotune_report", "bound_destroy",
                            "bound_bab_destroy"):
                getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(status):
    if status != BOUND_OK:
        raise BoundError(status, lib().bound_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------- entry points
def bound_init(layers, max_inst, max_rows, max_save_rows=0, stream=None):
    """layers: list of dicts with kind/in_shape/out_shape/(stride, pad) and device
    tensors W, b (kept alive by the caller).  Returns an opaque handle."""
    arr = (BoundLayer * len(layers))()
    for i, L in enumerate(layers):
        W, b = L["W"], L["b"]
        if L["kind"] == "conv":
            ci, hi, wi = L["in_shape"]
            co, ho, wo = L["out_shape"]
            arr[i] = BoundLayer(BOUND_CONV2D, ci, hi, wi, co, ho, wo, W.shape[2], W.shape[3],
                                L["stride"], L["pad"], W.data_ptr(), b.data_ptr())
        else:
            ishape = tuple(L.get("in_view", L["in_shape"]))
            ci, hi, wi = (ishape + (1, 1))[:3] if len(ishape) == 1 else ishape
            arr[i] = BoundLayer(BOUND_LINEAR, ci, hi, wi, L["out_shape"][0], 1, 1, 1, 1, 1, 0,
                                W.data_ptr(), b.data_ptr())
    h = _p()
    _check(lib().bound_init(arr, len(layers), int(max_inst), int(max_rows), int(max_save_rows),
                            _stream(stream), ctypes.byref(h)))
    return h


def bound_dims(handle):
    n = ctypes.c_int32()
    nr = ctypes.c_int32()
    _check(lib().bound_dims(handle, ctypes.byref(n), None, ctypes.byref(nr)))   # the layer count
    d = (ctypes.c_int32 * (n.value + 1))()
    _check(lib().bound_dims(handle, ctypes.byref(n), d, ctypes.byref(nr)))
    return [d[i] for i in range(n.value + 1)], nr.value


def _pass_out(n_inst, rows, target, spec, lo, hi, n_bounds, bound_of, alpha, split_off, split_idx,
              split_sign, nnz, beta, x_lo, x_hi, flags, lower, upper, ld, coeff, offset,
              offset_mag, best, stop_layer=0, stop_mode=0, best_upper=None):
    P = BoundPass(int(n_inst), int(rows), int(target), int(n_bounds), _ptr(spec), _ptr(lo), _ptr(hi),
                  _ptr(bound_of), _ptr(alpha), _ptr(split_off), _ptr(split_idx), _ptr(split_sign),
                  int(nnz), _ptr(beta), _ptr(x_lo), _ptr(x_hi), int(flags), int(stop_layer),
                  int(stop_mode))
    O = BoundOut(_ptr(lower), _ptr(upper), int(ld), _ptr(coeff), _ptr(offset), _ptr(offset_mag),
                 _ptr(best), None, _ptr(best_upper))
    return P, O


def bound_autotune(handle, n_inst, rows, target, *, grad_lower=None, spec=None, lo=None, hi=None,
                   n_bounds=0, bound_of=None, alpha=None, split_off=None, split_idx=None,
                   split_sign=None, nnz=0, beta=None, x_lo=None, x_hi=None, flags=0, lower=None,
                   upper=None, ld=0, coeff=None, offset=None, offset_mag=None, best=None,
                   stop_layer=0, stop_mode=0, best_upper=None, stream=None):
    """Tune every product of this pass (and its gradient); returns the timing log."""
    P, O = _pass_out(n_inst, rows, target, spec, lo, hi, n_bounds, bound_of, alpha, split_off,
                     split_idx, split_sign, nnz, beta, x_lo, x_hi, flags, lower, upper, ld, coeff,
                     offset, offset_mag, best, stop_layer, stop_mode, best_upper)
    _check(lib().bound_autotune(handle, ctypes.byref(P), ctypes.byref(O), _ptr(grad_lower),
                                _stream(stream)))
    return bound_autotune_report(handle)


def bound_autotune_report(handle):
    """The last autotuning log: one line per (product, candidate) with its time."""
    n = lib().bound_autotune_report(handle, None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib().bound_autotune_report(handle, buf, n + 1)
    return buf.value.decode()


def bound_backward(handle, n_inst, rows, target, *, spec=None, lo=None, hi=None, n_bounds=0,
                   bound_of=None, alpha=None, split_off=None, split_idx=None, split_sign=None,
                   nnz=0, beta=None, x_lo=None, x_hi=None, flags=0, lower=None, upper=None,
                   ld=0, coeff=None, offset=None, offset_mag=None, best=None, stop_layer=0,
                   stop_mode=0, best_upper=None, stream=None):
    """One bound pass; returns the pass id (a SAVE_FOR_GRAD pass's, else 0)."""
    P = BoundPass(int(n_inst), int(rows), int(target), int(n_bounds), _ptr(spec), _ptr(lo), _ptr(hi),
                  _ptr(bound_of), _ptr(alpha), _ptr(split_off), _ptr(split_idx), _ptr(split_sign),
                  int(nnz), _ptr(beta), _ptr(x_lo), _ptr(x_hi), int(flags), int(stop_layer),
                  int(stop_mode))
    pid = ctypes.c_int64(0)
    O = BoundOut(_ptr(lower), _ptr(upper), int(ld), _ptr(coeff), _ptr(offset), _ptr(offset_mag),
                 _ptr(best), ctypes.pointer(pid), _ptr(best_upper))
    _check(lib().bound_backward(handle, ctypes.byref(P), ctypes.byref(O), _stream(stream)))
    return pid.value


def bound_concretize(n_inst, rows, d0, coeff, offset, offset_mag, x_lo, x_hi, flags, lower,
                     stream=None):
    _check(lib().bound_concretize(int(n_inst), int(rows), int(d0), _ptr(coeff), _ptr(offset),
                                  _ptr(offset_mag), _ptr(x_lo), _ptr(x_hi), int(flags), _ptr(lower),
                                  _stream(stream)))


def bound_sample_bounds(handle, n_sub, per_sub, x, lo=None, hi=None, out=None, stream=None):
    _check(lib().bound_sample_bounds(handle, int(n_sub), int(per_sub), _ptr(x), _ptr(lo), _ptr(hi),
                                     _ptr(out), _stream(stream)))


def bound_sample_bounds_merge(handle, n_sub, per_sub, x, lo, hi, out=None, stream=None):
    _check(lib().bound_sample_bounds_merge(handle, int(n_sub), int(per_sub), _ptr(x), _ptr(lo),
                                           _ptr(hi), _ptr(out), _stream(stream)))


def bound_grad(handle, grad_lower, grad_alpha, grad_beta=None, pass_id=0, stream=None):
    """Shapes are taken from the buffers: grad_lower [n_inst, rows], grad_beta [nnz, rows]."""
    n_inst, rows = grad_lower.shape
    nnz = 0 if grad_beta is None else grad_beta.shape[0]
    _check(lib().bound_grad(handle, int(pass_id), int(n_inst), int(rows), int(nnz),
                            _ptr(grad_lower), _ptr(grad_alpha), _ptr(grad_beta), _stream(stream)))


def bound_grad_adam(handle, grad_lower, alpha, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8,
                    grad_scale=1.0, clip_lo=-float("inf"), clip_hi=float("inf"), grad_beta=None,
                    pass_id=0, stream=None):
    """bound_grad with the alpha-gradient fused into an Adam step on alpha (m, v: moments in
    slot order, shaped like alpha); grad_beta [nnz, rows] or None as in bound_grad."""
    n_inst, rows = grad_lower.shape
    nnz = 0 if grad_beta is None else grad_beta.shape[0]
    a = BoundAdamStep(_ptr(alpha), _ptr(m), _ptr(v), int(step), float(lr), float(b1), float(b2),
                      float(eps), float(grad_scale), float(clip_lo), float(clip_hi))
    _check(lib().bound_grad_adam(handle, int(pass_id), int(n_inst), int(rows), int(nnz),
                                 _ptr(grad_lower), ctypes.byref(a), _ptr(grad_beta), _stream(stream)))


def bound_adam(param, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, grad_scale=1.0,
               clip_lo=-float("inf"), clip_hi=float("inf"), stream=None):
    _check(lib().bound_adam(param.numel(), _ptr(param), _ptr(grad), _ptr(m), _ptr(v), int(step),
                            float(lr), float(b1), float(b2), float(eps), float(grad_scale),
                            float(clip_lo), float(clip_hi), _stream(stream)))


def bound_set_options(handle, options):
    _check(lib().bound_set_options(handle, int(options)))


def bound_set_plan(handle, product, layer, path, cfg, cc):
    _check(lib().bound_set_plan(handle, str(product).encode()[:1], int(layer), int(path), int(cfg),
                                int(cc)))


def bound_profile(handle, enable=True):
    _check(lib().bound_profile(handle, 1 if enable else 0))


def bound_profile_read(handle, cap=256):
    """{label: (total_ms, launches)} since the last read."""
    names = ctypes.create_string_buffer(48 * cap)
    tot = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int32 * cap)()
    n = lib().bound_profile_read(handle, cap, names, tot, cnt)
    if n < 0:
        _check(n)
    raw = names.raw
    out = {}
    for i in range(n):
        nm = raw[48 * i:48 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (tot[i], cnt[i])
    return out


def bound_destroy(handle):
    if handle:
        lib().bound_destroy(handle)


# ------------------------------------------------------- branch and bound over input boxes
def bound_bab_init(max_dom, dim, max_samples):
    h = _p()
    _check(lib().bound_bab_init(int(max_dom), int(dim), int(max_samples), ctypes.byref(h)))
    return h


def bound_bab_destroy(handle):
    if handle:
        lib().bound_bab_destroy(handle)


def bound_bab_pick_out(handle, n_dom, f_lo, f_hi, g, n_pick, eta, temperature, picked, rest,
                       stream=None):
    """g: standard Gumbel variates [n_dom] (the draw's random input)."""
    _check(lib().bound_bab_pick_out(handle, int(n_dom), _ptr(f_lo), _ptr(f_hi), _ptr(g),
                                    int(n_pick), float(eta), float(temperature), _ptr(picked),
                                    _ptr(rest), _stream(stream)))


def bound_bab_samples(handle, n, M, lo, hi, U, samples, stream=None):
    _check(lib().bound_bab_samples(handle, int(n), int(M), _ptr(lo), _ptr(hi), _ptr(U),
                                   _ptr(samples), _stream(stream)))


def bound_bab_cem_start(handle, n, lo, hi, u, u_div, mu, sigma, stream=None):
    _check(lib().bound_bab_cem_start(handle, int(n), _ptr(lo), _ptr(hi), _ptr(u), int(u_div),
                                     _ptr(mu), _ptr(sigma), _stream(stream)))


def bound_bab_cem_samples(handle, n, M, lo, hi, mu, sigma, Z, samples, archive=None, ld=0, a0=0,
                          stream=None):
    _check(lib().bound_bab_cem_samples(handle, int(n), int(M), _ptr(lo), _ptr(hi), _ptr(mu),
                                       _ptr(sigma), _ptr(Z), _ptr(samples), _ptr(archive), int(ld),
                                       int(a0), _stream(stream)))


def bound_bab_cem_refit(handle, n, M, values, samples, n_elite, jitter, mu, sigma,
                        archive_values=None, ld=0, a0=0, stream=None):
    _check(lib().bound_bab_cem_refit(handle, int(n), int(M), _ptr(values), _ptr(samples),
                                     int(n_elite), float(jitter), _ptr(mu), _ptr(sigma),
                                     _ptr(archive_values), int(ld), int(a0), _stream(stream)))


def bound_bab_search_summary(handle, n, M, values, samples, k, f_hi, top, stream=None):
    _check(lib().bound_bab_search_summary(handle, int(n), int(M), _ptr(values), _ptr(samples),
                                          int(k), _ptr(f_hi), _ptr(top), _stream(stream)))


def bound_bab_split(handle, n, lo, hi, top, k, child_lo, child_hi, split_dim=None, stream=None):
    _check(lib().bound_bab_split(handle, int(n), _ptr(lo), _ptr(hi), _ptr(top), int(k),
                                 _ptr(child_lo), _ptr(child_hi), _ptr(split_dim), _stream(stream)))


def bound_bab_update_best(handle, n, f_hi, top, k, best, u_best, stream=None):
    _check(lib().bound_bab_update_best(handle, int(n), _ptr(f_hi), _ptr(top), int(k), _ptr(best),
                                       _ptr(u_best), _stream(stream)))


def bound_bab_prune(handle, n, f_lo, best, keep, n_keep, stream=None):
    _check(lib().bound_bab_prune(handle, int(n), _ptr(f_lo), _ptr(best), _ptr(keep), _ptr(n_keep),
                                 _stream(stream)))


def bound_bab_prune_noalloc(n, f_lo, best, keep, n_keep, stream=None):
    _check(lib().bound_bab_prune_noalloc(int(n), _ptr(f_lo), _ptr(best), _ptr(keep), _ptr(n_keep),
                                         _stream(stream)))


def bound_last_error():
    return lib().bound_last_error().decode()
