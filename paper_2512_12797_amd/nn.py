"""Thin binding of the network kernels (include/fwi_nn.h); device buffers are torch tensors.

BF16 tensors are carried as torch.int16 storage of the raw bf16 bits (the kernels read
and write bf16 bit patterns); use ``as_float`` to view them as floats.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import fwi


class Shape(C.Structure):
    _fields_ = [("n", C.c_int32), ("h", C.c_int32), ("w", C.c_int32), ("c", C.c_int32)]


_L = None


def lib():
    global _L
    if _L is None:
        L = fwi.lib()
        P = C.c_void_p
        sig = {
            "fwi_nn_conv3x3": [P, Shape, P, C.c_int32, P, P, P, C.c_int32, P, P, P],
            "fwi_nn_conv3x3_upcat": [P, C.c_int32, P, Shape, P, C.c_int32, P, P, P, C.c_int32, P, P, P],
            "fwi_nn_wgrad": [P, P, P, Shape, C.c_int32, P, P, P, P],
            "fwi_nn_wgrad_upcat": [P, P, P, C.c_int32, P, Shape, C.c_int32, P, P, P, P],
            "fwi_nn_pool2": [P, Shape, P, P],
            "fwi_nn_pool2_bwd": [P, Shape, P, C.c_int32, P],
            "fwi_nn_up2": [P, Shape, P, P],
            "fwi_nn_up2_bwd": [P, Shape, P, P],
            "fwi_nn_concat": [P, C.c_int32, P, C.c_int32, C.c_int64, P, P],
            "fwi_nn_split_bwd": [P, C.c_int32, C.c_int32, C.c_int64, P, C.c_int32, P, C.c_int32, P],
            "fwi_nn_silu_bwd": [P, P, C.c_int64, P, P, P],
            "fwi_nn_rel_mse": [P, C.c_int32, P, C.c_int32, C.c_int64, P, P, P, P, P],
            "fwi_nn_adam": [P, P, P, P, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32, P],
            "fwi_nn_pack_weights": [P, C.c_int32, C.c_int32, P, P, P],
            "fwi_nn_to_bf16": [P, C.c_int64, P, P],
            "fwi_nn_prep": [P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_float, P, P, P, P, P],
            "fwi_nn_guard": [P, C.c_int32, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_float,
                             C.c_float, C.c_float, P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.fwi_nn_wgrad_work.argtypes = [Shape, C.c_int32]
        L.fwi_nn_wgrad_work.restype = C.c_int64
        L.fwi_nn_last_error.restype = C.c_char_p
        _L = L
    return _L


def _ok(st):
    if st != 0:
        raise fwi.FwiError(st, lib().fwi_nn_last_error().decode())


def _p(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _s():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def bf16_empty(*shape, device="cuda"):
    return torch.empty(*shape, dtype=torch.int16, device=device)


def as_float(t16):
    """FP32 view of raw bf16 bits (copy)."""
    return (t16.to(torch.int32) << 16).view(torch.float32) if t16.dtype == torch.int16 else t16


def conv3x3(x, shape, w, cout, bias=None, aux=None, act=False, out_f32=None, out_bf16=None, res=None):
    _ok(lib().fwi_nn_conv3x3(_p(x), Shape(*shape), _p(w), cout, _p(bias), _p(aux), _p(res), int(act), _p(out_f32),
                             _p(out_bf16), _s()))


def conv3x3_upcat(a, ca, b, shape, w, cout, bias=None, aux=None, act=False, out_f32=None, out_bf16=None, res=None):
    """conv3x3 over the concatenation [up2(a), b] (shape: the concatenated input)."""
    _ok(lib().fwi_nn_conv3x3_upcat(_p(a), ca, _p(b), Shape(*shape), _p(w), cout, _p(bias), _p(aux), _p(res),
                                   int(act), _p(out_f32), _p(out_bf16), _s()))


def wgrad_upcat(dz, dz_f32, a, ca, b, shape, cout, dw, db, work):
    _ok(lib().fwi_nn_wgrad_upcat(_p(dz), _p(dz_f32), _p(a), ca, _p(b), Shape(*shape), cout, _p(dw), _p(db),
                                 _p(work), _s()))


def wgrad_work(shape, cout):
    return int(lib().fwi_nn_wgrad_work(Shape(*shape), cout))


def wgrad(dz, dz_f32, x, shape, cout, dw, db, work):
    _ok(lib().fwi_nn_wgrad(_p(dz), _p(dz_f32), _p(x), Shape(*shape), cout, _p(dw), _p(db), _p(work), _s()))


def pool2(x, shape, out):
    _ok(lib().fwi_nn_pool2(_p(x), Shape(*shape), _p(out), _s()))


def pool2_bwd(dout, shape, dx, accumulate):
    _ok(lib().fwi_nn_pool2_bwd(_p(dout), Shape(*shape), _p(dx), int(accumulate), _s()))


def up2(x, shape, out):
    _ok(lib().fwi_nn_up2(_p(x), Shape(*shape), _p(out), _s()))


def up2_bwd(dout, shape, dx):
    _ok(lib().fwi_nn_up2_bwd(_p(dout), Shape(*shape), _p(dx), _s()))


def concat(a, ca, b, cb, npix, out):
    _ok(lib().fwi_nn_concat(_p(a), ca, _p(b), cb, npix, _p(out), _s()))


def split_bwd(d, ca, cb, npix, da, acc_a, db, acc_b):
    _ok(lib().fwi_nn_split_bwd(_p(d), ca, cb, npix, _p(da), int(acc_a), _p(db), int(acc_b), _s()))


def silu_bwd(da, z, dz_f32, dz_bf16):
    _ok(lib().fwi_nn_silu_bwd(_p(da), _p(z), da.numel(), _p(dz_f32), _p(dz_bf16), _s()))


def rel_mse(pred, c, target, nimg, hw, loss, dpred, dpred_bf16, work):
    _ok(lib().fwi_nn_rel_mse(_p(pred), c, _p(target), nimg, hw, _p(loss), _p(dpred), _p(dpred_bf16), _p(work), _s()))


def adam(p, g, m, v, lr, b1, b2, eps, t):
    _ok(lib().fwi_nn_adam(_p(p), _p(g), _p(m), _p(v), p.numel(), lr, b1, b2, eps, t, _s()))


def pack_weights(wf, cout, cin, w_bf16, wt_bf16):
    _ok(lib().fwi_nn_pack_weights(_p(wf), cout, cin, _p(w_bf16), _p(wt_bf16), _s()))


def to_bf16(x, out):
    _ok(lib().fwi_nn_to_bf16(_p(x), x.numel(), _p(out), _s()))


def prep(g, v, nimg, h, w, hp, v_shift, v_scale, scale_in=None, scale_out=None, x_bf16=None, res=None):
    _ok(lib().fwi_nn_prep(_p(g), _p(v), nimg, h, w, hp, v_shift, v_scale, _p(scale_in), _p(scale_out), _p(x_bf16),
                          _p(res), _s()))


def guard(pred, c, scale, g, nimg, h, w, hp, cos_min, ratio_lo, ratio_hi, out, keep, alpha=1.0):
    _ok(lib().fwi_nn_guard(_p(pred), c, _p(scale), _p(g), nimg, h, w, hp, cos_min, ratio_lo, ratio_hi, alpha,
                           _p(out), _p(keep), _s()))
