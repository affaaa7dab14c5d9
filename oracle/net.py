"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of net_oracle.c (the warm-start network's
plain-loop forward/backward reference)."""
import ctypes as C

import numpy as np

from . import lib as _lib

_init = False


def _L():
    global _init
    L = _lib()
    if not _init:
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.onet_param_count.restype = C.c_long
        L.onet_param_count.argtypes = [ip, C.c_int]
        L.onet_run.restype = C.c_double
        L.onet_run.argtypes = [ip, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, C.c_int, dp, dp]
        L.onet_conv3.argtypes = [C.c_int] * 4 + [dp] * 4
        L.onet_conv3_bwd.argtypes = [C.c_int] * 4 + [dp] * 6
        L.onet_bf16.restype = C.c_double
        L.onet_bf16.argtypes = [C.c_double]
        _init = True
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ch(ch):
    return (C.c_int * 4)(*ch)


def param_count(ch=(16, 32, 48, 64), cin=3):
    return int(_L().onet_param_count(_ch(ch), cin))


def run(params, inp, target, mask=None, ch=(16, 32, 48, 64), bf16=True, grad=True):
    """inp [B, cin, n, n, n], target/mask [B, n, n, n]; returns (loss, pred, grad)."""
    inp = np.ascontiguousarray(inp, dtype=np.float64)
    B, cin, n = inp.shape[0], inp.shape[1], inp.shape[2]
    target = np.ascontiguousarray(target, dtype=np.float64)
    mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.float64)
    params = np.ascontiguousarray(params, dtype=np.float64)
    pred = np.zeros((B, n, n, n))
    g = np.zeros_like(params) if grad else None
    loss = _L().onet_run(_ch(ch), cin, B, n, _p(params), _p(inp), _p(target), _p(mask), int(bf16), _p(pred), _p(g))
    return loss, pred, g


def conv3(inp, W, b):
    inp = np.ascontiguousarray(inp, dtype=np.float64)
    B, Ci, n = inp.shape[0], inp.shape[1], inp.shape[2]
    Co = W.shape[0]
    out = np.zeros((B, Co, n, n, n))
    _L().onet_conv3(B, Ci, Co, n, _p(inp), _p(np.ascontiguousarray(W, dtype=np.float64)),
                    _p(np.ascontiguousarray(b, dtype=np.float64)), _p(out))
    return out


def conv3_bwd(inp, W, dout):
    inp = np.ascontiguousarray(inp, dtype=np.float64)
    B, Ci, n = inp.shape[0], inp.shape[1], inp.shape[2]
    Co = W.shape[0]
    din = np.zeros_like(inp)
    dW = np.zeros((Co, Ci, 3, 3, 3))
    db = np.zeros(Co)
    _L().onet_conv3_bwd(B, Ci, Co, n, _p(inp), _p(np.ascontiguousarray(W, dtype=np.float64)),
                        _p(np.ascontiguousarray(dout, dtype=np.float64)), _p(din), _p(dW), _p(db))
    return din, dW, db


def bf16(v):
    return _L().onet_bf16(float(v))


LAYERS = ("E0a", "E0b", "E1a", "E1b", "E2a", "E2b", "E3a", "E3b", "D2a", "D2b", "D1a", "D1b", "D0a", "D0b")


def layer_slices(ch=(16, 32, 48, 64), cin=3):
    """(name, slice) of every parameter tensor in the flat layout of net_oracle.c: per 3x3x3
    layer its weights W[co][ci][3][3][3] then its bias b[co], then the head's c0 weights and
    its bias.  Decoder layer D_l a takes [upsampled level l + 1, skip of level l]."""
    dims = [(cin, ch[0]), (ch[0], ch[0]), (ch[0], ch[1]), (ch[1], ch[1]), (ch[1], ch[2]), (ch[2], ch[2]),
            (ch[2], ch[3]), (ch[3], ch[3]), (ch[3] + ch[2], ch[2]), (ch[2], ch[2]), (ch[2] + ch[1], ch[1]),
            (ch[1], ch[1]), (ch[1] + ch[0], ch[0]), (ch[0], ch[0])]
    out, o = [], 0
    for name, (ci, co) in zip(LAYERS, dims):
        out.append((name + ".W", slice(o, o + co * ci * 27)))
        o += co * ci * 27
        out.append((name + ".b", slice(o, o + co)))
        o += co
    out.append(("head.W", slice(o, o + ch[0])))
    out.append(("head.b", slice(o + ch[0], o + ch[0] + 1)))
    return out
