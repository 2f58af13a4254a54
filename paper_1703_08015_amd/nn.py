"""Python binding of the warm-start layer kernels (``include/lbm_nn.h``).

Argument marshalling only: every operation is a HIP kernel of liblbm.so.
Tensors are torch tensors on the GPU; activations are bfloat16, channels
last, shaped (nz, ny, nx, C) (C a multiple of 8); convolution weights are
bfloat16 (cout, taps, cin).
"""
import ctypes

from .lbm import LbmError, _check, lib

IDENT, CONV3, GATHER2, SCATTER2 = 0, 1, 2, 3


class Gemm(ctypes.Structure):
    _fields_ = [
        ("src_mode", ctypes.c_int32), ("dst_mode", ctypes.c_int32), ("rows", ctypes.c_int32 * 3),
        ("taps", ctypes.c_int32), ("cin", ctypes.c_int32), ("cout", ctypes.c_int32),
        ("x", ctypes.c_void_p), ("ldx", ctypes.c_int32), ("w", ctypes.c_void_p), ("bias", ctypes.c_void_p),
        ("y", ctypes.c_void_p), ("ldy", ctypes.c_int32), ("y_fp32", ctypes.c_int32), ("relu", ctypes.c_int32),
        ("gate_channels", ctypes.c_int32), ("gate", ctypes.c_void_p), ("ldg", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class WtJob(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("taps", ctypes.c_int32), ("cin", ctypes.c_int32), ("cout", ctypes.c_int32),
                ("w", ctypes.c_void_p), ("wt", ctypes.c_void_p)]


_sigs_done = False


def _lib():
    global _sigs_done
    L = lib()
    if not _sigs_done:
        P, I32, I64, F, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
        G = ctypes.POINTER(Gemm)
        sig = {
            "lbm_nn_forward": [G, P],
            "lbm_nn_forward_ws": [G, P, I64, P],
            "lbm_nn_wgrad": [G, P, P, P],
            "lbm_nn_wgrad_ws": [G, P, P, P, I64, P],
            "lbm_nn_backward_weights": [I32, I32, I32, I32, P, P, P],
            "lbm_nn_backward_weights_batch": [I32, ctypes.POINTER(WtJob), P],
            "lbm_nn_maxpool2": [P, I32, P, I32, P, I32, P, P],
            "lbm_nn_maxpool2_backward": [P, I32, P, I32, P, P, I32, I32, P],
            "lbm_nn_relu_backward": [I64, I32, P, I32, P, I32, P],
            "lbm_nn_mse": [I64, I32, P, P, P, F, P, I32, P, P],
            "lbm_nn_adam": [I64, P, P, P, P, P, F, F, F, F, I32, P],
            "lbm_nn_encode_input": [I64, P, P, P, P],
            "lbm_nn_mix": [I64, P, P, P, P],
            "lbm_nn_mix_backward": [I64, P, I32, P, P, I32, P],
            "lbm_nn_decode_output": [I64, P, P, D, D, I32, P, P, P, P],
            "lbm_nn_distance": [P, ctypes.c_uint32, P, I32, P, P, P],
            "lbm_nn_encode_geometry": [I64, P, P, F, F, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        for name in ("lbm_nn_wgrad_workspace", "lbm_nn_forward_workspace"):
            getattr(L, name).restype = I64
            getattr(L, name).argtypes = [G]
        _sigs_done = True
    return L


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def header_functions():
    import os
    import re
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lbm_nn.h")
    text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_nn_[a-z0-9_]+)\s*\(", text)))


def _gemm(src, dst, rows, taps, cin, cout, x, ldx, w, bias, y, ldy, y_fp32, relu):
    g = Gemm()
    g.src_mode, g.dst_mode = src, dst
    for k in range(3):
        g.rows[k] = int(rows[k])
    g.taps, g.cin, g.cout = taps, cin, cout
    g.x, g.ldx = x, ldx
    g.w, g.bias = w, bias
    g.y, g.ldy = y, ldy
    g.y_fp32, g.relu = int(y_fp32), int(relu)
    return g


def forward(src, dst, rows, taps, cin, cout, x, ldx, w, y, ldy, bias=None, y_fp32=False, relu=False, stream=None,
            x_offset=0, y_offset=0, gate=None, ldg=0, gate_channels=0, gate_offset=0, ws=None):
    """y = act(gather-GEMM(x, w) + bias); x_offset / y_offset / gate_offset
    are element offsets into x, y and gate (channel slices of wider rows).
    With a gate (BF16 rows of stride ldg on the output grid), the first
    gate_channels output channels are zeroed where the gate is not > 0.
    ws (FP32, at least forward_workspace(...) elements): lbm_nn_forward_ws."""
    g = _gemm(src, dst, rows, taps, cin, cout, x.data_ptr() + 2 * x_offset, ldx, w.data_ptr(),
              None if bias is None else bias.data_ptr(), y.data_ptr() + y.element_size() * y_offset, ldy, y_fp32, relu)
    if gate is not None:
        g.gate, g.ldg, g.gate_channels = gate.data_ptr() + 2 * gate_offset, ldg, gate_channels
    if ws is None:
        _check(_lib().lbm_nn_forward(ctypes.byref(g), _stream(stream)), "lbm_nn_forward")
    else:
        _check(_lib().lbm_nn_forward_ws(ctypes.byref(g), _ptr(ws), int(ws.numel()), _stream(stream)),
               "lbm_nn_forward_ws")


def forward_workspace(src, dst, rows, taps, cin, cout, ldx, ldy, y_fp32=False):
    """FP32 elements of the workspace lbm_nn_forward_ws uses for this layer."""
    g = _gemm(src, dst, rows, taps, cin, cout, 16, ldx, 16, None, 16, ldy, y_fp32, False)
    n = int(_lib().lbm_nn_forward_workspace(ctypes.byref(g)))
    if n < 0:
        raise LbmError(-1, "lbm_nn_forward_workspace", "invalid layer")
    return n


def wgrad(src, dst, rows, taps, cin, cout, x, ldx, dy, lddy, dw, db=None, stream=None, x_offset=0, dy_offset=0,
          ws=None):
    """lbm_nn_wgrad, or lbm_nn_wgrad_ws when a workspace tensor (FP32, at
    least wgrad_workspace(...) elements) is given."""
    g = _gemm(src, dst, rows, taps, cin, cout, x.data_ptr() + 2 * x_offset, ldx, None, None,
              dy.data_ptr() + 2 * dy_offset, lddy, False, False)
    if ws is None:
        _check(_lib().lbm_nn_wgrad(ctypes.byref(g), _ptr(dw), _ptr(db), _stream(stream)), "lbm_nn_wgrad")
    else:
        _check(_lib().lbm_nn_wgrad_ws(ctypes.byref(g), _ptr(dw), _ptr(db), _ptr(ws), int(ws.numel()),
                                      _stream(stream)), "lbm_nn_wgrad_ws")


def wgrad_workspace(src, dst, rows, taps, cin, cout, ldx, lddy):
    """FP32 elements of the workspace lbm_nn_wgrad_ws uses for this layer."""
    g = _gemm(src, dst, rows, taps, cin, cout, 16, ldx, None, None, 16, lddy, False, False)
    n = int(_lib().lbm_nn_wgrad_workspace(ctypes.byref(g)))
    if n < 0:
        raise LbmError(-1, "lbm_nn_wgrad_workspace", "invalid layer")
    return n


def backward_weights_batch(jobs, stream=None):
    """jobs: (mode, taps, cin, cout, w, wt) tuples; one launch for all."""
    arr = (WtJob * max(len(jobs), 1))()
    for k, (mode, taps, cin, cout, w, wt) in enumerate(jobs):
        arr[k].mode, arr[k].taps, arr[k].cin, arr[k].cout = mode, taps, cin, cout
        arr[k].w, arr[k].wt = w.data_ptr(), wt.data_ptr()
    _check(_lib().lbm_nn_backward_weights_batch(len(jobs), arr, _stream(stream)), "lbm_nn_backward_weights_batch")


def backward_weights(mode, taps, cin, cout, w, wt, stream=None):
    _check(_lib().lbm_nn_backward_weights(mode, taps, cin, cout, _ptr(w), _ptr(wt), _stream(stream)),
           "lbm_nn_backward_weights")


def _grid(rows):
    return (ctypes.c_int32 * 3)(*[int(v) for v in rows])


def maxpool2(rows, channels, x, ldx, y, ldy, arg, stream=None, x_offset=0):
    _check(_lib().lbm_nn_maxpool2(_grid(rows), channels, ctypes.c_void_p(x.data_ptr() + 2 * x_offset), ldx, _ptr(y),
                                  ldy, _ptr(arg), _stream(stream)), "lbm_nn_maxpool2")


def maxpool2_backward(rows, channels, dy, ldy, arg, dx, ldx, accumulate=False, stream=None, dx_offset=0):
    _check(_lib().lbm_nn_maxpool2_backward(_grid(rows), channels, _ptr(dy), ldy, _ptr(arg),
                                           ctypes.c_void_p(dx.data_ptr() + 2 * dx_offset), ldx, int(accumulate),
                                           _stream(stream)), "lbm_nn_maxpool2_backward")


def relu_backward(n, channels, y, ldy, dy, lddy, stream=None, y_offset=0, dy_offset=0):
    _check(_lib().lbm_nn_relu_backward(int(n), channels, ctypes.c_void_p(y.data_ptr() + 2 * y_offset), ldy,
                                       ctypes.c_void_p(dy.data_ptr() + 2 * dy_offset), lddy, _stream(stream)),
           "lbm_nn_relu_backward")


def mse(n, channels, pred, target, mask, scale, dpred, ldd, loss, stream=None):
    _check(_lib().lbm_nn_mse(int(n), channels, _ptr(pred), _ptr(target), _ptr(mask), float(scale), _ptr(dpred), ldd,
                             _ptr(loss), _stream(stream)), "lbm_nn_mse")


def adam(p, m, v, g, p16, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib().lbm_nn_adam(p.numel(), _ptr(p), _ptr(m), _ptr(v), _ptr(g), _ptr(p16), float(lr), float(beta1),
                              float(beta2), float(eps), int(step), _stream(stream)), "lbm_nn_adam")


def mix(y, direction, p, stream=None):
    d = (ctypes.c_float * 3)(*[float(v) for v in direction])
    _check(_lib().lbm_nn_mix(p.numel() // 4, _ptr(y), d, _ptr(p), _stream(stream)), "lbm_nn_mix")


def mix_backward(dp, ldp, direction, dy, ldy, stream=None):
    d = (ctypes.c_float * 3)(*[float(v) for v in direction])
    _check(_lib().lbm_nn_mix_backward(dy.numel() // ldy, _ptr(dp), ldp, d, _ptr(dy), ldy, _stream(stream)),
           "lbm_nn_mix_backward")


def encode_input(solid, direction, x, stream=None):
    d = (ctypes.c_float * 3)(*[float(v) for v in direction])
    _check(_lib().lbm_nn_encode_input(solid.numel(), _ptr(solid), d, _ptr(x), _stream(stream)),
           "lbm_nn_encode_input")


def distance(solid, dist, tmp, sweeps, periodic=7, stream=None):
    """dist (FP32, shape of solid) = link-path distance to the nearest solid node."""
    shape = (ctypes.c_int32 * 3)(int(solid.shape[-1]), int(solid.shape[-2]), int(solid.shape[-3]))
    _check(_lib().lbm_nn_distance(shape, int(periodic), _ptr(solid), int(sweeps), _ptr(dist), _ptr(tmp),
                                  _stream(stream)), "lbm_nn_distance")


def encode_geometry(solid, dist, scale, cap, x, stream=None):
    _check(_lib().lbm_nn_encode_geometry(solid.numel(), _ptr(solid), _ptr(dist), float(scale), float(cap), _ptr(x),
                                         _stream(stream)), "lbm_nn_encode_geometry")


def decode_output(pred, solid, rho0, scale, rho, u, scratch=None, renorm=True, stream=None):
    _check(_lib().lbm_nn_decode_output(solid.numel(), _ptr(pred), _ptr(solid), float(rho0), float(scale), int(renorm),
                                       _ptr(rho), _ptr(u), _ptr(scratch), _stream(stream)), "lbm_nn_decode_output")
