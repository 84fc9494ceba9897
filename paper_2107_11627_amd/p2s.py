"""ctypes binding of libp2s (include/p2s.h).

Argument marshalling only: every function checks the torch tensors it is
given (device, dtype, contiguity, shape), passes their device pointers and
the current HIP stream to the C ABI, and turns a negative status into an
exception.  All arithmetic happens in the library's kernels; if the library
is missing the import of this module's functions fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp2s.so")

P2S_OK, P2S_EINVAL, P2S_ENOMEM, P2S_EDEVICE, P2S_EUNSUPPORTED = 0, -1, -2, -3, -4
FP32, BF16, FP8E4M3 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8E4M3}

EXPORTS = [
    "p2s_version", "p2s_last_error", "p2s_noll_variance", "p2s_field_grid",
    "p2s_fields_workspace_bytes", "p2s_workspace_bytes", "p2s_basis_create",
    "p2s_basis_destroy", "p2s_basis_info", "p2s_mlp_create", "p2s_mlp_destroy",
    "p2s_mlp_info", "p2s_make_fields", "p2s_mlp", "p2s_blur", "p2s_mlp_blur", "p2s_warp",
    "p2s_simulate", "p2s_debug_noise", "p2s_batch_workspace_bytes", "p2s_batch_create",
    "p2s_batch_upload", "p2s_batch_launch", "p2s_batch_info", "p2s_batch_destroy", "p2s_simulate_batch",
    "p2s_simulate_noalloc", "p2s_anchor_create", "p2s_anchor_destroy", "p2s_anchor_info",
    "p2s_anchor_fields_workspace_bytes", "p2s_make_fields_anchor", "p2s_workspace_bytes_anchor",
    "p2s_simulate_anchor", "p2s_simulate_spectral",
]


class P2SError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"p2s error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("corr_len_px", C.c_float), ("q_sampling", C.c_float)]


class Frame(C.Structure):
    """One frame of a batch (device pointers)."""
    _fields_ = [("image", C.c_void_p), ("out", C.c_void_p), ("C", C.c_int), ("H", C.c_int), ("W", C.c_int),
                ("D_over_r0", C.c_double), ("seed", C.c_uint64)]


class BatchOptions(C.Structure):
    _fields_ = [("blur_tile_rows", C.c_int), ("persistent", C.c_int)]


N_BATCH_STAGES = 5   # column and row field transforms, network, blur, warp


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2107_11627_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i, sz, d, u64 = C.c_void_p, C.c_int, C.c_size_t, C.c_double, C.c_uint64
        L.p2s_version.restype = i
        L.p2s_last_error.restype = C.c_char_p
        L.p2s_noll_variance.argtypes = [i, C.POINTER(d)]
        L.p2s_field_grid.argtypes = [i, C.c_float, C.POINTER(i)]
        L.p2s_fields_workspace_bytes.argtypes = [i, i, i, vp]
        L.p2s_fields_workspace_bytes.restype = sz
        L.p2s_workspace_bytes.argtypes = [i, i, i, i, i, vp]
        L.p2s_workspace_bytes.restype = sz
        L.p2s_basis_create.argtypes = [vp, i, i, C.POINTER(vp)]
        L.p2s_basis_destroy.argtypes = [vp]
        L.p2s_basis_info.argtypes = [vp, C.POINTER(i), C.POINTER(i)]
        L.p2s_mlp_create.argtypes = [i, C.POINTER(i), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
        L.p2s_mlp_destroy.argtypes = [vp]
        L.p2s_mlp_info.argtypes = [vp, C.POINTER(i), C.POINTER(i)]
        L.p2s_make_fields.argtypes = [i, i, d, i, u64, vp, vp, vp, sz, vp]
        L.p2s_mlp.argtypes = [vp, vp, i, i, i, i, vp, vp]
        L.p2s_blur.argtypes = [vp, i, i, i, vp, vp, i, vp, vp]
        L.p2s_mlp_blur.argtypes = [vp, vp, i, vp, i, i, i, vp, i, vp, vp]
        L.p2s_warp.argtypes = [vp, i, i, i, vp, vp, vp, vp]
        L.p2s_simulate.argtypes = [vp, i, i, i, d, i, vp, vp, u64, i, vp, vp, vp, sz, vp]
        L.p2s_simulate_noalloc.argtypes = [vp, i, i, i, d, i, vp, vp, u64, i, vp, vp, vp]
        L.p2s_debug_noise.argtypes = [i, i, i, u64, vp, vp, vp]
        L.p2s_batch_workspace_bytes.argtypes = [vp, i, i, i, vp]
        L.p2s_batch_workspace_bytes.restype = sz
        L.p2s_batch_create.argtypes = [vp, i, i, vp, vp, i, vp, vp, vp, sz, C.POINTER(vp)]
        L.p2s_batch_upload.argtypes = [vp, vp]
        L.p2s_batch_launch.argtypes = [vp, vp]
        L.p2s_batch_info.argtypes = [vp, C.POINTER(i), C.POINTER(i)]
        L.p2s_batch_destroy.argtypes = [vp]
        L.p2s_simulate_batch.argtypes = [vp, i, i, vp, vp, i, vp, vp, sz, vp]
        L.p2s_anchor_create.argtypes = [i, i, vp, vp, C.POINTER(vp)]
        L.p2s_anchor_destroy.argtypes = [vp]
        L.p2s_anchor_info.argtypes = [vp, C.POINTER(i), C.POINTER(i)]
        L.p2s_anchor_fields_workspace_bytes.argtypes = [vp]
        L.p2s_anchor_fields_workspace_bytes.restype = sz
        L.p2s_make_fields_anchor.argtypes = [vp, i, i, d, u64, vp, vp, sz, vp]
        L.p2s_workspace_bytes_anchor.argtypes = [vp, i, i, i, i]
        L.p2s_workspace_bytes_anchor.restype = sz
        L.p2s_simulate_anchor.argtypes = [vp, i, i, i, d, vp, vp, vp, u64, i, vp, vp, vp, sz, vp]
        L.p2s_simulate_spectral.argtypes = [vp, i, i, i, d, i, vp, vp, u64, i, vp, vp, vp, sz, vp]
        sized = ("p2s_version", "p2s_last_error", "p2s_fields_workspace_bytes", "p2s_workspace_bytes",
                 "p2s_batch_workspace_bytes", "p2s_anchor_fields_workspace_bytes", "p2s_workspace_bytes_anchor")
        for name in EXPORTS:
            if name not in sized:
                getattr(L, name).restype = i
        _lib = L
    return _lib


def _check(rc: int):
    if rc != P2S_OK:
        raise P2SError(rc, lib().p2s_last_error().decode())


def _params(corr_len_px: float = 16.0, q_sampling: float = 2.0):
    return C.byref(Params(corr_len_px, q_sampling))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t, dtype=None, shape=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor, got {t.device}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


# ------------------------------------------------------------------- host
def version() -> int:
    return lib().p2s_version()


def noll_variance(j: int) -> float:
    v = C.c_double()
    _check(lib().p2s_noll_variance(j, C.byref(v)))
    return v.value


def field_grid(n: int, corr_len_px: float = 16.0) -> int:
    v = C.c_int()
    _check(lib().p2s_field_grid(n, C.c_float(corr_len_px), C.byref(v)))
    return v.value


def fields_workspace_bytes(H: int, W: int, n_zernike: int = 35, corr_len_px: float = 16.0) -> int:
    return lib().p2s_fields_workspace_bytes(H, W, n_zernike, _params(corr_len_px))


def workspace_bytes(C_: int, H: int, W: int, n_zernike: int, K: int, corr_len_px: float = 16.0) -> int:
    return lib().p2s_workspace_bytes(C_, H, W, n_zernike, K, _params(corr_len_px))


# ---------------------------------------------------------------- handles
class Basis:
    """Device-resident PSF basis (p2s_basis_create)."""

    def __init__(self, basis: np.ndarray):
        b = np.ascontiguousarray(basis, dtype=np.float64)
        if b.ndim != 3 or b.shape[1] != b.shape[2]:
            raise ValueError("basis must be [K][P][P]")
        self.K, self.P = int(b.shape[0]), int(b.shape[1])
        h = C.c_void_p()
        _check(lib().p2s_basis_create(b.ctypes.data_as(C.c_void_p), self.K, self.P, C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().p2s_basis_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """Device-resident P2S network (p2s_mlp_create)."""

    def __init__(self, weights: Sequence[np.ndarray], biases: Optional[Sequence[np.ndarray]] = None):
        Ws = [np.ascontiguousarray(w, dtype=np.float32) for w in weights]
        L = len(Ws)
        dims = [Ws[0].shape[1]] + [w.shape[0] for w in Ws]
        for l in range(1, L):
            if Ws[l].shape[1] != Ws[l - 1].shape[0]:
                raise ValueError("layer widths do not chain")
        bs = [np.ascontiguousarray(b, dtype=np.float32) for b in biases] if biases is not None else None
        self._keep = (Ws, bs)
        self.dims = dims
        cdims = (C.c_int * (L + 1))(*dims)
        cW = (C.c_void_p * L)(*[w.ctypes.data_as(C.c_void_p) for w in Ws])
        cb = (C.c_void_p * L)(*[b.ctypes.data_as(C.c_void_p) for b in bs]) if bs is not None else None
        h = C.c_void_p()
        _check(lib().p2s_mlp_create(L, cdims, cW, cb, C.byref(h)))
        self.handle = h
        self.n_in, self.n_out = dims[0], dims[-1]

    def close(self):
        if getattr(self, "handle", None):
            lib().p2s_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Anchors:
    """Device-resident anchor-grid field model (p2s_anchor_create): the
    lower Cholesky factors of the anchor correlation matrix [G^2][G^2] and of
    the mode covariance [n][n] per (D/r0)^(5/3)."""

    def __init__(self, G: int, spatial_factor: np.ndarray, mode_factor: np.ndarray):
        Ls = np.ascontiguousarray(spatial_factor, dtype=np.float64)
        Lz = np.ascontiguousarray(mode_factor, dtype=np.float64)
        if Ls.shape != (G * G, G * G):
            raise ValueError(f"spatial factor must be [{G * G}][{G * G}], got {Ls.shape}")
        if Lz.ndim != 2 or Lz.shape[0] != Lz.shape[1]:
            raise ValueError("mode factor must be square")
        self.G, self.n_zernike = int(G), int(Lz.shape[0])
        h = C.c_void_p()
        _check(lib().p2s_anchor_create(self.G, self.n_zernike, Ls.ctypes.data_as(C.c_void_p),
                                       Lz.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.handle = h

    def fields_workspace_bytes(self) -> int:
        return lib().p2s_anchor_fields_workspace_bytes(self.handle)

    def workspace_bytes(self, C_: int, H: int, W: int, K: int) -> int:
        return lib().p2s_workspace_bytes_anchor(self.handle, C_, H, W, K)

    def close(self):
        if getattr(self, "handle", None):
            lib().p2s_anchor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- compute
def make_fields_anchor(anchors: Anchors, H, W, d_over_r0, seed, fields, ws, stream=None):
    import torch
    _check(lib().p2s_make_fields_anchor(anchors.handle, H, W, float(d_over_r0), int(seed) & (2 ** 64 - 1),
                                        _ptr(fields, torch.float32, (anchors.n_zernike, H, W), "fields"),
                                        _ptr(ws, name="ws"), ws.numel() * ws.element_size(), _stream(stream)))


def simulate_anchor(image, d_over_r0, anchors: Anchors, basis: Basis, net: Mlp, seed, precision, out, ws,
                    q_sampling=2.0, stream=None):
    import torch
    C_, H, W = image.shape
    _check(lib().p2s_simulate_anchor(_ptr(image, torch.float32, None, "image"), C_, H, W, float(d_over_r0),
                                     anchors.handle, basis.handle, net.handle, int(seed) & (2 ** 64 - 1),
                                     _prec(precision), _params(16.0, q_sampling),
                                     _ptr(out, torch.float32, (C_, H, W), "out"),
                                     _ptr(ws, name="ws"), ws.numel() * ws.element_size(), _stream(stream)))


def make_fields(H, W, d_over_r0, n_zernike, seed, fields, ws, corr_len_px=16.0, stream=None):
    import torch
    _check(lib().p2s_make_fields(H, W, float(d_over_r0), n_zernike, int(seed) & (2 ** 64 - 1),
                                 _params(corr_len_px), _ptr(fields, torch.float32, (n_zernike, H, W), "fields"),
                                 _ptr(ws, name="ws"), ws.numel() * ws.element_size(), _stream(stream)))


def mlp(net: Mlp, fields, n_zernike, H, W, precision, w, stream=None):
    import torch
    _check(lib().p2s_mlp(net.handle, _ptr(fields, torch.float32, (n_zernike, H, W), "fields"), n_zernike, H, W,
                         _prec(precision), _ptr(w, torch.float32, (H * W, net.n_out), "w"), _stream(stream)))


def blur(image, basis: Basis, w, precision, out, stream=None):
    import torch
    C_, H, W = image.shape
    _check(lib().p2s_blur(_ptr(image, torch.float32, None, "image"), C_, H, W, basis.handle,
                          _ptr(w, torch.float32, (H * W, basis.K), "w"), _prec(precision),
                          _ptr(out, torch.float32, (C_, H, W), "out"), _stream(stream)))


def mlp_blur(net: Mlp, fields, n_zernike, image, basis: Basis, precision, out, stream=None):
    """Network and blur in one kernel (BF16 network; BF16 or FP8 blur)."""
    import torch
    C_, H, W = image.shape
    _check(lib().p2s_mlp_blur(net.handle, _ptr(fields, torch.float32, (n_zernike, H, W), "fields"), n_zernike,
                              _ptr(image, torch.float32, None, "image"), C_, H, W, basis.handle, _prec(precision),
                              _ptr(out, torch.float32, (C_, H, W), "out"), _stream(stream)))


def warp(inp, tilt, out, q_sampling=2.0, stream=None):
    import torch
    C_, H, W = inp.shape
    if tilt.shape[0] < 2 or tuple(tilt.shape[1:]) != (H, W):
        raise ValueError("tilt must be [>=2][H][W]")
    tilt2 = tilt[:2]
    _check(lib().p2s_warp(_ptr(inp, torch.float32, None, "in"), C_, H, W, _ptr(tilt2, torch.float32, None, "tilt"),
                          _params(16.0, q_sampling), _ptr(out, torch.float32, (C_, H, W), "out"), _stream(stream)))


def simulate(image, d_over_r0, basis: Basis, net: Mlp, seed, precision, out, ws, n_zernike=35,
             corr_len_px=16.0, q_sampling=2.0, stream=None):
    import torch
    C_, H, W = image.shape
    _check(lib().p2s_simulate(_ptr(image, torch.float32, None, "image"), C_, H, W, float(d_over_r0), n_zernike,
                              basis.handle, net.handle, int(seed) & (2 ** 64 - 1), _prec(precision),
                              _params(corr_len_px, q_sampling), _ptr(out, torch.float32, (C_, H, W), "out"),
                              _ptr(ws, name="ws"), ws.numel() * ws.element_size(), _stream(stream)))


def simulate_spectral(image, d_over_r0, bases: Sequence[Basis], nets: Sequence[Mlp], seed, precision, out, ws,
                      n_zernike=35, corr_len_px=16.0, q_sampling=2.0, stream=None):
    """One colour frame with a basis and a network per channel."""
    import torch
    C_, H, W = image.shape
    if len(bases) != C_ or len(nets) != C_:
        raise ValueError(f"need {C_} bases and {C_} networks, got {len(bases)} and {len(nets)}")
    cb = (C.c_void_p * C_)(*[b.handle for b in bases])
    cn = (C.c_void_p * C_)(*[n.handle for n in nets])
    _check(lib().p2s_simulate_spectral(_ptr(image, torch.float32, None, "image"), C_, H, W, float(d_over_r0),
                                       n_zernike, cb, cn, int(seed) & (2 ** 64 - 1), _prec(precision),
                                       _params(corr_len_px, q_sampling), _ptr(out, torch.float32, (C_, H, W), "out"),
                                       _ptr(ws, name="ws"), ws.numel() * ws.element_size(), _stream(stream)))


def simulate_noalloc(image, d_over_r0, basis: Basis, net: Mlp, seed, precision, out, n_zernike=35,
                     corr_len_px=16.0, q_sampling=2.0, stream=None):
    """p2s_simulate with the intermediates in the library's device scratch
    (no workspace, no allocation); calls on one GPU must not overlap."""
    import torch
    C_, H, W = image.shape
    _check(lib().p2s_simulate_noalloc(_ptr(image, torch.float32, None, "image"), C_, H, W, float(d_over_r0),
                                      n_zernike, basis.handle, net.handle, int(seed) & (2 ** 64 - 1),
                                      _prec(precision), _params(corr_len_px, q_sampling),
                                      _ptr(out, torch.float32, (C_, H, W), "out"), _stream(stream)))


def debug_noise(Nfy, Nfx, pair, seed, raw, normals=None, stream=None):
    import torch
    _check(lib().p2s_debug_noise(Nfy, Nfx, pair, int(seed) & (2 ** 64 - 1),
                                 _ptr(raw, torch.int32, (Nfy, Nfx, 4), "raw"),
                                 _ptr(normals, torch.float32, (Nfy, Nfx, 2), "normals") if normals is not None else None,
                                 _stream(stream)))


# --------------------------------------------------------------- batches
def _frames(images, outs, d_over_r0s, seeds):
    import torch
    n = len(images)
    if not (len(outs) == n and len(d_over_r0s) == n and len(seeds) == n):
        raise ValueError("images, outs, d_over_r0s and seeds must have the same length")
    arr = (Frame * max(n, 1))()
    for k in range(n):
        im, o = images[k], outs[k]
        if im.dim() != 3:
            raise ValueError(f"image {k} must be [C][H][W]")
        C_, H, W = im.shape
        arr[k] = Frame(_ptr(im, torch.float32, None, f"image {k}"), _ptr(o, torch.float32, (C_, H, W), f"out {k}"),
                       C_, H, W, float(d_over_r0s[k]), int(seeds[k]) & (2 ** 64 - 1))
    return arr, n


def batch_workspace_bytes(shapes, n_zernike: int, K: int, corr_len_px: float = 16.0) -> int:
    """Workspace bytes for frames of the given (C, H, W) shapes; 0 if invalid."""
    n = len(shapes)
    arr = (Frame * max(n, 1))()
    for k, (C_, H, W) in enumerate(shapes):
        arr[k] = Frame(None, None, C_, H, W, 0.0, 0)
    return lib().p2s_batch_workspace_bytes(arr, n, n_zernike, K, _params(corr_len_px))


class Batch:
    """A planned batch: frames of any sizes through the batched kernels.

    create (here) -> upload() -> launch() [graph-capturable, repeatable] -> close().
    The tensors passed in are kept referenced for the handle's lifetime."""

    def __init__(self, images, outs, d_over_r0s, seeds, basis: Basis, net: Mlp, precision, ws, n_zernike=35,
                 corr_len_px=16.0, q_sampling=2.0, blur_tile_rows=16, persistent=True):
        self.handle = None
        arr, n = _frames(images, outs, d_over_r0s, seeds)
        self._keep = (list(images), list(outs), basis, net, ws)
        self.n = n
        opt = BatchOptions(int(blur_tile_rows), 1 if persistent else 0)
        h = C.c_void_p()
        _check(lib().p2s_batch_create(arr, n, n_zernike, basis.handle, net.handle, _prec(precision),
                                      _params(corr_len_px, q_sampling), C.byref(opt),
                                      _ptr(ws, name="ws") if ws is not None else None,
                                      ws.numel() * ws.element_size() if ws is not None else 0, C.byref(h)))
        self.handle = h

    def upload(self, stream=None):
        _check(lib().p2s_batch_upload(self.handle, _stream(stream)))

    def launch(self, stream=None):
        _check(lib().p2s_batch_launch(self.handle, _stream(stream)))

    def info(self):
        items = (C.c_int * N_BATCH_STAGES)()
        grid = (C.c_int * N_BATCH_STAGES)()
        _check(lib().p2s_batch_info(self.handle, items, grid))
        return list(items), list(grid)

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().p2s_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate_batch(images, d_over_r0s, seeds, basis: Basis, net: Mlp, precision, outs, ws, n_zernike=35,
                   corr_len_px=16.0, q_sampling=2.0, stream=None):
    arr, n = _frames(images, outs, d_over_r0s, seeds)
    _check(lib().p2s_simulate_batch(arr, n, n_zernike, basis.handle, net.handle, _prec(precision),
                                    _params(corr_len_px, q_sampling),
                                    _ptr(ws, name="ws") if ws is not None else None,
                                    ws.numel() * ws.element_size() if ws is not None else 0, _stream(stream)))


class Simulator:
    """Resident basis + network + workspace for repeated frames of one size."""

    def __init__(self, basis: np.ndarray, weights, biases=None, n_zernike=35, corr_len_px=16.0, q_sampling=2.0):
        self.basis = Basis(basis)
        self.net = Mlp(weights, biases)
        self.n_zernike = n_zernike
        self.corr_len_px = corr_len_px
        self.q_sampling = q_sampling
        self._ws = None

    def workspace(self, C_, H, W):
        import torch
        n = workspace_bytes(C_, H, W, self.n_zernike, self.basis.K, self.corr_len_px)
        if n == 0:
            raise P2SError(P2S_EINVAL, "invalid frame size")
        if self._ws is None or self._ws.numel() < n:
            self._ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        return self._ws

    def __call__(self, image, d_over_r0, seed, precision="bf16", out=None, stream=None):
        import torch
        C_, H, W = image.shape
        if out is None:
            out = torch.empty_like(image)
        ws = self.workspace(C_, H, W)
        simulate(image, d_over_r0, self.basis, self.net, seed, precision, out, ws, self.n_zernike,
                 self.corr_len_px, self.q_sampling, stream)
        return out

    def batch_workspace(self, shapes):
        import torch
        n = batch_workspace_bytes(shapes, self.n_zernike, self.basis.K, self.corr_len_px)
        if n == 0 and len(shapes) > 0:
            raise P2SError(P2S_EINVAL, "invalid frame sizes")
        return torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")

    def plan(self, images, d_over_r0s, seeds, precision="bf16", outs=None, ws=None, **options):
        """A Batch over these frames (outputs allocated if not given)."""
        import torch
        if outs is None:
            outs = [torch.empty_like(im) for im in images]
        if ws is None:
            ws = self.batch_workspace([tuple(im.shape) for im in images])
        return Batch(images, outs, d_over_r0s, seeds, self.basis, self.net, precision, ws, self.n_zernike,
                     self.corr_len_px, self.q_sampling, **options), outs

    def batch(self, images, d_over_r0s, seeds, precision="bf16", outs=None, ws=None, stream=None):
        """All frames through one batched launch per stage; returns the outputs."""
        import torch
        if outs is None:
            outs = [torch.empty_like(im) for im in images]
        if ws is None:
            ws = self.batch_workspace([tuple(im.shape) for im in images])
        simulate_batch(images, d_over_r0s, seeds, self.basis, self.net, precision, outs, ws, self.n_zernike,
                       self.corr_len_px, self.q_sampling, stream)
        return outs
