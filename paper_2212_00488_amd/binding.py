"""ctypes binding of the C interface in include/stereo.h.

Marshalling only: torch tensors provide device memory and the HIP stream,
every step of the path runs in the library's kernels.  The library must be
built (``__graft_entry__.build()``); nothing falls back to another
implementation when it is missing.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB

OK, EINVAL, ENOMEM, EHIP, EUNIMPL = 0, -1, -2, -3, -4
F_KEEP_INTERMEDIATES = 1
F_STAGE_TIMING = 2
F_FULL_RES = 4
SOFT_F_REUSE_FEATURES = 1
SOFT_F_SAVE_WEIGHTS = 2
STAGES = ("downscale", "census_arms", "cost_aggregate_wta", "chunk_min",
          "crosscheck_median_fill", "upscale")

# stereo_intermediate: id -> (dtype, trailing dims)
INTERMEDIATES = {
    "half_l": (1, np.uint8, ()), "half_r": (2, np.uint8, ()),
    "census_l": (3, np.uint8, ()), "census_r": (4, np.uint8, ()),
    "arms_l": (5, np.uint8, (4,)), "arms_r": (6, np.uint8, (4,)),
    "cost_l_d": (7, np.uint16, ()), "cost_r_d": (8, np.uint16, ()),
    "cax_l_d": (9, np.uint32, ()), "cax_r_d": (10, np.uint32, ()),
    "ca_l_d": (11, np.uint32, ()), "ca_r_d": (12, np.uint32, ()),
    "mincost_l": (13, np.uint32, ()), "mincost_r": (14, np.uint32, ()),
    "disp_l": (15, np.int16, ()), "disp_r": (16, np.int16, ()),
    "gcp": (17, np.uint8, ()), "median": (18, np.int16, ()), "filled": (19, np.int16, ()),
}
I_LUT = 20


class Params(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("lambda_ad", ctypes.c_float),
                ("lambda_mc", ctypes.c_float), ("cost_scale", ctypes.c_int32),
                ("color_delta", ctypes.c_int32), ("arm_x", ctypes.c_int32),
                ("arm_y", ctypes.c_int32), ("fill_T", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("arm_x_r", ctypes.c_int32),
                ("fill_mode", ctypes.c_int32)]


class SoftParams(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("tau", ctypes.c_float),
                ("color_delta", ctypes.c_int32), ("arm_x", ctypes.c_int32),
                ("arm_y", ctypes.c_int32), ("slab", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("mem_budget", ctypes.c_uint64),
                ("params", Params), ("max_batch", ctypes.c_int32)]


class ServerResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("batch", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class StereoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"stereo error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB)
        P, I, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        L.stereo_default_params.argtypes = [ctypes.POINTER(Params)]
        L.stereo_default_params.restype = None
        L.stereo_create.argtypes = [ctypes.POINTER(P), I, U]
        L.stereo_create.restype = I
        L.stereo_destroy.argtypes = [P]
        L.stereo_destroy.restype = None
        L.stereo_last_error.argtypes = [P]
        L.stereo_last_error.restype = ctypes.c_char_p
        L.stereo_disparity.argtypes = [P, P, P, I, I, I, ctypes.POINTER(Params), P, P]
        L.stereo_disparity.restype = I
        L.stereo_disparity_noalloc.argtypes = [P, P, P, I, I, I, ctypes.POINTER(Params), P, P]
        L.stereo_disparity_noalloc.restype = I
        L.stereo_disparity_batch.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), I, I, I, I,
                                             ctypes.POINTER(Params), ctypes.POINTER(P), P]
        L.stereo_disparity_batch.restype = I
        L.stereo_get_intermediate.argtypes = [P, I, I, P, U, P]
        L.stereo_get_intermediate.restype = I
        L.stereo_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int), I]
        L.stereo_stage_times.restype = I
        L.stereo_autotune.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), I, I, I, I,
                                      ctypes.POINTER(Params), ctypes.POINTER(I),
                                      ctypes.POINTER(I), ctypes.POINTER(ctypes.c_float), I, P]
        L.stereo_autotune.restype = I
        SP = ctypes.POINTER(SoftParams)
        L.stereo_soft_default_params.argtypes = [SP]
        L.stereo_soft_default_params.restype = None
        L.stereo_soft_forward.argtypes = [P, P, P, I, I, I, I, P, SP, P, P, P]
        L.stereo_soft_forward.restype = I
        L.stereo_soft_backward.argtypes = [P, P, P, I, I, I, I, P, SP, P, P, P, P, P, P, P]
        L.stereo_soft_backward.restype = I
        L.stereo_soft_l1_loss.argtypes = [P, P, P, P, I, I, I, P, P]
        L.stereo_soft_l1_loss.restype = I
        L.stereo_soft_l1_grad.argtypes = [P, P, P, P, I, I, I, P, P, P]
        L.stereo_soft_l1_grad.restype = I
        L.stereo_calib_lds_read.argtypes = [P, I, I, P]
        L.stereo_calib_lds_read.restype = I
        L.stereo_calib_valu.argtypes = [P, I, I, P]
        L.stereo_calib_valu.restype = I
        L.stereo_calib_copy.argtypes = [P, P, U, I, P]
        L.stereo_calib_copy.restype = I
        L.stereo_server_default_config.argtypes = [ctypes.POINTER(ServerConfig)]
        L.stereo_server_default_config.restype = None
        L.stereo_server_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(ServerConfig)]
        L.stereo_server_create.restype = I
        L.stereo_server_submit.argtypes = [P, P, P, I, I, I, P, ctypes.c_uint64]
        L.stereo_server_submit.restype = I
        L.stereo_server_poll.argtypes = [P, ctypes.POINTER(ServerResult), I, I]
        L.stereo_server_poll.restype = I
        L.stereo_server_last_error.argtypes = [P]
        L.stereo_server_last_error.restype = ctypes.c_char_p
        L.stereo_server_destroy.argtypes = [P]
        L.stereo_server_destroy.restype = None
        _lib = L
    return _lib


def default_params(**overrides) -> Params:
    p = Params()
    lib().stereo_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def soft_default_params(**overrides) -> SoftParams:
    p = SoftParams()
    lib().stereo_soft_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_dev(t, name, dtype, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _check_image(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.uint8 or t.dim() != 3 or t.shape[2] != 3 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous uint8 [H][W][3] tensor")


class Stereo:
    """A library context on one HIP device."""

    def __init__(self, device: int = 0, mem_cap: int = 0):
        self.device = device
        h = ctypes.c_void_p()
        rc = lib().stereo_create(ctypes.byref(h), device, mem_cap)
        if rc:
            raise StereoError(rc, f"stereo_create(device={device}) failed")
        self._h = h
        self._last_shape = None

    def close(self):
        if getattr(self, "_h", None):
            lib().stereo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().stereo_last_error(self._h).decode()

    def _raise(self, rc):
        if rc:
            raise StereoError(rc, self.last_error())

    def disparity(self, left, right, dmax: int, params: Params | None = None, out=None,
                  stream=None):
        """Full-resolution int16 disparity map of one pair of [H][W][3] uint8 images."""
        import torch
        _check_image(left, "left")
        _check_image(right, "right")
        H, W, _ = left.shape
        if tuple(right.shape) != (H, W, 3):
            raise ValueError("left and right shapes differ")
        if out is None:
            out = torch.empty((H, W), dtype=torch.int16, device=left.device)
        rc = lib().stereo_disparity(self._h, left.data_ptr(), right.data_ptr(), W, H, int(dmax),
                                    ctypes.byref(params) if params is not None else None,
                                    out.data_ptr(), _stream_handle(stream))
        self._raise(rc)
        self._last_shape = (W, H, dmax, params is not None and bool(params.flags & F_FULL_RES))
        return out

    def disparity_noalloc(self, left, right, dmax: int, params: Params | None = None, out=None,
                          stream=None):
        """As disparity(), with the library's scratch in its fixed per-device
        array (no device allocation by the library; overlapping calls on one
        device race).  ``out`` should be given by callers that cannot
        allocate."""
        import torch
        _check_image(left, "left")
        _check_image(right, "right")
        H, W, _ = left.shape
        if tuple(right.shape) != (H, W, 3):
            raise ValueError("left and right shapes differ")
        if out is None:
            out = torch.empty((H, W), dtype=torch.int16, device=left.device)
        else:
            _check_dev(out, "out", torch.int16, (H, W))
        rc = lib().stereo_disparity_noalloc(self._h, left.data_ptr(), right.data_ptr(), W, H,
                                            int(dmax),
                                            ctypes.byref(params) if params is not None else None,
                                            out.data_ptr(), _stream_handle(stream))
        self._raise(rc)
        return out

    def disparity_batch(self, lefts, rights, dmax: int, params: Params | None = None,
                        outs=None, stream=None):
        import torch
        n = len(lefts)
        if n != len(rights) or n < 1:
            raise ValueError("need equally many left and right images")
        for t in list(lefts) + list(rights):
            _check_image(t, "image")
        H, W, _ = lefts[0].shape
        if outs is None:
            outs = [torch.empty((H, W), dtype=torch.int16, device=lefts[0].device)
                    for _ in range(n)]
        arr = ctypes.c_void_p * n
        rc = lib().stereo_disparity_batch(
            self._h, arr(*[t.data_ptr() for t in lefts]), arr(*[t.data_ptr() for t in rights]),
            n, W, H, int(dmax), ctypes.byref(params) if params is not None else None,
            arr(*[t.data_ptr() for t in outs]), _stream_handle(stream))
        self._raise(rc)
        self._last_shape = (W, H, dmax, params is not None and bool(params.flags & F_FULL_RES))
        return outs

    def autotune(self, lefts, rights, dmax: int, params: Params | None = None, stream=None):
        """Tune the d-chunk size of the fused kernel for this shape on the
        given pairs; returns (chosen size, {candidate size: ms per run})."""
        n = len(lefts)
        for t in list(lefts) + list(rights):
            _check_image(t, "image")
        H, W, _ = lefts[0].shape
        arr = ctypes.c_void_p * n
        chosen = ctypes.c_int()
        counts = (ctypes.c_int * 32)()
        times = (ctypes.c_float * 32)()
        rc = lib().stereo_autotune(self._h, arr(*[t.data_ptr() for t in lefts]),
                                   arr(*[t.data_ptr() for t in rights]), n, W, H, int(dmax),
                                   ctypes.byref(params) if params is not None else None,
                                   ctypes.byref(chosen), counts, times, 32,
                                   _stream_handle(stream))
        self._raise(rc)
        out = {}
        for c, v in zip(counts, times):
            if v < 0 or c <= 0:
                break
            out[int(c)] = float(v)
        return chosen.value, out

    def stage_times(self, reset: bool = True):
        """(per-stage milliseconds summed over timed calls, number of calls)."""
        ms = (ctypes.c_double * len(STAGES))()
        n = ctypes.c_int()
        self._raise(lib().stereo_stage_times(self._h, ms, ctypes.byref(n), int(reset)))
        return dict(zip(STAGES, list(ms))), n.value

    def intermediate(self, name: str, d: int = 0, stream=None) -> np.ndarray:
        """A plane of the last call made with F_KEEP_INTERMEDIATES, as numpy."""
        W, H, dmax, full = self._last_shape
        X, Y = (W, H) if full else ((W + 1) // 2, (H + 1) // 2)
        if name == "lut":
            buf = np.zeros(263, np.uint16)
            rc = lib().stereo_get_intermediate(self._h, I_LUT, 0, buf.ctypes.data, buf.nbytes,
                                               _stream_handle(stream))
            self._raise(rc)
            return buf
        which, dt, tail = INTERMEDIATES[name]
        buf = np.zeros((Y, X) + tail, dt)
        rc = lib().stereo_get_intermediate(self._h, which, int(d), buf.ctypes.data, buf.nbytes,
                                           _stream_handle(stream))
        self._raise(rc)
        return buf

    # ------------------------------------------------------ soft-argmin head
    def soft_forward(self, left, right, lambdas, dmax: int, params: SoftParams | None = None,
                     stream=None):
        """(d_hat, lse2), float [n][Y][X] each, of float [n][H][W][3] pairs."""
        import torch
        n, H, W, _ = left.shape
        _check_dev(left, "left", torch.float32, (n, H, W, 3))
        _check_dev(right, "right", torch.float32, (n, H, W, 3))
        _check_dev(lambdas, "lambdas", torch.float32, (2,))
        X, Y = (W + 1) // 2, (H + 1) // 2
        d_hat = torch.empty((n, Y, X), dtype=torch.float32, device=left.device)
        lse2 = torch.empty_like(d_hat)
        rc = lib().stereo_soft_forward(self._h, left.data_ptr(), right.data_ptr(), n, W, H,
                                       int(dmax), lambdas.data_ptr(),
                                       ctypes.byref(params) if params is not None else None,
                                       d_hat.data_ptr(), lse2.data_ptr(), _stream_handle(stream))
        self._raise(rc)
        return d_hat, lse2

    def soft_backward(self, left, right, lambdas, dmax: int, d_hat, lse2, g_dhat,
                      params: SoftParams | None = None, stream=None):
        """(g_left, g_right, g_lambdas) of the head given dL/dd_hat."""
        import torch
        n, H, W, _ = left.shape
        _check_dev(left, "left", torch.float32, (n, H, W, 3))
        _check_dev(right, "right", torch.float32, (n, H, W, 3))
        _check_dev(lambdas, "lambdas", torch.float32, (2,))
        for t, nm in ((d_hat, "d_hat"), (lse2, "lse2"), (g_dhat, "g_dhat")):
            _check_dev(t, nm, torch.float32, (n, (H + 1) // 2, (W + 1) // 2))
        g_left = torch.empty_like(left)
        g_right = torch.empty_like(right)
        g_lam = torch.empty(2, dtype=torch.float32, device=left.device)
        rc = lib().stereo_soft_backward(
            self._h, left.data_ptr(), right.data_ptr(), n, W, H, int(dmax), lambdas.data_ptr(),
            ctypes.byref(params) if params is not None else None, d_hat.data_ptr(),
            lse2.data_ptr(), g_dhat.data_ptr(), g_left.data_ptr(), g_right.data_ptr(),
            g_lam.data_ptr(), _stream_handle(stream))
        self._raise(rc)
        return g_left, g_right, g_lam

    def l1_loss(self, d_hat, gt, nonocc, stream=None):
        """Device float[1] loss of the head (gt int16, nonocc uint8, [n][H][W])."""
        import torch
        n, H, W = gt.shape
        _check_dev(d_hat, "d_hat", torch.float32, (n, (H + 1) // 2, (W + 1) // 2))
        _check_dev(gt, "gt", torch.int16)
        _check_dev(nonocc, "nonocc", torch.uint8, (n, H, W))
        loss = torch.empty(1, dtype=torch.float32, device=d_hat.device)
        rc = lib().stereo_soft_l1_loss(self._h, d_hat.data_ptr(), gt.data_ptr(),
                                       nonocc.data_ptr(), n, W, H, loss.data_ptr(),
                                       _stream_handle(stream))
        self._raise(rc)
        return loss

    def l1_grad(self, d_hat, gt, nonocc, gscale=None, stream=None):
        """dL/dd_hat of l1_loss, times the device scalar gscale (None = 1)."""
        import torch
        n, H, W = gt.shape
        _check_dev(d_hat, "d_hat", torch.float32, (n, (H + 1) // 2, (W + 1) // 2))
        _check_dev(gt, "gt", torch.int16)
        _check_dev(nonocc, "nonocc", torch.uint8, (n, H, W))
        if gscale is not None:
            _check_dev(gscale, "gscale", torch.float32)
        g = torch.empty_like(d_hat)
        rc = lib().stereo_soft_l1_grad(self._h, d_hat.data_ptr(), gt.data_ptr(),
                                       nonocc.data_ptr(), n, W, H,
                                       gscale.data_ptr() if gscale is not None else None,
                                       g.data_ptr(), _stream_handle(stream))
        self._raise(rc)
        return g


def measure_peaks(device: int = 0, repeats: int = 5) -> dict:
    """Peak rates of this device from the library's probes
    (include/stereo_calib.h), each the best of `repeats` timed launches:
    LDS read bandwidth (bytes/s), 32-bit integer VALU lane operations per
    second, and device-memory copy bandwidth (bytes read + written per s)."""
    import torch
    L = lib()
    dev = torch.device("cuda", device)
    props = torch.cuda.get_device_properties(dev)
    blocks = 8 * props.multi_processor_count
    sink = torch.empty(blocks * 1024, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    sh = ctypes.c_void_p(stream.cuda_stream)

    def best(launch, work):
        launch()  # warm
        t = []
        for _ in range(repeats):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            rc = launch()
            b.record(stream)
            if rc:
                raise StereoError(rc, "calibration launch failed")
            b.synchronize()
            t.append(a.elapsed_time(b) / 1e3)
        return work / min(t)

    lds_iters, valu_iters = 400, 400
    lds = best(lambda: L.stereo_calib_lds_read(sink.data_ptr(), blocks, lds_iters, sh),
               blocks * 1024 * lds_iters * 256)
    valu = best(lambda: L.stereo_calib_valu(sink.data_ptr(), blocks, valu_iters, sh),
                blocks * 1024 * valu_iters * 256)
    n = 1 << 30
    src = torch.ones(n // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    hbm = best(lambda: L.stereo_calib_copy(src.data_ptr(), dst.data_ptr(), n,
                                           4 * props.multi_processor_count, sh), 2 * n)
    del src, dst
    return {"lds_read_Bps": lds, "valu_int32_ops": valu, "hbm_copy_Bps": hbm,
            "cus": props.multi_processor_count}
