"""ctypes front end of the CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  Nothing here is shared
with the GPU library.

Parameters follow the paper (Sec. V: lambda_AD = 0.3, lambda_MC = 2.3,
T = 3; Table II footnote: arm caps 21 and 31, colour threshold 13).  The
lambdas are passed as the float32 values a C caller of the library holds,
widened to double.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile oracle.c with the host C compiler into liboracle.so."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I = ctypes.c_int
        Dd = ctypes.c_double
        sig = {
            "or_lut": [Dd, Dd, I, P, P],
            "or_gray": [P, I, I, P],
            "or_downscale": [P, I, I, P],
            "or_census": [P, I, I, P],
            "or_arms": [P, I, I, I, I, I, P],
            "or_cost_left": [P, P, P, P, I, I, I, P, P, P],
            "or_cost_right_from_left": [P, I, I, I, I, P],
            "or_agg_x": [P, P, I, I, P],
            "or_agg_y": [P, P, I, I, P],
            "or_wta": [P, P, P, P, P, P, I, I, I, P, P, P, P, P, P],
            "or_crosscheck": [P, P, I, I, P],
            "or_median": [P, I, I, P],
            "or_fill": [P, P, P, I, I, I, I, P],
            "or_upscale": [P, P, I, I, I, P],
            "or_disparity": [P, P, I, I, I, Dd, Dd, I, I, I, I, I, I, I, I, P] + [P] * 13,
            "or_num_threads": [],
            "or_set_num_threads": [I],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int if name in ("or_wta", "or_disparity", "or_num_threads") else None
        _lib = L
    return _lib


@dataclass
class Params:
    lambda_ad: float = float(np.float32(0.3))
    lambda_mc: float = float(np.float32(2.3))
    cost_scale: int = 1024
    color_delta: int = 13
    arm_x: int = 21
    arm_y: int = 31
    fill_T: int = 3
    arm_x_r: int = -1     # horizontal arm cap of the right image; -1: arm_x
    fill_mode: int = 0    # 0 bilateral (Sec. III-E), 1 closer GCP, 2 smaller disparity
    full_res: bool = False  # the method on the original images (no down/upscale)

    def cap_r(self) -> int:
        return self.arm_x if self.arm_x_r < 0 else self.arm_x_r


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def half_size(W: int, H: int):
    return (W + 1) // 2, (H + 1) // 2


def lut(p: Params = Params()):
    ad = np.zeros(256, np.uint16)
    mc = np.zeros(7, np.uint16)
    lib().or_lut(p.lambda_ad, p.lambda_mc, p.cost_scale, _p(ad), _p(mc))
    return ad, mc


def gray(rgb):
    rgb = _c(rgb, np.uint8)
    H, W, _ = rgb.shape
    g = np.zeros((H, W), np.uint8)
    lib().or_gray(_p(rgb), W, H, _p(g))
    return g


def downscale(g):
    g = _c(g, np.uint8)
    H, W = g.shape
    X, Y = half_size(W, H)
    h = np.zeros((Y, X), np.uint8)
    lib().or_downscale(_p(g), W, H, _p(h))
    return h


def census(h):
    h = _c(h, np.uint8)
    Y, X = h.shape
    c = np.zeros((Y, X), np.uint8)
    lib().or_census(_p(h), X, Y, _p(c))
    return c


def arms(h, p: Params = Params()):
    h = _c(h, np.uint8)
    Y, X = h.shape
    a = np.zeros((Y, X, 4), np.uint8)
    lib().or_arms(_p(h), X, Y, p.color_delta, p.arm_x, p.arm_y, _p(a))
    return a


def cost_left(hl, hr, cl, cr, d, p: Params = Params()):
    hl, hr, cl, cr = (_c(v, np.uint8) for v in (hl, hr, cl, cr))
    Y, X = hl.shape
    ad, mc = lut(p)
    out = np.zeros((Y, X), np.uint16)
    lib().or_cost_left(_p(hl), _p(hr), _p(cl), _p(cr), X, Y, int(d), _p(ad), _p(mc), _p(out))
    return out


def cost_right_from_left(cost_l, d, cmax):
    cost_l = _c(cost_l, np.uint16)
    Y, X = cost_l.shape
    out = np.zeros((Y, X), np.uint16)
    lib().or_cost_right_from_left(_p(cost_l), X, Y, int(d), int(cmax), _p(out))
    return out


def agg_x(cost, a):
    cost = _c(cost, np.uint16)
    a = _c(a, np.uint8)
    Y, X = cost.shape
    out = np.zeros((Y, X), np.uint32)
    lib().or_agg_x(_p(cost), _p(a), X, Y, _p(out))
    return out


def agg_y(cax, a):
    cax = _c(cax, np.uint32)
    a = _c(a, np.uint8)
    Y, X = cax.shape
    out = np.zeros((Y, X), np.uint32)
    lib().or_agg_y(_p(cax), _p(a), X, Y, _p(out))
    return out


def wta(hl, hr, cl, cr, al, ar, D, p: Params = Params()):
    hl, hr, cl, cr = (_c(v, np.uint8) for v in (hl, hr, cl, cr))
    al, ar = _c(al, np.uint8), _c(ar, np.uint8)
    Y, X = hl.shape
    ad, mc = lut(p)
    dl = np.zeros((Y, X), np.int16)
    dr = np.zeros((Y, X), np.int16)
    ml = np.zeros((Y, X), np.uint32)
    mr = np.zeros((Y, X), np.uint32)
    rc = lib().or_wta(_p(hl), _p(hr), _p(cl), _p(cr), _p(al), _p(ar), X, Y, int(D),
                      _p(ad), _p(mc), _p(dl), _p(dr), _p(ml), _p(mr))
    if rc:
        raise MemoryError("oracle or_wta failed")
    return dl, dr, ml, mr


def crosscheck(dl, dr):
    dl, dr = _c(dl, np.int16), _c(dr, np.int16)
    Y, X = dl.shape
    g = np.zeros((Y, X), np.uint8)
    lib().or_crosscheck(_p(dl), _p(dr), X, Y, _p(g))
    return g


def median(d):
    d = _c(d, np.int16)
    Y, X = d.shape
    m = np.zeros((Y, X), np.int16)
    lib().or_median(_p(d), X, Y, _p(m))
    return m


def fill(med, gcp, hl, T=3, mode=0):
    med, gcp, hl = _c(med, np.int16), _c(gcp, np.uint8), _c(hl, np.uint8)
    Y, X = med.shape
    out = np.zeros((Y, X), np.int16)
    lib().or_fill(_p(med), _p(gcp), _p(hl), X, Y, int(T), int(mode), _p(out))
    return out


def upscale(dp, gfull, T=3):
    dp, gfull = _c(dp, np.int16), _c(gfull, np.uint8)
    H, W = gfull.shape
    out = np.zeros((H, W), np.int16)
    lib().or_upscale(_p(dp), _p(gfull), W, H, int(T), _p(out))
    return out


def disparity(left, right, dmax, p: Params = Params()):
    """Whole pipeline; returns a dict with the output and every intermediate."""
    left, right = _c(left, np.uint8), _c(right, np.uint8)
    H, W, _ = left.shape
    X, Y = (W, H) if p.full_res else half_size(W, H)
    r = {
        "out": np.zeros((H, W), np.int16),
        "half_l": np.zeros((Y, X), np.uint8), "half_r": np.zeros((Y, X), np.uint8),
        "census_l": np.zeros((Y, X), np.uint8), "census_r": np.zeros((Y, X), np.uint8),
        "arms_l": np.zeros((Y, X, 4), np.uint8), "arms_r": np.zeros((Y, X, 4), np.uint8),
        "disp_l": np.zeros((Y, X), np.int16), "disp_r": np.zeros((Y, X), np.int16),
        "min_l": np.zeros((Y, X), np.uint32), "min_r": np.zeros((Y, X), np.uint32),
        "gcp": np.zeros((Y, X), np.uint8), "median": np.zeros((Y, X), np.int16),
        "filled": np.zeros((Y, X), np.int16),
    }
    keys = ["half_l", "half_r", "census_l", "census_r", "arms_l", "arms_r", "disp_l",
            "disp_r", "min_l", "min_r", "gcp", "median", "filled"]
    rc = lib().or_disparity(_p(left), _p(right), W, H, int(dmax), p.lambda_ad, p.lambda_mc,
                            p.cost_scale, p.color_delta, p.arm_x, p.arm_y, p.fill_T,
                            p.cap_r(), p.fill_mode, int(p.full_res),
                            _p(r["out"]), *[_p(r[k]) for k in keys])
    if rc:
        raise ValueError(f"oracle or_disparity failed ({rc})")
    return r


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's later calls."""
    lib().or_set_num_threads(int(n))
