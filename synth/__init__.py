"""Seeded synthetic luma inputs shared by the GPU path's tests/bench and the oracle.

This package renders frames only.  It contains none of the coding-tree search
arithmetic; see ``synth.c`` for the content model.  The thesis measures on
three camera clips (BasketballDrive, CrowdRun, DucksTakeOff) at 540p, 1080p and
2160p (Testing method section, test-video table); those clips are not
available, so seeded synthetic frames with the same resolutions stand in for
them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

SEED_BASE = 0x230112191


def build(force: bool = True) -> str:
    """Compile the generator into synth/libsynth.so with gcc (OpenMP over rows)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC,
                               "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.syn_scene_size.restype = ctypes.c_int
        lib.syn_scene_init.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32]
        lib.syn_render.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_int32]
        lib.syn_box_downscale.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.syn_white_noise.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_int32]
        _lib = lib
    return _lib


class Scene:
    """A seeded scene: background value noise, moving textured rectangles, sensor noise."""

    def __init__(self, seed: int, width: int, height: int, n_rects: int, mv_max: int,
                 pan_max: int = 0, sigma: float = 2.0):
        lib = _load()
        self.width, self.height = width, height
        self._buf = ctypes.create_string_buffer(lib.syn_scene_size())
        rc = lib.syn_scene_init(self._buf, seed & (2**64 - 1), width, height, n_rects, mv_max,
                                pan_max, int(round(sigma * 16)))
        if rc != 0:
            raise ValueError("invalid scene parameters")

    def render(self, t: int) -> np.ndarray:
        out = np.empty((self.height, self.width), dtype=np.uint8)
        rc = _load().syn_render(self._buf, t, out.ctypes.data, self.width)
        if rc != 0:
            raise ValueError("render failed")
        return out


def box_downscale(src: np.ndarray, n: int, dw: int, dh: int) -> np.ndarray:
    """Box filter by an integer factor n with rounding, then crop to (dw, dh)."""
    src = np.ascontiguousarray(src, dtype=np.uint8)
    sh, sw = src.shape
    if n == 1 and (dw, dh) == (sw, sh):
        return src.copy()
    out = np.empty((dh, dw), dtype=np.uint8)
    rc = _load().syn_box_downscale(src.ctypes.data, sw, sh, sw, n, out.ctypes.data, dw, dh, dw)
    if rc != 0:
        raise ValueError("invalid downscale")
    return out


def white_noise(seed: int, width: int, height: int) -> np.ndarray:
    out = np.empty((height, width), dtype=np.uint8)
    _load().syn_white_noise(seed & (2**64 - 1), width, height, out.ctypes.data, width)
    return out


def search_range_for_width(width: int) -> int:
    """Search range R = 8 * ceil(W / 240): 16 for 416/426, 24, 32, 48, 64, 128 for 3840."""
    return 8 * ((width + 239) // 240)


# The six-rung ladder derived from one 3840x2160 source: (width, height, box factor, QP).
LADDER = [
    (426, 240, 9, 37),
    (640, 360, 6, 35),
    (960, 540, 4, 32),
    (1280, 720, 3, 30),
    (1920, 1080, 2, 27),
    (3840, 2160, 1, 22),
]
