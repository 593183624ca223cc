"""CPU oracle for the coding-tree search -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (``paper_2301_12191_amd``)
never imports it, and the two share no code: the oracle is ``oracle.cpp``
compiled by gcc, loaded here with ctypes.

Functions and the passages they follow are documented in ``oracle.cpp``.
Parity status: every function is pinned by ``tests/test_oracle_pins.py``
(closed forms, hand-derived examples, brute force and invariants).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

NODE_FIELDS = ("kind", "mode", "mx", "my", "sad", "satd_inter", "satd_planar", "satd_dc",
               "leaf_j", "leaf_d", "leaf_r", "qmx", "qmy", "satd_angular_best")


def build(force: bool = True) -> str:
    """Compile oracle.cpp with g++ (-O2, no intrinsics) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", _SRC,
                               "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.orc_sqrt_lambda_q16.restype = i64
        L.orc_sqrt_lambda_q16.argtypes = [i32]
        L.orc_se_bits.restype = i32
        L.orc_se_bits.argtypes = [i32]
        L.orc_satd.restype = i64
        L.orc_satd.argtypes = [vp, i32, i32]
        L.orc_intra_predict.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, vp]
        L.orc_cu_motion_search.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, i32, i32, vp,
                                           vp, vp]
        L.orc_ctu_nodes.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, i32, i32, vp, i32,
                                    i32, i32, i32, vp]
        L.orc_ctu_search.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, vp, vp, i32, i32,
                                     i32, i32, vp, vp, vp, vp, vp, vp, vp, i32, i32]
        L.orc_mv_centre.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i32, i32, i32, vp,
                                    vp]
        L.orc_interp_qpel.argtypes = [vp, i32, i32, i32, i32, i32]
        L.orc_subpel_refine.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, i32, i32, i32,
                                        vp, vp, vp]
        L.orc_depth_bounds.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp]
        _lib = L
    return _lib


def sqrt_lambda_q16(qp: int) -> int:
    return int(lib().orc_sqrt_lambda_q16(qp))


def se_bits(v: int) -> int:
    return int(lib().orc_se_bits(v))


def satd(resid: np.ndarray) -> int:
    r = np.ascontiguousarray(resid, dtype=np.int32)
    n = r.shape[0]
    assert r.shape == (n, n) and n % 4 == 0
    return int(lib().orc_satd(_p(r), n, n))


def intra_predict(cur: np.ndarray, x0: int, y0: int, n: int, mode: int) -> np.ndarray:
    c = np.ascontiguousarray(cur, dtype=np.uint8)
    out = np.empty((n, n), dtype=np.int32)
    rc = lib().orc_intra_predict(_p(c), c.shape[1], c.shape[0], c.shape[1], x0, y0, n, mode,
                                 _p(out))
    if rc != 0:
        raise ValueError("orc_intra_predict: invalid arguments")
    return out


def cu_motion_search(cur, ref, x0, y0, n, R, qp):
    c = np.ascontiguousarray(cur, dtype=np.uint8)
    r = np.ascontiguousarray(ref, dtype=np.uint8)
    assert c.shape == r.shape
    mx, my, sad = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    rc = lib().orc_cu_motion_search(_p(c), _p(r), c.shape[1], c.shape[0], c.shape[1], x0, y0, n,
                                    R, qp, ctypes.byref(mx), ctypes.byref(my), ctypes.byref(sad))
    if rc != 0:
        raise ValueError("orc_cu_motion_search: invalid arguments")
    return mx.value, my.value, sad.value


class Seed:
    """Reference MVs for a seeded search: the [ceil(ref_h/8), ceil(ref_w/8), 2] int16 MV map of
    a ref_w x ref_h search of the same content (quarter-pel units when qpel), and the
    refinement half-width r."""

    def __init__(self, ref_mv, ref_w: int, ref_h: int, r: int, qpel: bool = False):
        self.ref_mv = np.ascontiguousarray(ref_mv, dtype=np.int16)
        assert self.ref_mv.shape == ((ref_h + 7) // 8, (ref_w + 7) // 8, 2)
        self.ref_w, self.ref_h, self.r = int(ref_w), int(ref_h), int(r)
        self.qpel = 1 if qpel else 0

    def args(self):
        return (_p(self.ref_mv), self.ref_w, self.ref_h, self.r, self.qpel)


_NO_SEED = (None, 0, 0, 0, 0)


def mv_centre(seed: Seed, cur_w, cur_h, R, x0, y0, n):
    """Search centre (cx, cy) of the n x n CU at (x0, y0) for a seeded search."""
    cx, cy = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().orc_mv_centre(*seed.args()[:3], cur_w, cur_h, R, seed.r, seed.qpel, x0, y0, n,
                             ctypes.byref(cx), ctypes.byref(cy))
    if rc != 0:
        raise ValueError("orc_mv_centre: invalid arguments")
    return cx.value, cy.value


def ctu_nodes(cur, ref, qp, R, ctu_x, ctu_y, seed: Seed | None = None,
              subpel: bool = False, angular: bool = False) -> np.ndarray:
    """(85, 14) int64 per-node leaf evaluation of one CTU (fields: NODE_FIELDS)."""
    c = np.ascontiguousarray(cur, dtype=np.uint8)
    r = np.ascontiguousarray(ref, dtype=np.uint8)
    rec = np.zeros((85, len(NODE_FIELDS)), dtype=np.int64)
    sa = seed.args() if seed is not None else _NO_SEED
    rc = lib().orc_ctu_nodes(_p(c), _p(r), c.shape[1], c.shape[0], c.shape[1], qp, R,
                             (1 if subpel else 0) | (2 if angular else 0), ctu_x, ctu_y, *sa,
                             _p(rec))
    if rc != 0:
        raise ValueError("orc_ctu_nodes: invalid arguments")
    return rec


def ctu_search(cur, ref, qp, R, bounds=None, ctu_list=None, n_threads=0,
               seed: Seed | None = None, subpel: bool = False, angular: bool = False):
    """Coding-tree search of a frame pair (all CTUs or a listed subset); seeded when ``seed``
    is given; with ``subpel`` the inter MVs are refined to quarter-pel (and output in
    quarter-pel units); with ``angular`` the 33 angular intra modes are searched beside
    planar and DC (mode codes 3..35 = 1 + the H.265 mode).

    Returns a dict of numpy arrays: depth, mode ([H8/8, W8/8] u8), mv ([H8/8, W8/8, 2] i16),
    cost, dist, bits ([ceil(H/64), ceil(W/64)] i64).  Units of CTUs outside the list keep 0.
    """
    c = np.ascontiguousarray(cur, dtype=np.uint8)
    r = np.ascontiguousarray(ref, dtype=np.uint8)
    assert c.shape == r.shape
    H, W = c.shape
    uh, uw = (H + 7) // 8, (W + 7) // 8
    th, tw = (uh * 8 + 63) // 64, (uw * 8 + 63) // 64
    out = dict(depth=np.zeros((uh, uw), np.uint8), mode=np.zeros((uh, uw), np.uint8),
               mv=np.zeros((uh, uw, 2), np.int16), cost=np.zeros((th, tw), np.int64),
               dist=np.zeros((th, tw), np.int64), bits=np.zeros((th, tw), np.int64))
    b = None
    if bounds is not None:
        b = np.ascontiguousarray(bounds, dtype=np.uint8)
        assert b.shape == (uh, uw, 2)
    lst = None
    if ctu_list is not None:
        lst = np.ascontiguousarray(np.asarray(ctu_list, dtype=np.int32))
    sa = seed.args() if seed is not None else _NO_SEED
    rc = lib().orc_ctu_search(_p(c), _p(r), W, H, W, qp, R,
                              (1 if subpel else 0) | (2 if angular else 0), _p(b), *sa,
                              _p(out["depth"]),
                              _p(out["mode"]), _p(out["mv"]), _p(out["cost"]), _p(out["dist"]),
                              _p(out["bits"]), _p(lst), 0 if lst is None else len(lst),
                              n_threads)
    if rc != 0:
        raise ValueError("orc_ctu_search: invalid arguments")
    return out


def depth_bounds(ref_depth, ref_w, ref_h, dep_w, dep_h, delta_lo, delta_hi):
    rd = np.ascontiguousarray(ref_depth, dtype=np.uint8)
    assert rd.shape == ((ref_h + 7) // 8, (ref_w + 7) // 8)
    out = np.zeros(((dep_h + 7) // 8, (dep_w + 7) // 8, 2), np.uint8)
    rc = lib().orc_depth_bounds(_p(rd), ref_w, ref_h, dep_w, dep_h, delta_lo, delta_hi, _p(out))
    if rc != 0:
        raise ValueError("orc_depth_bounds: invalid arguments")
    return out


def interp_qpel(ref, qx: int, qy: int) -> int:
    """Interpolated 8-bit prediction sample at quarter-pel position (qx, qy) of ``ref``."""
    r = np.ascontiguousarray(ref, dtype=np.uint8)
    v = lib().orc_interp_qpel(_p(r), r.shape[1], r.shape[0], r.shape[1], qx, qy)
    if v < 0:
        raise ValueError("orc_interp_qpel: invalid arguments")
    return int(v)


def subpel_refine(cur, ref, x0, y0, n, mx, my, qp):
    """Quarter-pel refinement of the integer MV (mx, my) of one CU: (qx, qy, satd)."""
    c = np.ascontiguousarray(cur, dtype=np.uint8)
    r = np.ascontiguousarray(ref, dtype=np.uint8)
    assert c.shape == r.shape
    qx, qy, sd = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    rc = lib().orc_subpel_refine(_p(c), _p(r), c.shape[1], c.shape[0], c.shape[1], x0, y0, n,
                                 mx, my, qp, ctypes.byref(qx), ctypes.byref(qy), ctypes.byref(sd))
    if rc != 0:
        raise ValueError("orc_subpel_refine: invalid arguments")
    return qx.value, qy.value, sd.value
