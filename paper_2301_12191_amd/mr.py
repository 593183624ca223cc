"""Thin Python binding of libmr (include/mr.h): argument marshalling only.

Every step of the coding-tree search runs in the HIP kernels of libmr.so; this
module turns torch device tensors into the plain pointers, sizes and stream
handle the C ABI takes.  There is no fallback: if libmr.so is missing or the
device is not a GPU, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmr.so")
_lib = None

MR_OK, MR_EINVAL, MR_ENOMEM, MR_EAGAIN, MR_EDEPEND, MR_EHIP, MR_ETIMEOUT, MR_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)


class MRError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {mr_status_str(code)} ({code})")


class mr_frame(ctypes.Structure):
    _fields_ = [("luma", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("stride", ctypes.c_int32)]


class mr_search_params(ctypes.Structure):
    _fields_ = [("qp", ctypes.c_int32), ("search_range", ctypes.c_int32)]


class mr_search_out(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("mode", ctypes.c_void_p), ("mv", ctypes.c_void_p),
                ("ctu_cost", ctypes.c_void_p), ("ctu_dist", ctypes.c_void_p),
                ("ctu_bits", ctypes.c_void_p)]


class mr_search_job(ctypes.Structure):
    _fields_ = [("cur", mr_frame), ("ref", mr_frame), ("params", mr_search_params),
                ("bounds", ctypes.c_void_p), ("out", mr_search_out)]


class mr_tune_result(ctypes.Structure):
    _fields_ = [("search_range", ctypes.c_int32), ("d", ctypes.c_int32),
                ("nbands", ctypes.c_int32), ("strip", ctypes.c_int32),
                ("search_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("tried", ctypes.c_int32)]


class mr_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 3), ("launches", ctypes.c_int64 * 3)]


def lib():
    """Load libmr.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libmr.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        L.mr_status_str.restype = ctypes.c_char_p
        L.mr_status_str.argtypes = [ctypes.c_int]
        L.mr_ctu_search.restype = ctypes.c_int
        L.mr_ctu_search.argtypes = [ctypes.POINTER(mr_frame), ctypes.POINTER(mr_frame),
                                    ctypes.POINTER(mr_search_params), vp,
                                    ctypes.POINTER(mr_search_out), vp]
        L.mr_depth_bounds.restype = ctypes.c_int
        L.mr_depth_bounds.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp]
        L.mr_ctu_search_batch.restype = ctypes.c_int
        L.mr_ctu_search_batch.argtypes = [ctypes.POINTER(mr_search_job), i32, vp]
        L.mr_batch_create.restype = ctypes.c_int
        L.mr_batch_create.argtypes = [ctypes.POINTER(mr_search_job), i32, ctypes.POINTER(vp)]
        L.mr_batch_set_jobs.restype = ctypes.c_int
        L.mr_batch_set_jobs.argtypes = [vp, ctypes.POINTER(mr_search_job), i32]
        L.mr_batch_launch.restype = ctypes.c_int
        L.mr_batch_launch.argtypes = [vp, vp]
        L.mr_batch_destroy.restype = ctypes.c_int
        L.mr_batch_destroy.argtypes = [vp]
        L.mr_autotune.restype = ctypes.c_int
        L.mr_autotune.argtypes = [ctypes.POINTER(mr_search_job), i32, i32,
                                  ctypes.POINTER(mr_tune_result)]
        L.mr_set_tiles3.restype = ctypes.c_int
        L.mr_set_tiles3.argtypes = [i32, i32, i32, i32]
        L.mr_set_tiles.restype = ctypes.c_int
        L.mr_set_tiles.argtypes = [i32, i32, i32]
        L.mr_profile_enable.restype = ctypes.c_int
        L.mr_profile_enable.argtypes = [ctypes.c_int]
        L.mr_profile_read.restype = ctypes.c_int
        L.mr_profile_read.argtypes = [ctypes.POINTER(mr_profile), ctypes.c_int]
        _lib = L
    return _lib


def mr_status_str(code: int) -> str:
    return lib().mr_status_str(code).decode()


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def unit_shape(width: int, height: int):
    return (height + 7) // 8, (width + 7) // 8


def ctu_shape(width: int, height: int):
    uh, uw = unit_shape(width, height)
    return (uh * 8 + 63) // 64, (uw * 8 + 63) // 64


def alloc_outputs(width: int, height: int, device="cuda"):
    """Caller-owned output buffers of mr_ctu_search for a width x height picture."""
    uh, uw = unit_shape(width, height)
    th, tw = ctu_shape(width, height)
    return dict(depth=torch.empty((uh, uw), dtype=torch.uint8, device=device),
                mode=torch.empty((uh, uw), dtype=torch.uint8, device=device),
                mv=torch.empty((uh, uw, 2), dtype=torch.int16, device=device),
                cost=torch.empty((th, tw), dtype=torch.int64, device=device),
                dist=torch.empty((th, tw), dtype=torch.int64, device=device),
                bits=torch.empty((th, tw), dtype=torch.int64, device=device))


def _frame(t: torch.Tensor, name):
    if t.dim() != 2:
        raise ValueError(f"{name} must be (H, W) uint8")
    return mr_frame(_dev_ptr(t, torch.uint8, name), t.shape[1], t.shape[0], t.stride(0))


def mr_ctu_search(cur: torch.Tensor, ref: torch.Tensor, qp: int, search_range: int,
                  bounds: torch.Tensor | None = None, out: dict | None = None, stream=None):
    """Coding-tree search of one frame pair (see mr_ctu_search in include/mr.h)."""
    H, W = cur.shape
    if out is None:
        out = alloc_outputs(W, H, cur.device)
    fc, fr = _frame(cur, "cur"), _frame(ref, "ref")
    prm = mr_search_params(qp, search_range)
    o = mr_search_out(_dev_ptr(out["depth"], torch.uint8, "depth"),
                      _dev_ptr(out["mode"], torch.uint8, "mode"),
                      _dev_ptr(out["mv"], torch.int16, "mv"),
                      _dev_ptr(out["cost"], torch.int64, "cost"),
                      _dev_ptr(out["dist"], torch.int64, "dist"),
                      _dev_ptr(out["bits"], torch.int64, "bits"))
    bp = None if bounds is None else _dev_ptr(bounds, torch.uint8, "bounds")
    rc = lib().mr_ctu_search(ctypes.byref(fc), ctypes.byref(fr), ctypes.byref(prm), bp,
                             ctypes.byref(o), _stream_handle(stream))
    if rc != MR_OK:
        raise MRError(rc, "mr_ctu_search")
    return out


def _out_struct(out):
    return mr_search_out(_dev_ptr(out["depth"], torch.uint8, "depth"),
                         _dev_ptr(out["mode"], torch.uint8, "mode"),
                         _dev_ptr(out["mv"], torch.int16, "mv"),
                         _dev_ptr(out["cost"], torch.int64, "cost"),
                         _dev_ptr(out["dist"], torch.int64, "dist"),
                         _dev_ptr(out["bits"], torch.int64, "bits"))


def _job_array(jobs):
    """jobs: list of dicts {cur, ref, qp, search_range, bounds (optional), out (optional)}."""
    arr = (mr_search_job * len(jobs))()
    for i, j in enumerate(jobs):
        cur = j["cur"]
        if j.get("out") is None:
            j["out"] = alloc_outputs(cur.shape[1], cur.shape[0], cur.device)
        b = j.get("bounds")
        arr[i] = mr_search_job(_frame(cur, "cur"), _frame(j["ref"], "ref"),
                               mr_search_params(j["qp"], j["search_range"]),
                               None if b is None else _dev_ptr(b, torch.uint8, "bounds"),
                               _out_struct(j["out"]))
    return arr


def mr_ctu_search_batch(jobs, stream=None):
    """Batched search (see mr_ctu_search_batch in include/mr.h); fills each job's "out"."""
    arr = _job_array(jobs)
    rc = lib().mr_ctu_search_batch(arr, len(jobs), _stream_handle(stream))
    if rc != MR_OK:
        raise MRError(rc, "mr_ctu_search_batch")
    return [j["out"] for j in jobs]


class Batch:
    """mr_batch_* handle: planned once, replayed as a captured graph."""

    def __init__(self, jobs):
        self._h = ctypes.c_void_p()
        self.jobs = jobs
        arr = _job_array(jobs)
        rc = lib().mr_batch_create(arr, len(jobs), ctypes.byref(self._h))
        if rc != MR_OK:
            raise MRError(rc, "mr_batch_create")

    def set_jobs(self, jobs):
        arr = _job_array(jobs)
        rc = lib().mr_batch_set_jobs(self._h, arr, len(jobs))
        if rc != MR_OK:
            raise MRError(rc, "mr_batch_set_jobs")
        self.jobs = jobs

    def launch(self, stream=None):
        rc = lib().mr_batch_launch(self._h, _stream_handle(stream))
        if rc != MR_OK:
            raise MRError(rc, "mr_batch_launch")
        return [j["out"] for j in self.jobs]

    def close(self):
        if self._h:
            rc = lib().mr_batch_destroy(self._h)
            self._h = ctypes.c_void_p()
            if rc != MR_OK:
                raise MRError(rc, "mr_batch_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mr_depth_bounds(ref_depth: torch.Tensor, ref_w: int, ref_h: int, dep_w: int, dep_h: int,
                    delta_lo: int, delta_hi: int, out: torch.Tensor | None = None, stream=None):
    """Depth bounds of a dependent representation (see mr_depth_bounds in include/mr.h)."""
    if out is None:
        uh, uw = unit_shape(dep_w, dep_h)
        out = torch.empty((uh, uw, 2), dtype=torch.uint8, device=ref_depth.device)
    rc = lib().mr_depth_bounds(_dev_ptr(ref_depth, torch.uint8, "ref_depth"), ref_w, ref_h,
                               dep_w, dep_h, delta_lo, delta_hi,
                               _dev_ptr(out, torch.uint8, "bounds_out"), _stream_handle(stream))
    if rc != MR_OK:
        raise MRError(rc, "mr_depth_bounds")
    return out


STAGES = ("prep", "search", "leaf")


def mr_profile_enable(on: bool) -> None:
    rc = lib().mr_profile_enable(1 if on else 0)
    if rc != MR_OK:
        raise MRError(rc, "mr_profile_enable")


def mr_profile_read(reset: bool = True) -> dict:
    """{stage: (total_ms, launches)} of the calls made while profiling was enabled."""
    p = mr_profile()
    rc = lib().mr_profile_read(ctypes.byref(p), 1 if reset else 0)
    if rc != MR_OK:
        raise MRError(rc, "mr_profile_read")
    return {name: (p.ms[i], p.launches[i]) for i, name in enumerate(STAGES)}


def mr_set_tiles(search_range: int, d: int, nbands: int = 1) -> None:
    """Override the search kernel's tile choice for one search range (d = 0 clears)."""
    rc = lib().mr_set_tiles(search_range, d, nbands)
    if rc != MR_OK:
        raise MRError(rc, "mr_set_tiles")


def mr_set_tiles3(search_range: int, d: int, nbands: int, strip: int) -> None:
    rc = lib().mr_set_tiles3(search_range, d, nbands, strip)
    if rc != MR_OK:
        raise MRError(rc, "mr_set_tiles3")


def mr_autotune(jobs, reps: int = 3) -> dict:
    """Tune the search tile shape on a batch (see mr_autotune in include/mr.h)."""
    arr = _job_array(jobs)
    res = mr_tune_result()
    rc = lib().mr_autotune(arr, len(jobs), reps, ctypes.byref(res))
    if rc != MR_OK:
        raise MRError(rc, "mr_autotune")
    return {f: getattr(res, f) for f, _ in mr_tune_result._fields_}
