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
MR_ESCRATCH = -8
MR_ECANCELED = -9
# Size of the per-GPU device array of mr_ctu_search_noalloc.
NOALLOC_SCRATCH_BYTES = 24 << 20


class MRError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {mr_status_str(code)} ({code})")


class mr_frame(ctypes.Structure):
    _fields_ = [("luma", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("stride", ctypes.c_int32)]


class mr_search_params(ctypes.Structure):
    _fields_ = [("qp", ctypes.c_int32), ("search_range", ctypes.c_int32),
                ("subpel", ctypes.c_int32), ("angular", ctypes.c_int32)]


class mr_search_out(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("mode", ctypes.c_void_p), ("mv", ctypes.c_void_p),
                ("ctu_cost", ctypes.c_void_p), ("ctu_dist", ctypes.c_void_p),
                ("ctu_bits", ctypes.c_void_p)]


class mr_mv_seed(ctypes.Structure):
    _fields_ = [("ref_mv", ctypes.c_void_p), ("ref_w", ctypes.c_int32), ("ref_h", ctypes.c_int32),
                ("refine_range", ctypes.c_int32), ("quarter_pel", ctypes.c_int32)]


class mr_search_job(ctypes.Structure):
    _fields_ = [("cur", mr_frame), ("ref", mr_frame), ("params", mr_search_params),
                ("bounds", ctypes.c_void_p), ("out", mr_search_out),
                ("seed", ctypes.POINTER(mr_mv_seed))]


class mr_tune_result(ctypes.Structure):
    _fields_ = [("search_range", ctypes.c_int32), ("d", ctypes.c_int32),
                ("nbands", ctypes.c_int32), ("strip", ctypes.c_int32),
                ("search_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("tried", ctypes.c_int32), ("split", ctypes.c_int32)]


class mr_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 4), ("launches", ctypes.c_int64 * 4)]


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
        L.mr_ctu_search_seeded.restype = ctypes.c_int
        L.mr_ctu_search_seeded.argtypes = [ctypes.POINTER(mr_frame), ctypes.POINTER(mr_frame),
                                           ctypes.POINTER(mr_search_params), vp,
                                           ctypes.POINTER(mr_mv_seed),
                                           ctypes.POINTER(mr_search_out), vp]
        L.mr_ctu_search_noalloc.restype = ctypes.c_int
        L.mr_ctu_search_noalloc.argtypes = L.mr_ctu_search_seeded.argtypes
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
        L.mr_set_tiles4.restype = ctypes.c_int
        L.mr_set_tiles4.argtypes = [i32, i32, i32, i32, i32]
        L.mr_set_tiles.restype = ctypes.c_int
        L.mr_set_tiles.argtypes = [i32, i32, i32]
        L.mr_profile_enable.restype = ctypes.c_int
        L.mr_profile_enable.argtypes = [ctypes.c_int]
        L.mr_profile_read.restype = ctypes.c_int
        L.mr_profile_read.argtypes = [ctypes.POINTER(mr_profile), ctypes.c_int]
        L.mr_sqrt_lambda_q16.restype = ctypes.c_int64
        L.mr_sqrt_lambda_q16.argtypes = [i32]
        L.mr_se_bits.restype = ctypes.c_int32
        L.mr_se_bits.argtypes = [i32]
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


def _seed_struct(seed):
    """seed: dict {ref_mv: (ceil(ref_h/8), ceil(ref_w/8), 2) int16 device tensor, ref_w, ref_h,
    r, qpel (optional: the map is in quarter-pel units)}, or None."""
    if seed is None:
        return None
    rm = seed["ref_mv"]
    if rm.dim() != 3 or rm.shape[2] != 2:
        raise ValueError("ref_mv must be (ceil(ref_h/8), ceil(ref_w/8), 2) int16")
    if tuple(rm.shape[:2]) != unit_shape(seed["ref_w"], seed["ref_h"]):
        raise ValueError("ref_mv shape does not match ref_w x ref_h")
    return mr_mv_seed(_dev_ptr(rm, torch.int16, "ref_mv"), seed["ref_w"], seed["ref_h"],
                      seed["r"], 1 if seed.get("qpel") else 0)


def mr_ctu_search(cur: torch.Tensor, ref: torch.Tensor, qp: int, search_range: int,
                  bounds: torch.Tensor | None = None, out: dict | None = None, stream=None,
                  seed: dict | None = None, subpel: bool = False, angular: bool = False):
    """Coding-tree search of one frame pair (see mr_ctu_search and mr_ctu_search_seeded in
    include/mr.h); seeded when ``seed`` is given; with ``subpel`` the MVs are refined to
    quarter-pel and returned in quarter-pel units; with ``angular`` the 33 angular intra
    modes are scored beside planar and DC."""
    H, W = cur.shape
    if out is None:
        out = alloc_outputs(W, H, cur.device)
    fc, fr = _frame(cur, "cur"), _frame(ref, "ref")
    prm = mr_search_params(qp, search_range, 1 if subpel else 0, 1 if angular else 0)
    o = mr_search_out(_dev_ptr(out["depth"], torch.uint8, "depth"),
                      _dev_ptr(out["mode"], torch.uint8, "mode"),
                      _dev_ptr(out["mv"], torch.int16, "mv"),
                      _dev_ptr(out["cost"], torch.int64, "cost"),
                      _dev_ptr(out["dist"], torch.int64, "dist"),
                      _dev_ptr(out["bits"], torch.int64, "bits"))
    bp = None if bounds is None else _dev_ptr(bounds, torch.uint8, "bounds")
    if seed is None:
        rc = lib().mr_ctu_search(ctypes.byref(fc), ctypes.byref(fr), ctypes.byref(prm), bp,
                                 ctypes.byref(o), _stream_handle(stream))
        where = "mr_ctu_search"
    else:
        sd = _seed_struct(seed)
        rc = lib().mr_ctu_search_seeded(ctypes.byref(fc), ctypes.byref(fr), ctypes.byref(prm),
                                        bp, ctypes.byref(sd), ctypes.byref(o),
                                        _stream_handle(stream))
        where = "mr_ctu_search_seeded"
    if rc != MR_OK:
        raise MRError(rc, where)
    return out


def mr_ctu_search_noalloc(cur: torch.Tensor, ref: torch.Tensor, qp: int, search_range: int,
                          out: dict, bounds: torch.Tensor | None = None, stream=None,
                          seed: dict | None = None, subpel: bool = False, angular: bool = False):
    """The allocation-free search (mr_ctu_search_noalloc in include/mr.h): the caller passes
    the outputs; the library allocates nothing.  Same arguments and results as
    mr_ctu_search."""
    fc, fr = _frame(cur, "cur"), _frame(ref, "ref")
    prm = mr_search_params(qp, search_range, 1 if subpel else 0, 1 if angular else 0)
    o = _out_struct(out)
    bp = None if bounds is None else _dev_ptr(bounds, torch.uint8, "bounds")
    sd = _seed_struct(seed)
    rc = lib().mr_ctu_search_noalloc(ctypes.byref(fc), ctypes.byref(fr), ctypes.byref(prm), bp,
                                     None if sd is None else ctypes.byref(sd), ctypes.byref(o),
                                     _stream_handle(stream))
    if rc != MR_OK:
        raise MRError(rc, "mr_ctu_search_noalloc")
    return out


def _out_struct(out):
    return mr_search_out(_dev_ptr(out["depth"], torch.uint8, "depth"),
                         _dev_ptr(out["mode"], torch.uint8, "mode"),
                         _dev_ptr(out["mv"], torch.int16, "mv"),
                         _dev_ptr(out["cost"], torch.int64, "cost"),
                         _dev_ptr(out["dist"], torch.int64, "dist"),
                         _dev_ptr(out["bits"], torch.int64, "bits"))


def _job_array(jobs):
    """jobs: list of dicts {cur, ref, qp, search_range, bounds (optional), out (optional),
    seed (optional, as for mr_ctu_search)}."""
    arr = (mr_search_job * len(jobs))()
    arr._seeds = []  # keep the seed structs alive with the array
    for i, j in enumerate(jobs):
        cur = j["cur"]
        if j.get("out") is None:
            j["out"] = alloc_outputs(cur.shape[1], cur.shape[0], cur.device)
        b = j.get("bounds")
        sd = _seed_struct(j.get("seed"))
        sp = None
        if sd is not None:
            arr._seeds.append(sd)
            sp = ctypes.pointer(sd)
        arr[i] = mr_search_job(_frame(cur, "cur"), _frame(j["ref"], "ref"),
                               mr_search_params(j["qp"], j["search_range"],
                                                1 if j.get("subpel") else 0,
                                                1 if j.get("angular") else 0),
                               None if b is None else _dev_ptr(b, torch.uint8, "bounds"),
                               _out_struct(j["out"]), sp)
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


STAGES = ("prep", "search", "subpel", "leaf")


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


def mr_set_tiles4(search_range: int, d: int, nbands: int, strip: int, split: int) -> None:
    rc = lib().mr_set_tiles4(search_range, d, nbands, strip, split)
    if rc != MR_OK:
        raise MRError(rc, "mr_set_tiles4")


def mr_autotune(jobs, reps: int = 3) -> dict:
    """Tune the search tile shape on a batch (see mr_autotune in include/mr.h)."""
    arr = _job_array(jobs)
    res = mr_tune_result()
    rc = lib().mr_autotune(arr, len(jobs), reps, ctypes.byref(res))
    if rc != MR_OK:
        raise MRError(rc, "mr_autotune")
    return {f: getattr(res, f) for f, _ in mr_tune_result._fields_}


# ------------------------------------------------------------------ ladder server
MR_MAX_RUNGS = 16


class mr_rung(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("qp", ctypes.c_int32),
                ("search_range", ctypes.c_int32), ("ref_rung", ctypes.c_int32),
                ("subpel", ctypes.c_int32), ("own_policy", ctypes.c_int32), ("delta_lo", ctypes.c_int32),
                ("delta_hi", ctypes.c_int32), ("reuse_mv", ctypes.c_int32),
                ("refine_range", ctypes.c_int32), ("angular", ctypes.c_int32)]


class mr_ladder_config(ctypes.Structure):
    _fields_ = [("n_rungs", ctypes.c_int32), ("rungs", mr_rung * MR_MAX_RUNGS),
                ("delta_lo", ctypes.c_int32),
                ("delta_hi", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("max_inflight", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("max_batch_jobs", ctypes.c_int32), ("reuse_mv", ctypes.c_int32),
                ("refine_range", ctypes.c_int32), ("job_timeout_us", ctypes.c_int32)]


class mr_job(ctypes.Structure):
    _fields_ = [("stream_id", ctypes.c_int32), ("frame_idx", ctypes.c_int32),
                ("rung", ctypes.c_int32)]


class mr_completion(ctypes.Structure):
    _fields_ = [("job_id", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("stream_id", ctypes.c_int32), ("frame_idx", ctypes.c_int32),
                ("rung", ctypes.c_int32), ("implied", ctypes.c_int32), ("n_ctus", ctypes.c_int32),
                ("t_arrive_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("out", mr_search_out)]


class mr_ladder_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("implied", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("ctus_done", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("ctus_per_s", ctypes.c_double),
                ("bytes_in_use", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("cancelled", ctypes.c_int64), ("timed_out", ctypes.c_int64),
                ("cached_bytes", ctypes.c_uint64), ("host_launch_ms", ctypes.c_double),
                ("device_allocs", ctypes.c_int64)]


def _ladder_lib():
    L = lib()
    if not getattr(L, "_ladder_bound", False):
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        L.mr_ladder_open.argtypes = [ctypes.POINTER(mr_ladder_config), ctypes.POINTER(vp)]
        L.mr_ladder_put_frame.argtypes = [vp, i32, i32, i32, vp, i32]
        L.mr_ladder_drop_frames.argtypes = [vp, i32, i32]
        L.mr_ladder_submit.argtypes = [vp, ctypes.POINTER(mr_job), ctypes.POINTER(ctypes.c_uint64)]
        L.mr_ladder_submit_many.argtypes = [vp, ctypes.POINTER(mr_job), i32,
                                            ctypes.POINTER(ctypes.c_uint64),
                                            ctypes.POINTER(i32)]
        L.mr_ladder_poll.argtypes = [vp, ctypes.POINTER(mr_completion), i32, i32,
                                     ctypes.POINTER(i32)]
        L.mr_ladder_release.argtypes = [vp, ctypes.c_uint64]
        L.mr_ladder_release_many.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), i32,
                                             ctypes.POINTER(i32)]
        L.mr_ladder_cancel.argtypes = [vp, ctypes.c_uint64]
        L.mr_ladder_get_stats.argtypes = [vp, ctypes.POINTER(mr_ladder_stats)]
        L.mr_ladder_close.argtypes = [vp]
        for f in ("mr_ladder_open", "mr_ladder_put_frame", "mr_ladder_drop_frames",
                  "mr_ladder_submit", "mr_ladder_submit_many", "mr_ladder_poll",
                  "mr_ladder_release", "mr_ladder_release_many", "mr_ladder_cancel",
                  "mr_ladder_get_stats",
                  "mr_ladder_close"):
            getattr(L, f).restype = ctypes.c_int
        L._ladder_bound = True
    return L


def _tensor_view(ptr, shape, dtype, device):
    """Non-owning torch view of ladder-owned device memory (valid until release)."""
    n = torch.empty((), dtype=dtype).element_size()
    for d in shape:
        n *= d

    class _Holder:
        __cuda_array_interface__ = {"shape": (n,), "typestr": "|u1", "data": (ptr, False),
                                    "version": 2}
    return torch.as_tensor(_Holder(), device=device).view(dtype).view(shape)


class _PreparedJobs:
    """A submission's argument array (see Ladder.prepare)."""
    __slots__ = ("arr", "n")

    def __init__(self, arr, n):
        self.arr, self.n = arr, n


class Ladder:
    """mr_ladder_* handle: continuous-batching server of ladder frame-pair jobs."""

    def __init__(self, rungs, delta_lo=0, delta_hi=1, budget_bytes=8 << 30, max_inflight=256,
                 max_queue=8192, max_batch_jobs=64, refine_range=None, job_timeout_us=0):
        L = _ladder_lib()
        cfg = mr_ladder_config()
        if not 1 <= len(rungs) <= MR_MAX_RUNGS:
            raise ValueError(f"1..{MR_MAX_RUNGS} rungs")
        cfg.n_rungs = len(rungs)
        for i, r in enumerate(rungs):
            # A rung dict with any of delta_lo / delta_hi / refine_range carries its own policy
            # (refine_range None or absent: not seeded); otherwise the ladder-wide one applies.
            own = any(k in r for k in ("delta_lo", "delta_hi", "refine_range"))
            rr = r.get("refine_range")
            cfg.rungs[i] = mr_rung(r["width"], r["height"], r["qp"], r["search_range"],
                                   r.get("ref_rung", -1), 1 if r.get("subpel") else 0,
                                   1 if own else 0, r.get("delta_lo", 0),
                                   r.get("delta_hi", 1), 0 if rr is None else 1,
                                   0 if rr is None else rr, 1 if r.get("angular") else 0)
        cfg.delta_lo, cfg.delta_hi = delta_lo, delta_hi
        cfg.hbm_budget_bytes = budget_bytes
        cfg.max_inflight, cfg.max_queue, cfg.max_batch_jobs = max_inflight, max_queue, max_batch_jobs
        # refine_range None: dependents run the bounded full search; an int r seeds them with
        # their reference job's MVs (refinement half-width r).
        cfg.reuse_mv = 0 if refine_range is None else 1
        cfg.refine_range = 0 if refine_range is None else refine_range
        cfg.job_timeout_us = job_timeout_us
        self.rungs = rungs
        self._h = ctypes.c_void_p()
        self._frames = {}
        rc = L.mr_ladder_open(ctypes.byref(cfg), ctypes.byref(self._h))
        if rc != MR_OK:
            raise MRError(rc, "mr_ladder_open")

    def put_frame(self, stream_id, frame_idx, rung, luma: torch.Tensor):
        self._frames[(stream_id, frame_idx, rung)] = luma  # keep resident
        rc = _ladder_lib().mr_ladder_put_frame(self._h, stream_id, frame_idx, rung,
                                               _dev_ptr(luma, torch.uint8, "luma"), luma.stride(0))
        if rc != MR_OK:
            raise MRError(rc, "mr_ladder_put_frame")

    def drop_frames(self, stream_id, before_frame):
        """Forget the frames of a stream before `before_frame` and stop keeping their tensors
        alive.  Jobs that read those frames must have completed (a job not yet started fails
        with MR_EDEPEND instead)."""
        rc = _ladder_lib().mr_ladder_drop_frames(self._h, stream_id, before_frame)
        if rc != MR_OK:
            raise MRError(rc, "mr_ladder_drop_frames")
        for key in [k for k in self._frames if k[0] == stream_id and k[1] < before_frame]:
            del self._frames[key]

    def submit(self, stream_id, frame_idx, rung) -> int:
        jid = ctypes.c_uint64()
        rc = _ladder_lib().mr_ladder_submit(self._h, ctypes.byref(mr_job(stream_id, frame_idx, rung)),
                                            ctypes.byref(jid))
        if rc != MR_OK:
            raise MRError(rc, "mr_ladder_submit")
        return jid.value

    @staticmethod
    def prepare(jobs):
        """The argument array of a later submit_many, built ahead of time (a client that
        submits the next frame's jobs the moment the last one completes builds them before)."""
        jobs = list(jobs)
        return _PreparedJobs((mr_job * max(len(jobs), 1))(*[mr_job(s, f, r) for s, f, r in jobs]),
                             len(jobs))

    def submit_many(self, jobs) -> list:
        """jobs: (stream_id, frame_idx, rung) tuples, or the result of prepare(), submitted
        together in order. On a refusal raises MRError whose `submitted` holds the ids of the
        jobs accepted before it."""
        if isinstance(jobs, _PreparedJobs):
            arr, n = jobs.arr, jobs.n
        else:
            jobs = list(jobs)
            n = len(jobs)
            arr = (mr_job * max(n, 1))(*[mr_job(s, f, r) for s, f, r in jobs])
        ids = (ctypes.c_uint64 * max(n, 1))()
        done = ctypes.c_int32()
        rc = _ladder_lib().mr_ladder_submit_many(self._h, arr, n, ids, ctypes.byref(done))
        got = [ids[i] for i in range(done.value)]
        if rc != MR_OK:
            err = MRError(rc, "mr_ladder_submit_many")
            err.submitted = got
            raise err
        return got

    def poll(self, max_n=64, timeout_us=0):
        arr = (mr_completion * max_n)()
        n = ctypes.c_int32()
        rc = _ladder_lib().mr_ladder_poll(self._h, arr, max_n, timeout_us, ctypes.byref(n))
        if rc == MR_ETIMEOUT:
            return []
        if rc != MR_OK:
            raise MRError(rc, "mr_ladder_poll")
        return [arr[i] for i in range(n.value)]

    def outputs(self, c, device="cuda"):
        """torch views of a completion's device outputs (valid until release)."""
        r = self.rungs[c.rung]
        uh, uw = unit_shape(r["width"], r["height"])
        th, tw = ctu_shape(r["width"], r["height"])
        return dict(depth=_tensor_view(c.out.depth, (uh, uw), torch.uint8, device),
                    mode=_tensor_view(c.out.mode, (uh, uw), torch.uint8, device),
                    mv=_tensor_view(c.out.mv, (uh, uw, 2), torch.int16, device),
                    cost=_tensor_view(c.out.ctu_cost, (th, tw), torch.int64, device),
                    dist=_tensor_view(c.out.ctu_dist, (th, tw), torch.int64, device),
                    bits=_tensor_view(c.out.ctu_bits, (th, tw), torch.int64, device))

    def cancel(self, job_id):
        """Cancel a job not launched yet (MRError with MR_ESTATE once it has been)."""
        rc = _ladder_lib().mr_ladder_cancel(self._h, job_id)
        if rc != MR_OK:
            raise MRError(rc, "mr_ladder_cancel")

    def release(self, job_id):
        rc = _ladder_lib().mr_ladder_release(self._h, job_id)
        if rc != MR_OK:
            raise MRError(rc, "mr_ladder_release")

    def release_many(self, job_ids):
        """Release several completed jobs in one call (stops at the first failure)."""
        ids = list(job_ids)
        if not ids:
            return
        arr = (ctypes.c_uint64 * len(ids))(*ids)
        n = ctypes.c_int32(0)
        rc = _ladder_lib().mr_ladder_release_many(self._h, arr, len(ids), ctypes.byref(n))
        if rc != MR_OK:
            raise MRError(rc, f"mr_ladder_release_many (released {n.value} of {len(ids)})")

    def stats(self) -> dict:
        s = mr_ladder_stats()
        rc = _ladder_lib().mr_ladder_get_stats(self._h, ctypes.byref(s))
        if rc != MR_OK:
            raise MRError(rc, "mr_ladder_get_stats")
        return {f: getattr(s, f) for f, _ in mr_ladder_stats._fields_}

    def close(self):
        if self._h:
            rc = _ladder_lib().mr_ladder_close(self._h)
            self._h = ctypes.c_void_p()
            if rc != MR_OK:
                raise MRError(rc, "mr_ladder_close")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
