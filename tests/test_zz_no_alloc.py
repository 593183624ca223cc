"""The allocation-free search (mr_ctu_search_noalloc) against mr_ctu_search /
mr_ctu_search_seeded, element by element, on calls in a row through the C ABI.

The array it works in is shared by every call on the GPU and keeps the previous call's
contents, so each sequence runs a larger search first and then smaller ones.  Flat and
ramp pictures make many candidates tie on SAD, which exercises the rank order of the key
tables the entry point builds on the device.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("depth", "mode", "mv", "cost", "dist", "bits")


@pytest.fixture(scope="module")
def mr():
    import torch
    from paper_2301_12191_amd import mr as m
    assert torch.cuda.is_available()
    m.lib()
    oracle.build(force=False)
    synth.build(force=False)
    return m


def _pair(w, h, seed, objects=6, mv=12):
    import torch
    sc = synth.Scene(seed, w, h, objects, mv, 2)
    ref, cur = sc.render(0), sc.render(1)
    return ref, cur, torch.from_numpy(ref).cuda(), torch.from_numpy(cur).cuda()


def _run_both(mr, cur, ref, qp, R, bounds=None, seed=None, subpel=False, label=""):
    import torch
    print(f"noalloc vs search: {label} {tuple(cur.shape)} QP {qp} R {R} bounds "
          f"{bounds is not None} seed {seed is not None} subpel {subpel}", flush=True)
    H, W = cur.shape
    exp = mr.mr_ctu_search(cur, ref, qp, R, bounds=bounds, seed=seed, subpel=subpel)
    got = mr.alloc_outputs(W, H)
    for t in got.values():
        t.fill_(0x5A)  # whatever the entry point leaves unwritten shows up
    mr.mr_ctu_search_noalloc(cur, ref, qp, R, got, bounds=bounds, seed=seed, subpel=subpel)
    torch.cuda.synchronize()
    for k in FIELDS:
        assert torch.equal(got[k], exp[k]), f"{label}: {k} differs from the allocating search"
    return {k: v.cpu().numpy() for k, v in got.items()}


def test_noalloc_equals_search_large_then_smaller(mr):
    import torch
    _, _, r1080, c1080 = _pair(1920, 1080, synth.SEED_BASE + 1, 24, 48)
    _run_both(mr, c1080, r1080, 27, 64, label="1080p full")
    ref, cur, r240, c240 = _pair(416, 240, synth.SEED_BASE)
    depth_ref = mr.mr_ctu_search(c240[::2, ::2].contiguous(), r240[::2, ::2].contiguous(), 32,
                                 8)["depth"]
    bounds = mr.mr_depth_bounds(depth_ref, 208, 120, 416, 240, 0, 1)
    got = _run_both(mr, c240, r240, 32, 16, bounds=bounds, label="416x240 bounded")
    exp = oracle.ctu_search(cur, ref, 32, 16, bounds=bounds.cpu().numpy())
    for k in FIELDS:
        assert np.array_equal(got[k], exp[k]), f"416x240 bounded: {k} differs from the oracle"
    torch.cuda.synchronize()


def test_noalloc_seeded_and_subpel_then_smaller(mr):
    ref, cur, r, c = _pair(640, 360, synth.SEED_BASE + 5)
    base = mr.mr_ctu_search(c[::2, ::2].contiguous(), r[::2, ::2].contiguous(), 32, 12)
    seed = dict(ref_mv=base["mv"], ref_w=320, ref_h=180, r=4)
    _run_both(mr, c, r, 30, 24, seed=seed, label="640x360 seeded")
    _run_both(mr, c, r, 30, 24, subpel=True, label="640x360 sub-pel")
    _run_both(mr, c[:136, :200].contiguous(), r[:136, :200].contiguous(), 35, 16, subpel=True,
              seed=dict(ref_mv=base["mv"], ref_w=320, ref_h=180, r=2),
              label="200x136 seeded sub-pel")


@pytest.mark.parametrize("d", [2, 4, 8])
def test_noalloc_tables_with_ties(mr, d):
    """Flat and ramp pictures at each lane shape D: every candidate of a flat pair has the
    same SAD, so the arg-min is decided by MV cost and raster order alone."""
    import torch
    try:
        for R in (24, 7, 0):
            mr.mr_set_tiles(R, d, 1 + R % 3)
        flat = torch.full((200, 264), 97, dtype=torch.uint8, device="cuda")
        ramp = (torch.arange(264, device="cuda", dtype=torch.int32)[None, :] * 3 +
                torch.arange(200, device="cuda", dtype=torch.int32)[:, None]) % 256
        ramp = ramp.to(torch.uint8).contiguous()
        ramp2 = torch.roll(ramp, shifts=(1, -2), dims=(0, 1)).contiguous()
        _run_both(mr, flat, flat, 22, 24, label=f"flat D{d}")
        _run_both(mr, ramp2, ramp, 37, 24, label=f"ramp D{d}")
        _run_both(mr, ramp2[:72, :100].contiguous(), ramp[:72, :100].contiguous(), 51, 7,
                  label=f"ramp small D{d}")
        _run_both(mr, flat[:8, :8].contiguous(), flat[:8, :8].contiguous(), 0, 0,
                  label=f"8x8 R0 D{d}")
    finally:
        for R in (24, 7, 0):
            mr.mr_set_tiles(R, 0, 1)


def test_noalloc_refuses_oversize_without_launch(mr):
    import torch
    big = torch.zeros((4320, 8192), dtype=torch.uint8, device="cuda")
    out = mr.alloc_outputs(8192, 4320)
    with pytest.raises(mr.MRError) as ei:
        mr.mr_ctu_search_noalloc(big, big, 30, 16, out)
    assert ei.value.code == mr.MR_ESCRATCH
    # The array still serves the next call.
    _, _, r, c = _pair(416, 240, synth.SEED_BASE)
    _run_both(mr, c, r, 32, 16, label="after refusal")
