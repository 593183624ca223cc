"""GPU parity of the angular intra modes (mr_search_params.angular = 1) against the oracle,
element by element: ragged pictures (edge nodes, neighbour substitution at every border),
bounds, seeded and sub-pel searches, flat content (every mode ties), and a batch that mixes
angular and plain jobs."""
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


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _cmp(got, exp, label):
    for k in FIELDS:
        g = got[k].cpu().numpy() if hasattr(got[k], "cpu") else got[k]
        assert np.array_equal(g, exp[k]), f"{label}: {k}"


@pytest.mark.parametrize("W,H,qp,R", [(200, 136, 37, 8), (136, 72, 22, 4), (64, 64, 30, 2),
                                      (72, 40, 45, 3), (5, 3, 32, 1), (1, 1, 12, 0),
                                      (264, 200, 27, 6)])
def test_angular_search_bit_exact(mr, W, H, qp, R):
    import torch
    sc = synth.Scene(0x7100 + W + H, W, H, 5, max(2, R), 1)
    ref, cur = sc.render(0), sc.render(1)
    print(f"\nangular {W}x{H} QP {qp} R {R}", flush=True)
    got = mr.mr_ctu_search(_dev(cur), _dev(ref), qp, R, angular=True)
    torch.cuda.synchronize()
    exp = oracle.ctu_search(cur, ref, qp, R, angular=True)
    _cmp(got, exp, f"{W}x{H}")
    if W * H > 64:
        assert exp["mode"].max() >= 3  # some CUs pick angular modes


def test_angular_with_bounds_seed_and_subpel(mr):
    import torch
    W, H, qp, R = 200, 136, 33, 8
    sc = synth.Scene(0x7200, W, H, 6, 8, 2)
    ref, cur = sc.render(0), sc.render(1)
    rng = np.random.default_rng(3)
    lo = rng.integers(0, 4, size=((H + 7) // 8, (W + 7) // 8), dtype=np.uint8)
    hi = np.maximum(lo, rng.integers(0, 4, size=lo.shape, dtype=np.uint8))
    b = np.stack([lo, hi], axis=-1)
    small = (cur[::2, ::2].copy(), ref[::2, ::2].copy())
    base = oracle.ctu_search(small[0], small[1], qp, 4)
    for label, kw_gpu, kw_orc in (
            ("bounds", dict(bounds=_dev(b)), dict(bounds=b)),
            ("seed", dict(seed=dict(ref_mv=_dev(base["mv"]), ref_w=100, ref_h=68, r=2)),
             dict(seed=oracle.Seed(base["mv"], 100, 68, 2))),
            ("subpel", dict(subpel=True), dict(subpel=True))):
        print(f"angular + {label}", flush=True)
        got = mr.mr_ctu_search(_dev(cur), _dev(ref), qp, R, angular=True, **kw_gpu)
        torch.cuda.synchronize()
        _cmp(got, oracle.ctu_search(cur, ref, qp, R, angular=True, **kw_orc), label)


def test_flat_and_ramp_pictures(mr):
    """Flat content: all intra predictions equal, so planar wins every intra tie; ramps
    favour particular directions."""
    import torch
    flat = np.full((72, 136), 90, np.uint8)
    yy, xx = np.mgrid[0:72, 0:136]
    ramp = ((3 * xx + yy) % 256).astype(np.uint8)
    diag = ((xx - 2 * yy) % 97 + 60).astype(np.uint8)
    for name, cur, ref in (("flat", flat, flat), ("ramp", ramp, np.roll(ramp, 1, axis=1)),
                           ("diag", diag, np.roll(diag, 2, axis=0))):
        for qp in (12, 40):
            got = mr.mr_ctu_search(_dev(cur), _dev(ref), qp, 2, angular=True)
            torch.cuda.synchronize()
            _cmp(got, oracle.ctu_search(cur, ref, qp, 2, angular=True), f"{name} QP {qp}")


def test_batch_mixes_angular_and_plain_jobs(mr):
    import torch
    jobs, host = [], []
    for i, (W, H, R, ang) in enumerate(((200, 136, 8, True), (136, 72, 4, False),
                                        (72, 40, 2, True), (200, 136, 8, False))):
        sc = synth.Scene(0x7300 + i, W, H, 5, R, 1)
        ref, cur = sc.render(0), sc.render(1)
        host.append((cur, ref, R, ang))
        jobs.append(dict(cur=_dev(cur), ref=_dev(ref), qp=30 + i, search_range=R, angular=ang))
    outs = mr.mr_ctu_search_batch(jobs)
    torch.cuda.synchronize()
    for i, ((cur, ref, R, ang), o) in enumerate(zip(host, outs)):
        _cmp(o, oracle.ctu_search(cur, ref, 30 + i, R, angular=ang), f"job {i}")
