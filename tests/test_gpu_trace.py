"""GPU ray tracing (gbs_trace through the C ABI) against the per-ray oracle
tracer: every array of the table identical, bit for bit (the tracer's
arithmetic is IEEE double without fused multiply-adds on both sides, so the
hit decisions, face ids and CSR offsets are exact and the doubles equal).

Cases: a panelled 3 x 3 city, the 10 x 10 city of the full-size workload,
the open plane with image completion, several ragged sources in one fan,
degenerate fans (no rays, axis-aligned rays, no reflections), the full
1,000,000-ray city with 1,000 sampled rays re-traced by the oracle, and the
traced table fed to the beam summation against the oracle end to end.
"""
import types

import numpy as np
import pytest
import torch

import paper_2501_13382_amd as gbs
from oracle import tracer as ot
from paper_2501_13382_amd import _lib
from scenes import fibonacci_fan, grid_city, receiver_grid
from tests.gpu_util import assert_within, compare, oracle_threads

pytestmark = pytest.mark.gpu

KEYS = ("ray_ptr", "seg_a", "seg_t", "seg_s0", "seg_lo", "seg_hi", "face_ptr", "face_ids")


def gpu_trace(src, d, w, **kw):
    t = gbs.trace(src, d, w, **kw)
    torch.cuda.synchronize()
    return {k: getattr(t, k).cpu().numpy() for k in KEYS}, t


def assert_same(ref, got):
    for k in KEYS:
        a, b = np.asarray(ref[k]), np.asarray(got[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        if not np.array_equal(a, b):
            rows = np.flatnonzero((a != b).reshape(len(a), -1).any(axis=1))
            raise AssertionError(f"{k}: {len(rows)} rows differ, first {rows[:5]}")


def test_panelled_city_bit_exact():
    city = grid_city(3, 40.0, 20.0, 10.0, 40.0, seed=11, panels=2)
    src = np.array([[50.0, 50.0, 6.0]])
    d, w = fibonacci_fan(3000)
    print("case trace panelled 3x3 city, 3000 rays", flush=True)
    ref = ot.trace(src, d, w, boxes=city.boxes, panels=2, s_max=500.0, max_refl=6)
    got, t = gpu_trace(src, d, w, boxes=city.boxes, panels=2, s_max=500.0, max_refl=6)
    assert_same(ref, got)
    assert t.n_faces == 1 + 9 * 20 and len(np.unique(got["face_ids"])) > 30


def test_city_10x10_bit_exact():
    city = grid_city(10, 40.0, 20.0, 10.0, 60.0, seed=1)
    src = np.array([[310.0, 310.0, 5.0]])
    d, w = fibonacci_fan(2500)
    print("case trace 10x10 city, 2500 rays", flush=True)
    ref = ot.trace(src, d, w, boxes=city.boxes, s_max=876.8, max_refl=10)
    got, _ = gpu_trace(src, d, w, boxes=city.boxes, s_max=876.8, max_refl=10)
    assert_same(ref, got)
    assert np.diff(got["ray_ptr"]).max() >= 8          # long reflection chains occur


def test_open_plane_image_completion_bit_exact():
    d, w = fibonacci_fan(2000)
    src = np.array([[0.0, 0.0, 10.0]])
    print("case trace open plane EC", flush=True)
    ref = ot.trace(src, d, w, s_max=170.3, max_refl=1, image_complete=True)
    got, _ = gpu_trace(src, d, w, s_max=170.3, max_refl=1, image_complete=True)
    assert_same(ref, got)
    assert np.all(np.diff(got["ray_ptr"]) == 2)


def test_several_sources_ragged_bit_exact():
    city = grid_city(4, 40.0, 20.0, 10.0, 60.0, seed=5)
    src = np.array([[30.0, 30.0, 3.0], [150.0, 90.0, 12.0], [200.0, 230.0, 25.0]])
    fans = [fibonacci_fan(n) for n in (500, 1700, 900)]
    d = np.concatenate([f[0] for f in fans])
    w = np.concatenate([f[1] for f in fans])
    rs = np.repeat(np.arange(3, dtype=np.int32), [500, 1700, 900])
    print("case trace 3 ragged sources", flush=True)
    ref = ot.trace(src, d, w, ray_src=rs, boxes=city.boxes, s_max=600.0, max_refl=8)
    got, t = gpu_trace(src, d, w, ray_src=rs, boxes=city.boxes, s_max=600.0, max_refl=8)
    assert_same(ref, got)
    assert t.n_src == 3 and torch.equal(t.ray_src.cpu(), torch.as_tensor(rs))


def test_sources_with_their_own_budget_bit_exact():
    """Per-source arc-length budgets (the batched city gives every source its own s_max)."""
    city = grid_city(4, 40.0, 20.0, 10.0, 60.0, seed=5)
    src = np.array([[30.0, 30.0, 3.0], [150.0, 90.0, 12.0], [200.0, 230.0, 25.0]])
    s_max = np.array([250.0, 600.0, 410.0])
    fans = [fibonacci_fan(n) for n in (700, 1200, 900)]
    d = np.concatenate([f[0] for f in fans])
    w = np.concatenate([f[1] for f in fans])
    rs = np.repeat(np.arange(3, dtype=np.int32), [700, 1200, 900])
    print("case trace per-source budgets", flush=True)
    ref = ot.trace(src, d, w, ray_src=rs, boxes=city.boxes, s_max=s_max, max_refl=8)
    got, _ = gpu_trace(src, d, w, ray_src=rs, boxes=city.boxes, s_max=s_max, max_refl=8)
    assert_same(ref, got)
    last = got["ray_ptr"][1:] - 1                       # every path ends at its source's budget
    np.testing.assert_allclose(got["seg_s0"][last] + got["seg_hi"][last], s_max[rs], rtol=1e-12)
    with pytest.raises(_lib.GbsError):
        gbs.trace(src, d, w, ray_src=rs, boxes=city.boxes, s_max=np.array([250.0, -1.0, 400.0]))
    with pytest.raises(ValueError):
        gbs.trace(src, d, w, ray_src=rs, boxes=city.boxes, s_max=np.array([250.0, 300.0]))


def test_degenerate_fans():
    city = grid_city(2, 40.0, 20.0, 10.0, 30.0, seed=7)
    src = np.array([[40.0, 40.0, 5.0]])
    axes = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0], [0, 0, 1.0], [0, 0, -1.0]])
    print("case trace degenerate fans", flush=True)
    for max_refl in (0, 1, 5):
        ref = ot.trace(src, axes, np.ones(6), boxes=city.boxes, s_max=300.0, max_refl=max_refl)
        got, _ = gpu_trace(src, axes, np.ones(6), boxes=city.boxes, s_max=300.0, max_refl=max_refl)
        assert_same(ref, got)
    # straight down onto a roof, and from a source above every roof
    ref = ot.trace(np.array([[30.0, 30.0, 80.0]]), axes, np.ones(6), boxes=city.boxes, s_max=300.0, max_refl=4)
    got, _ = gpu_trace(np.array([[30.0, 30.0, 80.0]]), axes, np.ones(6), boxes=city.boxes, s_max=300.0, max_refl=4)
    assert_same(ref, got)
    # no rays at all
    got, t = gpu_trace(src, np.zeros((0, 3)), np.zeros(0), boxes=city.boxes, s_max=300.0)
    assert t.n_segs == 0 and list(got["ray_ptr"]) == [0] and list(got["face_ptr"]) == [0]


def test_count_token_reuse_and_staleness():
    """gbs_trace with the token of the last count reuses it (same table as a
    full trace); a token from an earlier count, or for other arguments, is
    refused."""
    import ctypes
    city = grid_city(3, 40.0, 20.0, 10.0, 40.0, seed=11)
    src = torch.as_tensor(np.array([[50.0, 50.0, 6.0]]), device="cuda")
    d, w = fibonacci_fan(2000)
    dd = torch.as_tensor(d, device="cuda")
    bx = torch.as_tensor(city.boxes, device="cuda")
    rs = torch.zeros(len(d), dtype=torch.int32, device="cuda")
    ctx = gbs.context("cuda")
    ctx.bind_stream()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    scene = _lib.GbsScene(len(city.boxes), 1, ptr(bx), 400.0, 6, 0)
    fan = _lib.GbsFan(1, ptr(src), len(d), ptr(dd), ptr(rs), None)
    ns, nf, tok1, tok2 = (ctypes.c_int64(0) for _ in range(4))
    cnt = lambda tok: ctx.lib.gbs_trace_count(ctx.handle, ctypes.byref(scene), ctypes.byref(fan), ctypes.byref(ns),
                                              ctypes.byref(nf), ctypes.byref(tok))
    assert cnt(tok1) == 0 and cnt(tok2) == 0 and tok1.value != tok2.value != 0
    S, F = ns.value, nf.value
    out = [torch.empty(len(d) + 1, dtype=torch.int64, device="cuda"), torch.empty((S, 3), dtype=torch.float64,
           device="cuda"), torch.empty((S, 3), dtype=torch.float64, device="cuda")] + \
        [torch.empty(S, dtype=torch.float64, device="cuda") for _ in range(3)] + \
        [torch.empty(S + 1, dtype=torch.int64, device="cuda"), torch.empty(F, dtype=torch.int32, device="cuda")]
    run = lambda tok: ctx.lib.gbs_trace(ctx.handle, ctypes.byref(scene), ctypes.byref(fan), tok, S, F,
                                        *[ptr(t) for t in out], None, ctypes.byref(ns), ctypes.byref(nf))
    assert run(tok1.value) == _lib.GBS_E_INVALID           # an earlier count
    assert cnt(tok2) == 0
    scene_other = _lib.GbsScene(len(city.boxes), 1, ptr(bx), 300.0, 6, 0)
    assert ctx.lib.gbs_trace(ctx.handle, ctypes.byref(scene_other), ctypes.byref(fan), tok2.value, S, F,
                             *[ptr(t) for t in out], None, ctypes.byref(ns), ctypes.byref(nf)) == _lib.GBS_E_INVALID
    assert cnt(tok2) == 0 and run(tok2.value) == 0         # reuses the count
    torch.cuda.synchronize()
    reused = [t.cpu().numpy() for t in out]
    assert run(0) == 0                                      # full trace, no token
    torch.cuda.synchronize()
    for a, b in zip(reused, out):
        assert np.array_equal(a, b.cpu().numpy())
    ref = ot.trace(np.array([[50.0, 50.0, 6.0]]), d, w, boxes=city.boxes, s_max=400.0, max_refl=6)
    assert np.array_equal(reused[0], ref["ray_ptr"]) and np.array_equal(reused[7], ref["face_ids"])


def test_invalid_requests_rejected():
    city = grid_city(2, 40.0, 20.0, 10.0, 30.0, seed=7)
    d, w = fibonacci_fan(10)
    src = np.array([[40.0, 40.0, 5.0]])
    with pytest.raises(_lib.GbsError):
        gbs.trace(src, d, w, boxes=city.boxes, s_max=100.0, image_complete=True)
    with pytest.raises(_lib.GbsError):
        gbs.trace(src, d, w, boxes=city.boxes, s_max=100.0, max_refl=33)
    with pytest.raises(_lib.GbsError):
        gbs.trace(src, 2.0 * d, w, boxes=city.boxes, s_max=100.0)
    with pytest.raises(_lib.GbsError):
        gbs.trace(np.array([[40.0, 40.0, -1.0]]), d, w, s_max=100.0)
    with pytest.raises(_lib.GbsError):
        gbs.trace(np.concatenate([src, src]), d, w, ray_src=np.array([1] * 5 + [0] * 5), s_max=100.0)
    with pytest.raises(_lib.GbsError):
        gbs.trace(src, d, w, ray_src=np.array([0] * 5 + [1] * 5), s_max=100.0)     # one source only
    bad = city.boxes.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(_lib.GbsError):
        gbs.trace(src, d, w, boxes=bad, s_max=100.0)


def test_full_size_city_sampled_rays():
    """The 1,000,000-ray 10 x 10 city traced on the device; 1,000 seeded
    rays re-traced one by one by the oracle match exactly."""
    city = grid_city(10, 40.0, 20.0, 10.0, 60.0, seed=1)
    src = np.array([[310.0, 310.0, 5.0]])
    d, w = fibonacci_fan(1_000_000)
    print("case trace full-size city, 1M rays", flush=True)
    got, t = gpu_trace(src, d, w, boxes=city.boxes, s_max=876.8, max_refl=10)
    rp = got["ray_ptr"]
    assert rp[0] == 0 and np.all(np.diff(rp) >= 1) and np.all(np.diff(rp) <= 11)
    assert 3.0 < t.n_segs / 1e6 < 4.2
    rays = np.sort(np.random.default_rng(6).choice(1_000_000, size=1000, replace=False))
    ref = ot.trace(src, d, w, boxes=city.boxes, s_max=876.8, max_refl=10, rays=rays)
    seg = np.concatenate([np.arange(rp[i], rp[i + 1]) for i in rays])
    assert np.array_equal(np.diff(ref["ray_ptr"]), rp[rays + 1] - rp[rays])
    for k in ("seg_a", "seg_t", "seg_s0", "seg_lo", "seg_hi"):
        assert np.array_equal(ref[k], got[k][seg]), k
    fp = got["face_ptr"]
    assert np.array_equal(np.diff(ref["face_ptr"]), fp[seg + 1] - fp[seg])
    fidx = np.concatenate([np.arange(fp[j], fp[j + 1]) for j in seg])
    assert np.array_equal(ref["face_ids"], got["face_ids"][fidx])


def test_traced_table_through_the_summation():
    """Trace on the device, sum on the device (MIX and F64) against the
    oracle tracer's table summed by the oracle."""
    import oracle
    city = grid_city(3, 40.0, 20.0, 10.0, 40.0, seed=11)
    src = np.array([[50.0, 50.0, 6.0]])
    d, w = fibonacci_fan(6000)
    ref = ot.trace(src, d, w, boxes=city.boxes, s_max=400.0, max_refl=6)
    rng = np.random.default_rng(12)
    gamma = np.concatenate([[1.0 + 0j], rng.uniform(0.6, 0.95, ref["n_faces"] - 1) *
                            np.exp(1j * rng.uniform(-0.4, 0.4, ref["n_faces"] - 1))])
    rcv = receiver_grid(40, 40, 0.0, 200.0, 0.0, 200.0, 1.5)
    freqs, eps = np.array([500.0]), np.array([[20.0]])
    tab = types.SimpleNamespace(**ref, n_src=1, n_rays=len(d), n_segs=len(ref["seg_s0"]))
    print("case traced table -> summation", flush=True)
    P_ref, TL_ref, ab = oracle.forward(tab, gamma, rcv, freqs, eps, n_threads=oracle_threads(), return_absum=True)
    t = gbs.trace(src, d, w, boxes=city.boxes, s_max=400.0, max_refl=6)
    for mode in ("f64", "mix"):
        P, TL = gbs.forward(t, rcv, freqs, eps, gamma, mode=mode)
        torch.cuda.synchronize()
        assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), mode)


def _launch_frames(d, seed):
    from scenes import normal_frame
    psi = np.random.default_rng(seed).uniform(0, np.pi, len(d))
    h = normal_frame(d)
    return np.cos(psi)[:, None] * h + np.sin(psi)[:, None] * np.cross(d, h)


@pytest.mark.parametrize("case", ["city", "open_plane"])
def test_frames_carried_bit_exact(case):
    """With launch frames (anisotropic beams' widths turned per ray) the device
    tracer carries the frame to every segment, mirrored at each reflection,
    bit for bit as the oracle tracer does; the table with its frames then
    sums, on the device, to the oracle's anisotropic field."""
    from scenes import normal_frame
    d, w = fibonacci_fan(1200)
    e0 = _launch_frames(d, 5)
    if case == "city":
        city = grid_city(3, 40.0, 20.0, 10.0, 40.0, seed=11, panels=2)
        src = np.array([[50.0, 50.0, 6.0]])
        kw = dict(boxes=city.boxes, panels=2, s_max=400.0, max_refl=6)
    else:
        src = np.array([[0.0, 0.0, 10.0]])
        kw = dict(s_max=200.0, max_refl=1, image_complete=True)
    print(f"case trace frames {case}", flush=True)
    ref = ot.trace(src, d, w, e1=e0, **kw)
    got, t = gpu_trace(src, d, w, e1=e0, **kw)
    assert_same(ref, got)
    assert np.array_equal(t.seg_e1.cpu().numpy(), ref["seg_e1"])
    # the device table with its frames, summed on the device, against the oracle's sum of the oracle's table
    rcv = receiver_grid(6, 6, -40.0, 140.0, -40.0, 140.0, 1.5)
    f = np.array([500.0])
    eps = np.array([[12.0]])
    e2 = np.array([[20.0]])
    gam = np.full(t.n_faces, 0.9 * np.exp(0.2j))
    tab = types.SimpleNamespace(n_faces=t.n_faces, **{k: ref[k] for k in KEYS}, ray_w=ref["ray_w"],
                                ray_src=ref["ray_src"], src_xyz=ref["src_xyz"])
    tab.n_src, tab.n_rays, tab.n_segs = 1, len(ref["ray_w"]), len(ref["seg_s0"])
    import oracle
    P_ref, TL_ref, ab = oracle.forward(tab, gam, rcv, f, eps, eps_e2=e2, seg_e1=ref["seg_e1"],
                                       n_threads=oracle_threads(), return_absum=True)
    P, TL = gbs.forward(t, rcv, f, eps, gam, mode="f64", eps_e2=e2)
    torch.cuda.synchronize()
    st = compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab)
    assert st["rel_max"] <= 1e-8 and st["dtl_max"] <= 1e-6, st
    # without frames in the table the library's default (horizontal) frame gives another field
    assert not np.allclose(ref["seg_e1"], normal_frame(ref["seg_t"]))


def test_bad_launch_frames_rejected():
    d, w = fibonacci_fan(50)
    with pytest.raises(_lib.GbsError) as e:
        gbs.trace(np.array([[0.0, 0.0, 10.0]]), d, w, s_max=100.0, max_refl=1, e1=d)
    assert e.value.code == _lib.GBS_E_INVALID and "e1" in str(e.value)
