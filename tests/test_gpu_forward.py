"""GPU forward parity: the HIP library through its C ABI against the FP64 oracle.

Element-by-element on seeded inputs at sizes the oracle finishes in seconds
(several patches, ragged tails), plus sampled receivers at the full
100,000-ray, eight-band, 512 x 512 open-plane size in the benchmark's launch
configuration.  Tolerances (relative complex error, |dTL|) per mode are in
gpu_util.TOL: F64 1e-9 / 1e-6 dB, MIX 1e-4 / 0.05 dB, F32 - / 0.2 dB; TL is
compared where the sum is not cancelled beyond sum|u| / |P| <= 1e4.
"""
import json
import os
import tempfile

import numpy as np
import pytest
import torch

import paper_2501_13382_amd as gbs
from paper_2501_13382_amd import _lib
from scenes import (OCTAVES_8, RayTable, city_10x10, city_5x5_panels, city_batched, open_plane, open_plane_100k,
                    open_plane_2k, receiver_subsample)
from tests.gpu_util import assert_within, compare, reference

pytestmark = pytest.mark.gpu

MODES = ["f64", "mix", "f32"]


def gpu_forward(sc, rcv=None, mode="mix", table=None, **kw):
    t = gbs.Table(sc.table if table is None else table, device="cuda")
    P, TL = gbs.forward(t, sc.rcv if rcv is None else rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate,
                        mode=mode, **kw)
    torch.cuda.synchronize()
    return P.cpu().numpy(), TL.cpu().numpy()


@pytest.fixture(scope="module")
def plane2k():
    sc = open_plane_2k(eps="rule")
    return sc, reference(sc)


@pytest.fixture(scope="module")
def plane2k_literal():
    sc = open_plane_2k(eps="literal")
    return sc, reference(sc)


@pytest.mark.parametrize("mode", MODES)
def test_open_plane_2k(plane2k, mode):
    sc, (P_ref, TL_ref, ab) = plane2k
    print(f"case open_plane_2k mode={mode}", flush=True)
    P, TL = gpu_forward(sc, mode=mode)
    st = compare(P, TL, P_ref, TL_ref, ab)
    print(st)
    assert_within(st, mode)


@pytest.mark.parametrize("mode", MODES)
def test_open_plane_2k_literal_eps(plane2k_literal, mode):
    sc, (P_ref, TL_ref, ab) = plane2k_literal
    print(f"case open_plane_2k_literal mode={mode}", flush=True)
    P, TL = gpu_forward(sc, mode=mode)
    st = compare(P, TL, P_ref, TL_ref, ab)
    print(st)
    assert_within(st, mode)


@pytest.mark.parametrize("mode", ["f64", "mix"])
def test_ragged_random_receivers(mode):
    """3,001 scattered receivers (not a multiple of any patch size), three bands."""
    sc = open_plane(n_rays=4000, grid=2, half=300.0, freqs=(125.0, 1000.0, 4000.0),
                    gamma_ground=0.8 * np.exp(1j * np.pi / 8))
    rng = np.random.default_rng(17)
    rcv = np.stack([rng.uniform(-300, 300, 3001), rng.uniform(-300, 300, 3001), rng.uniform(0.5, 20, 3001)], 1)
    P_ref, TL_ref, ab = reference(sc, rcv=rcv)
    print(f"case ragged mode={mode}", flush=True)
    P, TL = gpu_forward(sc, rcv=rcv, mode=mode)
    assert_within(compare(P, TL, P_ref, TL_ref, ab), mode)


@pytest.fixture(scope="module")
def city_small():
    sc = city_10x10(n_rays=20000, grid=48)
    return sc, reference(sc)


@pytest.mark.parametrize("mode", MODES)
def test_city_10x10(city_small, mode):
    sc, (P_ref, TL_ref, ab) = city_small
    print(f"case city_10x10 mode={mode}", flush=True)
    P, TL = gpu_forward(sc, mode=mode)
    st = compare(P, TL, P_ref, TL_ref, ab)
    print(st)
    assert_within(st, mode)


@pytest.mark.parametrize("mode", ["f64", "mix"])
def test_panel_city_complex_coefficients(mode):
    sc = city_5x5_panels(n_rays=15000, grid=40)
    P_ref, TL_ref, ab = reference(sc)
    print(f"case city_5x5_panels mode={mode}", flush=True)
    P, TL = gpu_forward(sc, mode=mode)
    assert_within(compare(P, TL, P_ref, TL_ref, ab), mode)


@pytest.mark.parametrize("mode", ["f64", "mix"])
def test_batched_sources_and_bands(mode):
    """Several sources with ragged ray counts and four bands in one launch."""
    sc = city_batched(n_src=4, ray_lo=2000, ray_hi=9000, grid=24)
    P_ref, TL_ref, ab = reference(sc)
    print(f"case batched mode={mode}", flush=True)
    P, TL = gpu_forward(sc, mode=mode)
    assert P.shape == (4, 4, len(sc.rcv))
    assert_within(compare(P, TL, P_ref, TL_ref, ab), mode)


def test_batched_city_f32_ablation():
    """The all-FP32 ablation on the batched city: within its 0.2 dB bar in
    the 125 Hz and 500 Hz bands.  At 2 and 8 kHz, over paths of several
    hundred metres, FP32 geometry and phase lose that bar (the reason the
    FP32 + FP64 phase mode exists: FP32 arc lengths of ~900 m are off by
    ~5e-5 m, a phase error of k 5e-5 ~ 7e-3 rad per term at 8 kHz, amplified
    where terms cancel); the test then reports the measured error as an
    expected failure instead of hiding those bands."""
    sc = city_batched(n_src=4, ray_lo=2000, ray_hi=9000, grid=24)
    P_ref, TL_ref, ab = reference(sc)
    print("case batched f32", flush=True)
    P, TL = gpu_forward(sc, mode="f32")
    shape = (sc.table.n_src, len(sc.freqs), len(sc.rcv))     # (source, band, receiver)
    P, TL, P_ref, TL_ref, ab = (np.reshape(x, shape) for x in (P, TL, P_ref, TL_ref, ab))
    missed = []
    for b, f in enumerate(sc.freqs):
        st = compare(P[:, b], TL[:, b], P_ref[:, b], TL_ref[:, b], ab[:, b])
        print(f"{f:.0f} Hz: {st}", flush=True)
        if f <= 500.0:
            assert_within(st, "f32")
        else:
            assert st["dead_ok"] and st["masked_frac"] <= 0.01, st
            if st["dtl_max"] > 0.2:
                missed.append(f"{f:.0f} Hz: max |dTL| {st['dtl_max']:.3f} dB, max relative error "
                              f"{st['rel_max']:.2e}")
    if missed:
        pytest.xfail("F32 ablation over the 0.2 dB bar at " + "; ".join(missed))


def test_deterministic_repeat(city_small):
    sc, _ = city_small
    P1, _ = gpu_forward(sc, mode="mix")
    P2, _ = gpu_forward(sc, mode="mix")
    assert np.array_equal(P1, P2)


@pytest.mark.parametrize("case", ["city_1band", "batched_4band", "plane_8band"])
def test_cull_records_replayed_or_recomputed_agree(case, city_small, monkeypatch):
    """The cull's fill pass replays the batch records of its count pass, and
    recomputes the waves whose records did not fit in GBS_CULL_RECORD_BYTES:
    the same lists, so the same sums bit for bit, whether every wave, one
    block of records per region (the rest recomputed) or no wave is recorded."""
    if case == "city_1band":
        sc, nb = city_small[0], 1
    elif case == "batched_4band":
        sc, nb = city_batched(n_src=4, ray_lo=2000, ray_hi=9000, grid=24), 4
    else:
        sc, nb = open_plane(n_rays=20000, grid=64, freqs=OCTAVES_8, name="plane_8band"), 8
    one_block_per_region = 4 * 256 * (260 + 144 * nb)
    out = {}
    for label, limit in (("all", None), ("some", one_block_per_region), ("none", 0)):
        if limit is None:
            monkeypatch.delenv("GBS_CULL_RECORD_BYTES", raising=False)
        else:
            monkeypatch.setenv("GBS_CULL_RECORD_BYTES", str(limit))
        print(f"case {case} records={label}", flush=True)
        out[label] = [gpu_forward(sc, mode="mix")[0] for _ in range(2)]
    ref = out["all"][1]
    for label, runs in out.items():
        for P in runs:
            assert np.array_equal(P, ref), label


@pytest.mark.parametrize("nr", [1, 2, 4])
def test_receivers_per_lane_agree(city_small, nr):
    sc, (P_ref, TL_ref, ab) = city_small
    print(f"case rcv_per_lane={nr}", flush=True)
    P, TL = gpu_forward(sc, mode="f64", rcv_per_lane=nr)
    assert_within(compare(P, TL, P_ref, TL_ref, ab), "f64")
    P1, _ = gpu_forward(sc, mode="f64", rcv_per_lane=1)
    assert np.max(np.abs(P - P1) / np.maximum(np.abs(P1), 1e-300)) <= 1e-12


def test_chunked_passes_match(city_small):
    """A tiny chunk budget (many passes over the table) matches one pass."""
    sc, (P_ref, TL_ref, ab) = city_small
    P1, _ = gpu_forward(sc, mode="f64")
    P2, TL2 = gpu_forward(sc, mode="f64", chunk_segs=5000)
    assert gbs.stats()["n_chunks"] > 5
    assert np.max(np.abs(P2 - P1) / np.maximum(np.abs(P1), 1e-300)) <= 1e-11
    assert_within(compare(P2, TL2, P_ref, TL_ref, ab), "f64")


def test_host_table_streamed(city_small):
    """A table in pinned host memory, streamed in chunks, matches the device table."""
    sc, (P_ref, TL_ref, ab) = city_small
    t = gbs.Table(sc.table, device="cuda", on_host=True)
    P, TL = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="f64", chunk_segs=20000)
    torch.cuda.synchronize()
    assert gbs.stats()["n_chunks"] >= 3
    assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), "f64")
    # copies of pass i+1 overlap pass i: the result is the device table's, bit for bit, on repeated calls
    d = gbs.Table(sc.table, device="cuda")
    Pd, _ = gbs.forward(d, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="mix", chunk_segs=20000)
    for _ in range(2):
        Ph, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="mix",
                            chunk_segs=20000)
        assert torch.equal(Ph, Pd)


def test_single_receiver_and_empty():
    sc = open_plane(n_rays=800, grid=2, half=50.0, freqs=(500.0,))
    one = np.array([[10.0, -5.0, 1.5]])
    P_ref, TL_ref, ab = reference(sc, rcv=one)
    P, TL = gpu_forward(sc, rcv=one, mode="f64")
    assert_within(compare(P, TL, P_ref, TL_ref, ab), "f64")
    P0, TL0 = gpu_forward(sc, rcv=np.zeros((0, 3)), mode="mix")
    assert P0.shape == (1, 1, 0)


def test_source_without_rays_and_far_receivers():
    """A source that launched no ray, and receivers no beam reaches: P = 0 exactly, TL = +inf."""
    sc = open_plane(n_rays=600, grid=4, half=60.0, freqs=(500.0,))
    t = sc.table
    two = RayTable(src_xyz=np.vstack([t.src_xyz, [[5.0, 5.0, 5.0]]]), ray_ptr=t.ray_ptr, ray_w=t.ray_w,
                   ray_src=t.ray_src, seg_a=t.seg_a, seg_t=t.seg_t, seg_s0=t.seg_s0, seg_lo=t.seg_lo,
                   seg_hi=t.seg_hi, face_ptr=t.face_ptr, face_ids=t.face_ids, n_faces=1)
    sc.table = two
    sc.eps = np.vstack([sc.eps, sc.eps])
    far = np.vstack([sc.rcv, [[1e5, 1e5, 3.0]]])
    P_ref, TL_ref, ab = reference(sc, rcv=far)
    P, TL = gpu_forward(sc, rcv=far, mode="mix")
    assert np.all(P[1] == 0) and np.all(np.isinf(TL[1]))
    assert P[0, 0, -1] == 0 and np.isinf(TL[0, 0, -1])
    assert_within(compare(P, TL, P_ref, TL_ref, ab), "mix")


@pytest.mark.parametrize("entry,chunk", [("gbs_forward", 0), ("gbs_forward", 300), ("gbs_forward_noalloc", 0)])
def test_outputs_overwritten_whatever_they_held(entry, chunk):
    """P and TL are outputs only: buffers that hold NaN before the call come
    back with the sums of a call into fresh buffers, bit for bit, in one pass
    (the reduction writes every output itself), in several passes (P is
    cleared, then accumulated) and without allocation; receivers no beam
    reaches get P = 0 and TL = +inf."""
    from paper_2501_13382_amd import gbs as G
    sc = open_plane(n_rays=600, grid=4, half=60.0, freqs=(250.0, 1000.0))
    far = np.vstack([sc.rcv, [[1e5, 1e5, 3.0]]])
    t = gbs.Table(sc.table, device="cuda")
    P0, TL0 = gbs.forward(t, far, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="mix",
                          chunk_segs=chunk)
    shape = (1, len(sc.freqs), len(far))
    P = torch.full(shape + (2,), float("nan"), dtype=torch.float64, device="cuda")
    TL = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    print(f"case {entry} chunk_segs={chunk}", flush=True)
    Pc, TLc = G._forward(entry, t, far, sc.freqs, sc.eps, sc.gamma, sc.c, sc.gate, "mix", chunk, 0, 0, False,
                         False, True, None, None, (P, TL))
    torch.cuda.synchronize()
    if chunk:
        assert gbs.stats()["n_chunks"] > 1
    assert torch.equal(torch.view_as_real(Pc), torch.view_as_real(P0))
    assert torch.equal(TLc, TL0)
    assert torch.all(Pc[..., -1] == 0) and torch.all(torch.isinf(TLc[..., -1]))
    assert not torch.isnan(TLc).any()


def test_invalid_arguments_rejected():
    sc = open_plane(n_rays=200, grid=4, half=50.0, freqs=(500.0,))
    t = gbs.Table(sc.table, device="cuda")
    with pytest.raises(_lib.GbsError) as e:
        gbs.forward(t, sc.rcv, np.array([-1.0]), sc.eps, sc.gamma)
    assert e.value.code == _lib.GBS_E_INVALID
    with pytest.raises(_lib.GbsError) as e:
        gbs.forward(t, sc.rcv, sc.freqs, -sc.eps, sc.gamma)
    assert e.value.code == _lib.GBS_E_INVALID
    with pytest.raises(_lib.GbsError) as e:
        gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=0.0)
    assert e.value.code == _lib.GBS_E_INVALID
    with pytest.raises(_lib.GbsError) as e:
        gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, rcv_per_lane=3)
    assert e.value.code == _lib.GBS_E_INVALID


@pytest.fixture(scope="module")
def plane100k():
    sc = open_plane_100k()
    idx = receiver_subsample(len(sc.rcv), n=256, seed=5)
    return sc, idx, reference(sc, rcv=sc.rcv[idx])


@pytest.mark.parametrize("mode", ["mix", "f64"])
def test_full_size_open_plane_sampled(plane100k, mode):
    """The benchmark workload at full size (100,000 rays, 8 bands, 512 x 512
    receivers, default launch shape); 256 seeded receivers checked against
    the oracle."""
    sc, idx, (P_ref, TL_ref, ab) = plane100k
    print(f"case full-size open plane mode={mode}", flush=True)
    P, TL = gpu_forward(sc, mode=mode)
    st = compare(P[:, :, idx], TL[:, :, idx], P_ref, TL_ref, ab)
    print(st, gbs.stats())
    assert_within(st, mode)


def test_autotune_picks_a_valid_shape_and_results_agree(city_small):
    """The autotuner times the receivers-per-lane shapes and keeps one; later
    calls with the automatic shape give the same field."""
    sc, (P_ref, TL_ref, ab) = city_small
    t = gbs.Table(sc.table, device="cuda")
    cache = os.path.join(tempfile.mkdtemp(), "tune.json")
    choice = gbs.autotune(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="f64", cache=cache)
    assert choice["rcv_per_lane"] in (1, 2, 4) and choice["work_chunk"] in (1024, 2048, 4096)
    P, TL = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="f64")
    assert gbs.stats()["patch_rcv"] == 64 * choice["rcv_per_lane"]
    assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), "f64")
    # the JSON cache answers the same question without timing again
    with open(cache) as f:
        assert list(json.load(f).values()) == [choice]
    assert gbs.autotune(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="f64",
                        cache=cache) == choice
    # every work-unit size gives the same field to rounding
    for wc in (256, 1024, 65536):
        P2, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="f64", work_chunk=wc)
        assert np.max(np.abs(P2.cpu().numpy() - P.cpu().numpy()) / np.maximum(np.abs(P.cpu().numpy()), 1e-300)) <= 1e-11


def test_stats_are_consistent(city_small):
    sc, _ = city_small
    gpu_forward(sc, mode="mix", count_active=True, time_kernels=True)
    st = gbs.stats()
    assert st["dense_pairs"] == sc.dense_pairs
    assert 0 < st["active_pairs"] <= st["listed_pairs"]
    assert st["ms_pairs"] > 0 and st["ms_cull"] > 0 and st["grid"] > 0
