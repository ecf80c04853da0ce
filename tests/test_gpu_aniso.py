"""GPU anisotropic beams (Eq. (1) with Q = diag(q1, q2)) against the oracle's
anisotropic sum, element by element: F64, MIX and F32 on the open plane (ground
reflections, image fan), F64 and MIX on a batched city (walls and roofs,
several sources and bands), with atmospheric absorption, over several passes of the
table, from a host-resident table and through a graph; equal widths give the
isotropic kernel's field; unsupported requests fail with an error.
The oracle takes each segment's frame vector as input (scenes.normal_frame,
the horizontal normal z x t), the library forms it from the axis itself.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_13382_amd as gbs
from scenes import city_batched, normal_frame, open_plane_2k
from tests.gpu_util import TOL, compare, oracle_threads

pytestmark = pytest.mark.gpu

# F64 bar for anisotropic beams: 1e-8 relative (the stated bar is 1e-4).  The
# library forms the frame from the axis, n2^2 as n^2 - n1^2 and the amplitude
# from real square roots, the oracle from complex roots and e2 = t x e1; per
# term the two agree to the rounding of phase arguments of up to ~1e5 rad
# (~1e-11), which cancellation at receivers with sum|u| / |P| up to 1e4
# amplifies.  On the batched city an FP64 numpy evaluation of the library's
# formula order lands at 2e-9 from the oracle (1.5e-9 on the GPU); the
# isotropic formula order at 4e-10.
TOL_ANISO = {"f64": (1e-8, 1e-6), "mix": TOL["mix"], "f32": TOL["f32"]}


def assert_within(stats, mode):
    rel_tol, dtl_tol = TOL_ANISO[mode]
    assert stats["dead_ok"], "receivers with no beam must get exactly zero"
    if rel_tol is not None:
        assert stats["rel_max"] <= rel_tol, (mode, stats)
    assert stats["dtl_max"] <= dtl_tol, (mode, stats)
    assert stats["masked_frac"] <= 0.01, stats


def ref_aniso(sc, eps_e2, alpha=None):
    return oracle.forward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, c=sc.c, gate=sc.gate,
                          n_threads=oracle_threads(), return_absum=True, alpha=alpha, eps_e2=eps_e2,
                          seg_e1=normal_frame(sc.table.seg_t))


@pytest.fixture(scope="module")
def plane():
    sc = open_plane_2k(eps="rule")
    sc.gamma = np.array([0.8 * np.exp(1j * np.pi / 8)])
    e2 = 1.8 * np.asarray(sc.eps)
    return sc, e2, ref_aniso(sc, e2)


@pytest.fixture(scope="module")
def city():
    sc = city_batched(n_src=3, ray_lo=2000, ray_hi=6000, grid=20)
    rng = np.random.default_rng(12)
    e2 = np.asarray(sc.eps).reshape(-1) * rng.uniform(0.5, 2.0, np.asarray(sc.eps).size)
    return sc, e2, ref_aniso(sc, e2)


@pytest.mark.parametrize("mode", ["f64", "mix", "f32"])
def test_open_plane_anisotropic(plane, mode):
    sc, e2, (P_ref, TL_ref, ab) = plane
    print(f"case aniso open plane mode={mode}", flush=True)
    t = gbs.Table(sc.table, device="cuda")
    P, TL = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode=mode, eps_e2=e2)
    torch.cuda.synchronize()
    assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), mode)


# F32 is the ablation mode: on this city (8 kHz, paths up to ~900 m) neither FP32
# form meets its 0.2 dB bar (a float32 numpy evaluation of the library's formula
# orders: isotropic 0.51 dB, anisotropic 6.1 dB), so F32 is checked on the open plane.
@pytest.mark.parametrize("mode", ["f64", "mix"])
def test_city_anisotropic(city, mode):
    sc, e2, (P_ref, TL_ref, ab) = city
    print(f"case aniso city mode={mode}", flush=True)
    t = gbs.Table(sc.table, device="cuda")
    P, TL = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode=mode,
                        eps_e2=torch.as_tensor(e2, device="cuda"))
    torch.cuda.synchronize()
    assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), mode)


def test_city_anisotropic_with_absorption():
    sc = city_batched(n_src=2, ray_lo=2000, ray_hi=4000, grid=16)
    e2 = 0.6 * np.asarray(sc.eps).reshape(-1)
    # three times the paper's atmosphere: up to ~24 Np over the longest beams at 8 kHz
    # (MIX carries the amplitude in FP32, whose range ends near exp(-87))
    alpha = np.tile(gbs.air_absorption(sc.freqs), (2, 1)) * 3.0
    P_ref, TL_ref, ab = ref_aniso(sc, e2, alpha)
    P0, TL0, _ = ref_aniso(sc, e2)
    fin = np.isfinite(TL_ref) & np.isfinite(TL0)
    assert np.median(TL_ref[fin] - TL0[fin]) > 1.0        # the absorption is not negligible here
    print("case aniso city absorption", flush=True)
    t = gbs.Table(sc.table, device="cuda")
    for mode in ("f64", "mix"):
        P, TL = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode=mode, eps_e2=e2,
                            alpha=alpha)
        torch.cuda.synchronize()
        assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), mode)


def test_passes_host_table_and_graph(plane):
    """Several passes over the table, a host-resident table and a graph
    replay give the one-pass device result (MIX)."""
    sc, e2, (P_ref, TL_ref, ab) = plane
    print("case aniso passes/host/graph", flush=True)
    t = gbs.Table(sc.table, device="cuda")
    P0, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, eps_e2=e2)
    P1, TL1 = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, eps_e2=e2, chunk_segs=1500)
    torch.cuda.synchronize()
    assert gbs.stats()["n_chunks"] >= 2
    h = gbs.Table(sc.table, device="cuda", on_host=True)
    P2, _ = gbs.forward(h, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, eps_e2=e2, chunk_segs=1500)
    g = gbs.Graph(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, eps_e2=e2)
    outs = []
    for _ in range(3):
        P3, _ = g.launch()
        torch.cuda.synchronize()
        outs.append(P3.clone())
    torch.cuda.synchronize()
    assert_within(compare(P1.cpu().numpy(), TL1.cpu().numpy(), P_ref, TL_ref, ab), "mix")
    assert torch.equal(P1, P2)
    for P3 in outs:
        assert torch.equal(P3, P0)


def test_equal_widths_match_the_isotropic_kernel(plane):
    sc, _, _ = plane
    t = gbs.Table(sc.table, device="cuda")
    for mode in ("f64", "mix"):
        Pi, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode=mode)
        Pa, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode=mode, eps_e2=sc.eps)
        torch.cuda.synchronize()
        tol = 1e-12 if mode == "f64" else 1e-5
        assert (Pa - Pi).abs().max().item() <= tol * Pi.abs().max().item(), mode


def test_unsupported_requests_fail(plane):
    sc, e2, _ = plane
    t = gbs.Table(sc.table, device="cuda")
    with pytest.raises(gbs._lib.GbsError):
        gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, eps_e2=-e2)
    with pytest.raises(ValueError):
        gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, eps_e2=np.ones(3))
    # the context stays usable
    P, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, eps_e2=e2)
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(P)).all()


def test_adjoint_and_impulse_response_reject_anisotropic_beams(plane):
    """Through the C ABI: gbs_backward and gbs_impulse_response return
    GBS_E_UNSUPPORTED when params.eps_e2 is set, and write nothing."""
    import ctypes
    from paper_2501_13382_amd import _lib
    from paper_2501_13382_amd.gbs import _Call, _ptr, context
    sc, e2, _ = plane
    t = gbs.Table(sc.table, device="cuda")
    ctx = context(t.device)
    ctx.bind_stream()
    call = _Call(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, sc.c, sc.gate, "mix", 0, 0, False, False, eps_e2=e2)
    lam = torch.ones(call.shape + (2,), dtype=torch.float64, device="cuda")
    d_gamma = torch.full((t.n_faces, 2), 7.0, dtype=torch.float64, device="cuda")
    rc = ctx.lib.gbs_backward(*call.common(ctx), _ptr(lam), _ptr(d_gamma), None, None)
    assert rc == _lib.GBS_E_UNSUPPORTED
    assert b"isotropic" in ctx.lib.gbs_last_error(ctx.handle)
    h = torch.full((t.n_src, call.n_rcv, 64), 7.0, dtype=torch.float64, device="cuda")
    rc = ctx.lib.gbs_impulse_response(ctx.handle, ctypes.byref(call.rays), ctypes.byref(call.segs),
                                      ctypes.byref(call.faces), _ptr(call.rcv), call.n_rcv, 2.0, 1, 1,
                                      _ptr(call.eps), None, ctypes.byref(call.params), 64, 64, _ptr(h))
    assert rc == _lib.GBS_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((d_gamma == 7.0).all()) and bool((h == 7.0).all())


def test_counting_kept_pairs(plane):
    """count_active counts the pairs the exact anisotropic gate keeps: the
    number the oracle's definition keeps (counted here in numpy from the same
    gate), and the field equals the uncounted call."""
    sc, e2, _ = plane
    t = gbs.Table(sc.table, device="cuda")
    P0, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, eps_e2=e2)
    P1, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, eps_e2=e2, count_active=True)
    torch.cuda.synchronize()
    st = gbs.stats()
    T = sc.table
    f1 = normal_frame(T.seg_t)
    f2 = np.cross(T.seg_t, f1)
    k = 2 * np.pi * sc.freqs[0] / sc.c
    e1, eb = float(np.asarray(sc.eps).reshape(-1)[0]), float(e2.reshape(-1)[0])
    kept = 0
    for r in sc.rcv:
        v = r[None, :] - T.seg_a
        sig = (v * T.seg_t).sum(1)
        s = T.seg_s0 + sig
        n1 = (v * f1).sum(1)
        n2 = (v * f2).sum(1)
        g = 0.5 * k * (e1 * n1 * n1 / (s * s + e1 * e1) + eb * n2 * n2 / (s * s + eb * eb))
        kept += int(np.count_nonzero((sig >= T.seg_lo) & (sig < T.seg_hi) & (g <= sc.gate)))
    assert 0 < st["active_pairs"] <= st["listed_pairs"]
    assert abs(st["active_pairs"] - kept) <= 1e-6 * kept + 2, (st["active_pairs"], kept)
    assert (P1 - P0).abs().max().item() <= 1e-6 * P0.abs().max().item()
