"""GPU anisotropic beams (Eq. (1) with Q = diag(q1, q2)) against the oracle's
anisotropic sum, element by element: F64, MIX and F32 on the open plane (ground
reflections, image fan), F64 and MIX on a batched city (walls and roofs,
several sources and bands), with atmospheric absorption, over several passes of the
table, from a host-resident table and through a graph; equal widths give the
isotropic kernel's field; unsupported requests fail with an error.
The oracle takes each segment's frame vector as input (scenes.normal_frame,
the horizontal normal z x t), the library forms it from the axis itself when
the table carries none.  With a frame carried in the table: an open plane
over a tilted ground (launch widths turned per ray, mirrored at the ground)
in every mode, streamed and replayed.  The anisotropic adjoint against the
oracle's hand adjoint and through torch's gradcheck.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_13382_amd as gbs
from scenes import city_batched, normal_frame, open_plane_2k, rotate_table, transported_frame
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


def test_impulse_response_rejects_anisotropic_beams(plane):
    """Through the C ABI: gbs_impulse_response returns GBS_E_UNSUPPORTED when
    params.eps_e2 is set, and writes nothing."""
    import ctypes
    from paper_2501_13382_amd import _lib
    from paper_2501_13382_amd.gbs import _Call, _ptr, context
    sc, e2, _ = plane
    t = gbs.Table(sc.table, device="cuda")
    ctx = context(t.device)
    ctx.bind_stream()
    call = _Call(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, sc.c, sc.gate, "mix", 0, 0, False, eps_e2=e2)
    h = torch.full((t.n_src, call.n_rcv, 64), 7.0, dtype=torch.float64, device="cuda")
    rc = ctx.lib.gbs_impulse_response(ctx.handle, ctypes.byref(call.rays), ctypes.byref(call.segs),
                                      ctypes.byref(call.faces), _ptr(call.rcv), call.n_rcv, 2.0, 1, 1,
                                      _ptr(call.eps), None, ctypes.byref(call.params), 64, 64, _ptr(h))
    assert rc == _lib.GBS_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((h == 7.0).all())


def _rot(ax, ang):
    c, s = np.cos(ang), np.sin(ang)
    if ax == 0:
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


@pytest.fixture(scope="module")
def tilted():
    """An open plane over a ground tilted by 20 degrees (a face that is not
    axis-aligned): the level scene turned by R, with the ray frame carried in
    the table (launch widths turned by a random angle per ray, mirrored at the
    ground, then turned by R)."""
    sc = open_plane_2k(eps="rule", n_rays=2000, grid=24)
    psi = np.random.default_rng(3).uniform(0, np.pi, sc.table.n_rays)
    R = _rot(2, 0.3) @ _rot(0, np.deg2rad(20.0))
    tab = rotate_table(sc.table, R)
    e1 = transported_frame(sc.table, psi) @ R.T
    rcv = sc.rcv @ R.T
    gam = np.array([0.8 * np.exp(1j * np.pi / 8)])
    e2 = 1.9 * np.asarray(sc.eps)
    ref = oracle.forward(tab, gam, rcv, sc.freqs, sc.eps, c=sc.c, gate=sc.gate, n_threads=oracle_threads(),
                         return_absum=True, eps_e2=e2, seg_e1=e1)
    return sc, tab, e1, rcv, gam, e2, ref


@pytest.mark.parametrize("mode", ["f64", "mix", "f32"])
def test_table_frame_on_tilted_ground(tilted, mode):
    sc, tab, e1, rcv, gam, e2, (P_ref, TL_ref, ab) = tilted
    print(f"case aniso table frame tilted ground mode={mode}", flush=True)
    t = gbs.Table(tab, device="cuda", seg_e1=e1)
    P, TL = gbs.forward(t, rcv, sc.freqs, sc.eps, gam, c=sc.c, gate=sc.gate, mode=mode, eps_e2=e2)
    torch.cuda.synchronize()
    assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), mode)


def test_table_frame_host_streamed_and_graph(tilted):
    sc, tab, e1, rcv, gam, e2, (P_ref, TL_ref, ab) = tilted
    print("case aniso table frame host streamed and graph", flush=True)
    th = gbs.Table(tab, device="cuda", on_host=True, seg_e1=e1)
    kw = dict(c=sc.c, gate=sc.gate, mode="mix", eps_e2=e2, chunk_segs=tab.n_segs // 3 + 1)
    P, TL = gbs.forward(th, rcv, sc.freqs, sc.eps, gam, **kw)
    torch.cuda.synchronize()
    assert gbs.stats()["n_chunks"] >= 3
    assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), "mix")
    g = gbs.Graph(th, rcv, sc.freqs, sc.eps, gam, **kw)
    for rep in range(2):
        Pg, TLg = g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(Pg.cpu().numpy(), P.cpu().numpy())


def test_table_frame_rejected_when_not_normal(tilted):
    sc, tab, e1, rcv, gam, e2, _ = tilted
    bad = e1.copy()
    bad[5] = tab.seg_t[5]
    t = gbs.Table(tab, device="cuda", seg_e1=bad)
    with pytest.raises(gbs._lib.GbsError) as e:
        gbs.forward(t, rcv, sc.freqs, sc.eps, gam, c=sc.c, gate=sc.gate, mode="mix", eps_e2=e2)
    assert e.value.code == gbs._lib.GBS_E_INVALID and "frame" in str(e.value)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def adj_city():
    """A paneled city (complex coefficients, up to four reflections), launch
    widths turned by a random angle per ray and carried through every
    reflection, two bands with eps_e2 / eps of 1.7 and 0.6, random lambda."""
    from scenes import city_scene
    sc = city_scene(n_blocks=2, n_rays=1500, grid=8, freqs=(400.0, 900.0), max_refl=4, city_seed=5, panels=2,
                    complex_gamma=True)
    psi = np.random.default_rng(4).uniform(0, np.pi, sc.table.n_rays)
    e1 = transported_frame(sc.table, psi, panels=2)
    eps2 = sc.eps * np.array([[1.7, 0.6]])
    rng = np.random.default_rng(21)
    lam = rng.standard_normal((sc.n_jobs, len(sc.rcv))) + 1j * rng.standard_normal((sc.n_jobs, len(sc.rcv)))
    ref = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam, c=sc.c, gate=sc.gate, eps_e2=eps2,
                          seg_e1=e1)
    return sc, e1, eps2, lam, ref


@pytest.mark.parametrize("mode", ["f64", "mix"])
def test_aniso_adjoint_matches_oracle(adj_city, mode):
    """The anisotropic adjoint (frame terms in d_rcv, d_eps and d_eps_e2,
    coefficient sums) against the oracle's hand adjoint, bitwise repeatable,
    and the same over several passes."""
    sc, e1, eps2, lam, (rG, rR, rE, rE2) = adj_city
    t = gbs.Table(sc.table, device="cuda", seg_e1=e1)
    tol = 1e-8 if mode == "f64" else 1e-3
    first = None
    for chunk in (0, 0, sc.table.n_segs // 3 + 1):
        print(f"case aniso adjoint mode={mode} chunk={chunk}", flush=True)
        out = gbs.backward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, lam, c=sc.c, gate=sc.gate, mode=mode,
                           eps_e2=eps2, chunk_segs=chunk)
        torch.cuda.synchronize()
        dG, dR, dE, dE2 = [x.cpu().numpy() for x in out]
        errs = (_rel(dG, rG), _rel(dR, rR), _rel(dE.reshape(-1), rE), _rel(dE2.reshape(-1), rE2))
        print(errs, flush=True)
        assert max(errs) <= tol
        if first is None:
            first = (dG, dR, dE, dE2)
        elif chunk == 0:
            for x, y in zip(first, (dG, dR, dE, dE2)):
                assert np.array_equal(x, y)


def test_aniso_gradcheck_through_autograd():
    """torch.autograd.gradcheck of TL with respect to the coefficients, the
    receivers, eps and eps_e2 for anisotropic beams (GPU F64 path, the
    table's frame held fixed)."""
    from scenes import city_scene
    sc = city_scene(n_blocks=2, n_rays=500, grid=3, freqs=(400.0,), max_refl=4, city_seed=5, panels=2,
                    complex_gamma=True)
    e1 = transported_frame(sc.table, 0.7, panels=2)
    t = gbs.Table(sc.table, device="cuda", seg_e1=e1)
    gamma = torch.tensor(sc.gamma, dtype=torch.complex128, device="cuda", requires_grad=True)
    # the far corner of the 3 x 3 grid, (140, 140), gets no beam (P = 0, TL =
    # inf): no finite difference exists there
    rcv = torch.tensor(sc.rcv[:8], dtype=torch.float64, device="cuda", requires_grad=True)
    eps = torch.tensor(sc.eps, dtype=torch.float64, device="cuda", requires_grad=True)
    eps2 = torch.tensor(1.6 * sc.eps, dtype=torch.float64, device="cuda", requires_grad=True)
    opts = {"mode": "f64", "c": sc.c, "gate": sc.gate}
    freqs = torch.tensor(sc.freqs, dtype=torch.float64, device="cuda")

    def f(g, r, e, e2):
        P, TL = gbs.GBSFunction.apply(g, r, e, t, freqs, opts, e2)
        return TL
    assert torch.autograd.gradcheck(f, (gamma, rcv, eps, eps2), eps=1e-6, atol=1e-5, rtol=1e-4, nondet_tol=1e-9)


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
