"""Pins for the oracle's anisotropic beams (Eq. (1) with Q = diag(q1, q2)).

Each test compares the oracle with something its formula does not contain:
the free-field monopole and Lloyd's mirror (closed forms the beam sum must
reach whatever the beam widths and frame), the on-axis beam with its Gouy
phase split over the two axes, the Gaussian decay along each frame vector,
the isotropic oracle (a separate code path) at equal widths, and the exact
symmetry that swaps the two axes.  A swapped width, a wrong square-root
branch, a dropped factor or a wrong frame vector fails at least one of them.
"""
import numpy as np
import pytest

import oracle
from scenes import eps_rule, fibonacci_fan, normal_frame, open_plane_2k, trace_open_plane

from .test_oracle_pins import monopole, single_ray_table

C = 343.0


def _frame(table, up=(0.0, 0.0, 1.0)):
    return normal_frame(table.seg_t, up)


@pytest.mark.parametrize("up", [(0.0, 0.0, 1.0), (1.0, 2.0, 3.0)])
def test_free_field_monopole_anisotropic(oracle_lib, up):
    """Beams twice as wide along e2 as along e1 still sum to exp(ikr)/(4 pi r)
    (the stationary-phase value of the beam integral does not depend on the
    initial Q), for the horizontal frame and for a tilted one."""
    f = 500.0
    k = 2 * np.pi * f / C
    rng = np.random.default_rng(11)
    d = rng.standard_normal((48, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(10.0, 140.0, 48)
    S = np.array([0.0, 0.0, 10.0])
    R = S + d * r[:, None]
    dirs, w = fibonacci_fan(20000)
    table = trace_open_plane(S, dirs, w, s_max=180.0, policy="EC")
    e = eps_rule([f], 150.0)[0]
    P, TL = oracle.forward(table, np.array([0.0 + 0j]), R, [f], [0.8 * e], eps_e2=[1.6 * e],
                           seg_e1=_frame(table, up))
    ref = monopole(R, S, k)
    dTL = np.abs(TL[0] + 20 * np.log10(np.abs(ref)))
    rel = np.abs(P[0] - ref) / np.abs(ref)
    assert dTL.max() <= 0.1, dTL.max()
    assert rel.max() <= 0.05, rel.max()
    assert np.percentile(rel, 50) <= 0.03


@pytest.mark.parametrize("gamma", [1.0 + 0j, 0.8 * np.exp(1j * np.pi / 8)])
def test_lloyds_mirror_anisotropic(oracle_lib, gamma):
    """Lloyd's mirror with anisotropic beams in the horizontal frame (which
    the ground reflection maps to itself): the direct plus Gamma times the
    image monopole, on the 64 x 64 grid at 500 Hz."""
    sc = open_plane_2k(eps="rule")
    k = 2 * np.pi * 500.0 / C
    e = sc.eps[0]
    P, TL = oracle.forward(sc.table, np.array([gamma]), sc.rcv, sc.freqs, [e], eps_e2=[1.8 * e],
                           seg_e1=_frame(sc.table), n_threads=4)
    S = sc.table.src_xyz[0]
    Pd = monopole(sc.rcv, S, k)
    Pi = gamma * monopole(sc.rcv, S * np.array([1, 1, -1]), k)
    ref = Pd + Pi
    err_norm = np.abs(P[0] - ref) / (np.abs(Pd) + np.abs(Pi))
    dTL = np.abs(TL[0] + 20 * np.log10(np.abs(ref)))
    assert np.percentile(dTL, 99) <= 0.1, np.percentile(dTL, 99)
    assert np.percentile(err_norm, 99) <= 0.03, np.percentile(err_norm, 99)
    assert np.median(dTL) <= 0.01


def test_on_axis_beam_anisotropic():
    """On the axis the term is w k / (8 pi^2) sqrt(eps1 eps2 / (|q1| |q2|))
    exp(i (k s + (atan(eps1/s) + atan(eps2/s)) / 2)): each axis contributes
    half its Gouy phase (the isotropic beam's is atan(eps/s)).  The far-field footprint
    2 pi / (k sqrt(eps1 eps2)) times the on-axis magnitude is the monopole."""
    w = 1e-3
    table = single_ray_table(a=[0, 0, 0], t=[0, 1, 0], s0=12.0, lo=-100, hi=100.0, faces=[], w=w)
    f, e1, e2 = 700.0, 3.0, 7.5
    k = 2 * np.pi * f / C
    s = 37.0
    P, _ = oracle.forward(table, np.ones(4, complex), np.array([[0, 25.0, 0]]), [f], [e1], eps_e2=[e2],
                          seg_e1=np.array([[0.0, 0.0, 1.0]]))
    mag = w * k / (8 * np.pi ** 2) * np.sqrt(e1 * e2 / (np.hypot(s, e1) * np.hypot(s, e2)))
    phase = k * s + 0.5 * (np.arctan(e1 / s) + np.arctan(e2 / s))
    expect = mag * np.exp(1j * phase)
    assert abs(P[0, 0] - expect) <= 1e-13 * abs(expect)
    s_far = 1e5
    table = single_ray_table(a=[0, 0, 0], t=[0, 1, 0], s0=12.0, lo=-100, hi=2 * s_far, faces=[], w=w)
    P, _ = oracle.forward(table, np.ones(4, complex), np.array([[0, s_far - 12.0, 0]]), [f], [e1], eps_e2=[e2],
                          seg_e1=np.array([[0.0, 0.0, 1.0]]), gate=1e9)
    footprint = 2 * np.pi / (k * np.sqrt(e1 * e2))
    assert abs(abs(P[0, 0]) * footprint / w - 1 / (4 * np.pi * s_far)) <= 1e-3 / (4 * np.pi * s_far)


def test_gaussian_decay_along_each_axis():
    """Off the axis by n along e1 the magnitude falls by exp(-(k/2) n^2
    eps1/(s^2 + eps1^2)), along e2 by the same with eps2: the width that goes
    with each frame vector."""
    table = single_ray_table(a=[0, 0, 0], t=[1, 0, 0], s0=5.0, lo=-100, hi=100.0, faces=[], w=1.0)
    f, e1, e2 = 300.0, 4.0, 12.0
    k = 2 * np.pi * f / C
    x, n = 20.0, 3.0
    s = 5.0 + x
    f1 = np.array([[0.0, 1.0, 0.0]])                  # e1 = y, e2 = t x e1 = z
    R = np.array([[x, 0, 0], [x, n, 0], [x, 0, n]])
    P, _ = oracle.forward(table, np.ones(4, complex), R, [f], [e1], eps_e2=[e2], seg_e1=f1, gate=1e9)
    r1 = abs(P[0, 1]) / abs(P[0, 0])
    r2 = abs(P[0, 2]) / abs(P[0, 0])
    assert abs(r1 - np.exp(-0.5 * k * n * n * e1 / (s * s + e1 * e1))) <= 1e-13
    assert abs(r2 - np.exp(-0.5 * k * n * n * e2 / (s * s + e2 * e2))) <= 1e-13


def test_equal_widths_is_the_isotropic_beam(oracle_lib):
    """eps1 = eps2 gives the isotropic oracle's field (another code path: the
    q0/q amplitude and the n^2/q exponent) for any frame."""
    sc = open_plane_2k(eps="rule")
    rng = np.random.default_rng(2)
    idx = rng.choice(len(sc.rcv), 200, replace=False)
    g = np.array([0.8 * np.exp(1j * np.pi / 8)])
    P0, _ = oracle.forward(sc.table, g, sc.rcv[idx], sc.freqs, sc.eps, n_threads=4)
    P1, _ = oracle.forward(sc.table, g, sc.rcv[idx], sc.freqs, sc.eps, eps_e2=sc.eps,
                           seg_e1=_frame(sc.table, (0.3, -1.0, 0.2)), n_threads=4)
    scale = np.abs(P0).max()
    assert np.abs(P1 - P0).max() <= 1e-12 * scale


def test_axis_swap_symmetry(oracle_lib):
    """Exchanging the widths and the frame vectors (e1 -> e2 = t x e1) leaves
    the field unchanged."""
    sc = open_plane_2k(eps="rule")
    rng = np.random.default_rng(9)
    idx = rng.choice(len(sc.rcv), 150, replace=False)
    g = np.array([0.9 + 0.1j])
    e = sc.eps[0]
    f1 = _frame(sc.table)
    f2 = np.cross(sc.table.seg_t, f1)
    Pa, _ = oracle.forward(sc.table, g, sc.rcv[idx], sc.freqs, [0.6 * e], eps_e2=[2.0 * e], seg_e1=f1, n_threads=4)
    Pb, _ = oracle.forward(sc.table, g, sc.rcv[idx], sc.freqs, [2.0 * e], eps_e2=[0.6 * e], seg_e1=f2, n_threads=4)
    assert np.abs(Pa - Pb).max() <= 1e-12 * np.abs(Pa).max()
    Pc, _ = oracle.forward(sc.table, g, sc.rcv[idx], sc.freqs, [2.0 * e], eps_e2=[0.6 * e], seg_e1=f1, n_threads=4)
    assert np.abs(Pc - Pa).max() > 1e-3 * np.abs(Pa).max()     # the widths do matter


def test_horizontal_frame_is_transported_by_reflections():
    """In a traced city (ground, roofs, walls: every face axis-aligned) the
    frame carried along each ray by the reflections (the mirror flips the
    component of e1 along the face normal, as it flips the axis) equals,
    up to sign, the horizontal normal of each reflected axis: the frame the
    library forms from the axis alone is the transported one."""
    from scenes import city_scene
    sc = city_scene(n_blocks=3, n_rays=3000, grid=4, freqs=(500.0,), max_refl=8, city_seed=5)
    tab = sc.table
    checked = 0
    for i in range(tab.n_rays):
        b, e = tab.ray_ptr[i], tab.ray_ptr[i + 1]
        f = normal_frame(tab.seg_t[b:b + 1])[0]
        for j in range(b + 1, e):
            t0, t1 = tab.seg_t[j - 1], tab.seg_t[j]
            flipped = np.nonzero(np.sign(t0) != np.sign(t1))[0]
            assert len(flipped) == 1 and np.allclose(np.abs(t0), np.abs(t1), rtol=0, atol=0)
            f = f.copy()
            f[flipped[0]] = -f[flipped[0]]
            g = normal_frame(t1[None, :])[0]
            assert abs(abs(float(f @ g)) - 1.0) <= 1e-12
            checked += 1
    assert checked > 2000


# ------------------------------------------------------ anisotropic adjoint
def _aniso_adjoint_case(up=(1.0, 2.0, 3.0)):
    """A small paneled city (complex coefficients, several reflections) with
    a tilted frame, so that every frame term of the receiver gradient is
    exercised, and random adjoint weights."""
    from scenes import city_scene
    sc = city_scene(n_blocks=2, n_rays=400, grid=3, freqs=(400.0, 900.0), max_refl=4, city_seed=5, panels=2,
                    complex_gamma=True)
    e1 = _frame(sc.table, up)
    eps2 = sc.eps * np.array([[1.7, 0.6]])
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((sc.n_jobs, len(sc.rcv))) + 1j * rng.standard_normal((sc.n_jobs, len(sc.rcv)))
    return sc, e1, eps2, lam


def _aniso_loss(sc, e1, lam, gamma, rcv, eps, eps2, mask):
    P, _ = oracle.forward(sc.table, gamma, rcv, sc.freqs, eps, eps_e2=eps2, seg_e1=e1, mask_mode=2, mask=mask)
    return float(np.real(np.sum(lam * P)))


def test_aniso_adjoint_matches_finite_differences(oracle_lib):
    """Central differences of the anisotropic sum with the active set frozen
    agree with the hand adjoint for Gamma, the receivers (frame terms along
    e1 and e2 = t x e1) and both beam parameters."""
    sc, e1, eps2, lam = _aniso_adjoint_case()
    n_jobs, n_rcv, n_segs = sc.n_jobs, len(sc.rcv), sc.table.n_segs
    mask = np.zeros((n_jobs, n_rcv, n_segs), np.uint8)
    oracle.forward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, eps_e2=eps2, seg_e1=e1, mask_mode=1, mask=mask)
    assert mask.sum() > 50
    dG, dR, dE, dE2 = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam, eps_e2=eps2, seg_e1=e1)
    L = lambda g=sc.gamma, r=sc.rcv, e=sc.eps, e2=eps2: _aniso_loss(sc, e1, lam, g, r, e, e2, mask)
    used = np.unique(sc.table.face_ids)
    rng = np.random.default_rng(1)
    for f in rng.choice(used, size=min(6, len(used)), replace=False):
        for comp, unit in ((0, 1.0), (1, 1j)):
            h = 1e-6
            gp = sc.gamma.copy(); gp[f] += h * unit
            gm = sc.gamma.copy(); gm[f] -= h * unit
            fd = (L(g=gp) - L(g=gm)) / (2 * h)
            assert abs(fd - dG[f, comp]) <= 1e-6 * max(1.0, abs(fd)), (f, comp, fd, dG[f, comp])
    for r in range(n_rcv):
        for d in range(3):
            h = 1e-6 * max(1.0, abs(sc.rcv[r, d]))
            Rp = sc.rcv.copy(); Rp[r, d] += h
            Rm = sc.rcv.copy(); Rm[r, d] -= h
            fd = (L(r=Rp) - L(r=Rm)) / (2 * h)
            assert abs(fd - dR[r, d]) <= 1e-5 * max(1e-3, np.abs(dR).max()), (r, d, fd, dR[r, d])
    for j in range(n_jobs):
        for which, base, got in (("eps", sc.eps, dE), ("eps_e2", eps2, dE2)):
            h = 1e-6 * base.reshape(-1)[j]
            ep = base.reshape(-1).copy(); ep[j] += h
            em = base.reshape(-1).copy(); em[j] -= h
            if which == "eps":
                fd = (L(e=ep) - L(e=em)) / (2 * h)
            else:
                fd = (L(e2=ep) - L(e2=em)) / (2 * h)
            assert abs(fd - got[j]) <= 1e-6 * max(1e-3, abs(fd)), (which, j, fd, got[j])


def test_aniso_adjoint_equal_widths_is_isotropic(oracle_lib):
    """With eps_e2 = eps the anisotropic adjoint (any frame) equals the
    isotropic one, and its two beam-parameter derivatives add up to the
    isotropic d/deps (another code path)."""
    sc, e1, _, lam = _aniso_adjoint_case()
    dG, dR, dE, dE2 = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam, eps_e2=sc.eps, seg_e1=e1)
    iG, iR, iE = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam)
    scale = lambda x: max(np.abs(x).max(), 1e-300)
    assert np.abs(dG - iG).max() <= 1e-10 * scale(iG)
    assert np.abs(dR - iR).max() <= 1e-10 * scale(iR)
    assert np.abs(dE + dE2 - iE).max() <= 1e-10 * scale(iE)


def test_aniso_adjoint_axis_swap(oracle_lib):
    """Swapping the widths together with the frame vectors (e1 -> e2 = t x e1)
    leaves the field unchanged, so d_gamma and d_rcv are unchanged and the two
    beam-parameter derivatives trade places."""
    sc, e1, eps2, lam = _aniso_adjoint_case()
    e2 = np.cross(sc.table.seg_t, e1)
    a = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam, eps_e2=eps2, seg_e1=e1)
    b = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, eps2, lam, eps_e2=sc.eps, seg_e1=e2)
    scale = lambda x: max(np.abs(x).max(), 1e-300)
    assert np.abs(a[0] - b[0]).max() <= 1e-10 * scale(a[0])
    assert np.abs(a[1] - b[1]).max() <= 1e-10 * scale(a[1])
    assert np.abs(a[2] - b[3]).max() <= 1e-10 * scale(a[2])
    assert np.abs(a[3] - b[2]).max() <= 1e-10 * scale(a[3])


# ---------------------------------------------- frames carried in the table
def _rot(ax, ang):
    c, s = np.cos(ang), np.sin(ang)
    if ax == 0:
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def test_tilted_ground_rotation_invariance(oracle_lib):
    """An open plane over a ground tilted by 20 degrees (the whole scene turned
    by a rotation R, a face that is not axis-aligned) with the frame carried by
    the table (R times the frame transported in the level scene, launch
    widths turned by a per-ray angle) gives, at the turned receivers, the
    level scene's anisotropic field to rounding.  The default horizontal
    frame of the turned axes (z x t) is not the transported one there and
    gives another field."""
    from scenes import rotate_table, transported_frame
    sc = open_plane_2k(eps="rule", n_rays=1500, grid=12)
    psi = np.random.default_rng(3).uniform(0, np.pi, sc.table.n_rays)
    e1 = transported_frame(sc.table, psi)
    e2 = 1.9 * np.asarray(sc.eps)
    gam = np.array([0.8 * np.exp(1j * np.pi / 8)])
    R = _rot(2, 0.3) @ _rot(0, np.deg2rad(20.0))
    tab_r = rotate_table(sc.table, R)
    P0, _ = oracle.forward(sc.table, gam, sc.rcv, sc.freqs, sc.eps, eps_e2=e2, seg_e1=e1, n_threads=4)
    P1, _ = oracle.forward(tab_r, gam, sc.rcv @ R.T, sc.freqs, sc.eps, eps_e2=e2, seg_e1=e1 @ R.T, n_threads=4)
    scale = np.abs(P0).max()
    assert np.abs(P1 - P0).max() <= 1e-9 * scale
    P2, _ = oracle.forward(tab_r, gam, sc.rcv @ R.T, sc.freqs, sc.eps, eps_e2=e2, seg_e1=normal_frame(tab_r.seg_t),
                           n_threads=4)
    assert np.abs(P2 - P0).max() >= 1e-4 * scale
