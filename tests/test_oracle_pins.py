"""Pins for the FP64 oracle against what the physics and mathematics fix.

None of these re-type the oracle's formula: each compares it with a closed
form (free-field monopole, Lloyd's mirror), an exact invariance (rotation and
mirror symmetry of a product fan, multilinearity in the reflection
coefficients, order independence, interval tie-breaks), the gate threshold
placed analytically, or finite differences (for the hand adjoint).  A dropped
term, a wrong sign or index or a transposed operand in the oracle breaks at
least one of them.
"""
import numpy as np
import pytest

import oracle
from scenes import (RayTable, eps_literal, eps_rule, fibonacci_fan, open_plane, open_plane_2k, theta_phi_fan,
                    trace_open_plane, city_scene)

C = 343.0


def monopole(R, S, k):
    r = np.linalg.norm(R - S, axis=-1)
    return np.exp(1j * k * r) / (4.0 * np.pi * r)


def single_ray_table(a, t, s0, lo, hi, faces=(), w=1.0, n_faces=4):
    """Hand-built table: one ray, one segment per entry of the lists."""
    a = np.atleast_2d(np.asarray(a, float))
    t = np.atleast_2d(np.asarray(t, float))
    t = t / np.linalg.norm(t, axis=1, keepdims=True)
    n = a.shape[0]
    faces = list(faces) if len(faces) and isinstance(faces[0], (list, tuple)) else [list(faces)] * n
    fptr = np.concatenate([[0], np.cumsum([len(f) for f in faces])]).astype(np.int64)
    return RayTable(src_xyz=np.zeros((1, 3)), ray_ptr=np.array([0, n], np.int64), ray_w=np.array([w]),
                    ray_src=np.zeros(1, np.int32), seg_a=a, seg_t=t, seg_s0=np.atleast_1d(np.asarray(s0, float)),
                    seg_lo=np.atleast_1d(np.asarray(lo, float)), seg_hi=np.atleast_1d(np.asarray(hi, float)),
                    face_ptr=fptr, face_ids=np.array([f for fs in faces for f in fs], np.int32), n_faces=n_faces)


# ---------------------------------------------------------------- free field
def test_free_field_monopole(oracle_lib):
    """A dense fan with no ground reflection reproduces exp(ikr)/(4 pi r):
    pins the ray weighting of Eq. (3), the q0/q amplitude of Eq. (1), the
    sign of the phase and the Gaussian exponent."""
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
    eps = eps_rule([f], 150.0)
    P, TL = oracle.forward(table, np.array([0.0 + 0j]), R, [f], eps)
    ref = monopole(R, S, k)
    dTL = np.abs(TL[0] + 20 * np.log10(np.abs(ref)))
    rel = np.abs(P[0] - ref) / np.abs(ref)
    assert dTL.max() <= 0.1, dTL.max()
    assert rel.max() <= 0.05, rel.max()
    assert np.percentile(rel, 50) <= 0.03


def test_free_field_literal_eps_is_wrong(oracle_lib):
    """Documents why epsilon = lambda/2 is not used for physics: the paraxial
    error r/(k eps^2) is large and the free-field check fails by many dB."""
    f = 500.0
    k = 2 * np.pi * f / C
    S = np.array([0.0, 0.0, 10.0])
    R = S + np.array([[60.0, 20.0, -5.0], [100.0, -30.0, 2.0], [-80.0, 40.0, 1.0]])
    dirs, w = fibonacci_fan(20000)
    table = trace_open_plane(S, dirs, w, s_max=180.0, policy="EC")
    P, TL = oracle.forward(table, np.array([0.0 + 0j]), R, [f], eps_literal([f]))
    dTL = np.abs(TL[0] + 20 * np.log10(np.abs(monopole(R, S, k))))
    assert dTL.max() > 3.0


# ------------------------------------------------------------- Lloyd's mirror
@pytest.mark.parametrize("gamma", [1.0 + 0j, 0.8 * np.exp(1j * np.pi / 8)])
def test_lloyds_mirror(oracle_lib, gamma):
    """Point source over a reflecting plane: exp(ikr1)/(4 pi r1) +
    Gamma exp(ikr2)/(4 pi r2) (the verification case of the paper's Sec. 4.1,
    here on a 64 x 64 grid at 500 Hz).  Pins reflection, the image fan and
    the ground-extended beam intervals."""
    sc = open_plane_2k(eps="rule")
    sc.gamma = np.array([gamma])
    k = 2 * np.pi * 500.0 / C
    P, TL = oracle.scene_forward(sc, n_threads=4)
    S = sc.table.src_xyz[0]
    Pd = monopole(sc.rcv, S, k)
    Pi = gamma * monopole(sc.rcv, S * np.array([1, 1, -1]), k)
    ref = Pd + Pi
    err_norm = np.abs(P[0] - ref) / (np.abs(Pd) + np.abs(Pi))
    dTL = np.abs(TL[0] + 20 * np.log10(np.abs(ref)))
    assert np.percentile(dTL, 99) <= 0.1, np.percentile(dTL, 99)
    assert np.percentile(err_norm, 99) <= 0.03, np.percentile(err_norm, 99)
    assert np.median(dTL) <= 0.01


def test_truncated_ground_policy_is_wrong(oracle_lib):
    """Documents why beams are extended through the ground: truncating them
    at the reflection point misses Lloyd's mirror by several dB."""
    sc = open_plane_2k(eps="rule", policy="T")
    k = 2 * np.pi * 500.0 / C
    P, TL = oracle.scene_forward(sc, n_threads=4)
    S = sc.table.src_xyz[0]
    ref = monopole(sc.rcv, S, k) + monopole(sc.rcv, S * np.array([1, 1, -1]), k)
    dTL = np.abs(TL[0] + 20 * np.log10(np.abs(ref)))
    assert np.median(dTL) > 1.0


# ------------------------------------------------------------------ symmetry
def _sym_setup():
    S = np.array([0.0, 0.0, 10.0])
    M = 24
    dirs, w = theta_phi_fan(30, M)
    table = trace_open_plane(S, dirs, w, s_max=150.0, policy="EC")
    rng = np.random.default_rng(3)
    R = np.stack([rng.uniform(-60, 60, 10), rng.uniform(-60, 60, 10), rng.uniform(0.5, 8.0, 10)], axis=1)
    return S, M, table, R


def test_rotation_symmetry(oracle_lib):
    """The product fan is invariant under rotation by 2 pi / M about the
    source's vertical, so rotated receivers see the same field."""
    S, M, table, R = _sym_setup()
    g = np.array([0.8 * np.exp(1j * np.pi / 8)])
    P0, _ = oracle.forward(table, g, R, [500.0], [20.0])
    for m in (1, 5, 13):
        ang = 2 * np.pi * m / M
        rot = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1]])
        Pm, _ = oracle.forward(table, g, R @ rot.T, [500.0], [20.0])
        assert np.max(np.abs(Pm - P0) / np.abs(P0)) <= 1e-9


def test_mirror_symmetry(oracle_lib):
    """phi -> -phi maps the fan onto itself: mirrored receivers (y -> -y)
    see the same field."""
    S, M, table, R = _sym_setup()
    g = np.array([0.7 - 0.2j])
    P0, _ = oracle.forward(table, g, R, [250.0], [30.0])
    Pm, _ = oracle.forward(table, g, R * np.array([1, -1, 1]), [250.0], [30.0])
    assert np.max(np.abs(Pm - P0) / np.abs(P0)) <= 1e-9


# ------------------------------------------------------- structure of the sum
def test_linear_in_ground_coefficient(oracle_lib):
    """Over one plane every segment carries Gamma^0 or Gamma^1, so
    P(Gamma) = P(0) + Gamma (P(1) - P(0)) exactly (no conjugation)."""
    sc = open_plane(n_rays=3000, grid=6, half=80.0, freqs=(250.0, 1000.0))
    P0, _ = oracle.scene_forward(sc, gamma=np.array([0.0 + 0j]))
    P1, _ = oracle.scene_forward(sc, gamma=np.array([1.0 + 0j]))
    g = 0.3 - 0.9j
    Pg, _ = oracle.scene_forward(sc, gamma=np.array([g]))
    ref = P0 + g * (P1 - P0)
    assert np.max(np.abs(Pg - ref) / np.abs(ref)) <= 1e-12


def test_face_product_exact():
    """A beam that hit faces (1, 2, 1) carries Gamma_1^2 Gamma_2."""
    table = single_ray_table(a=[0, 0, 0], t=[1, 0.2, 0.1], s0=30.0, lo=0.0, hi=100.0, faces=[1, 2, 1])
    R = np.array([[40.0, 9.0, 3.0], [10.0, 1.0, 2.5]])
    gam = np.array([1.0, 0.6 + 0.3j, -0.2 + 0.9j, 0.5])
    P1, _ = oracle.forward(table, np.ones(4, complex), R, [400.0], [5.0])
    Pg, _ = oracle.forward(table, gam, R, [400.0], [5.0])
    assert np.allclose(Pg / P1, gam[1] ** 2 * gam[2], rtol=1e-13, atol=0)


def test_order_invariance(oracle_lib):
    """Permuting rays or receivers permutes nothing in the result."""
    sc = city_scene(n_blocks=3, n_rays=600, grid=5, freqs=(500.0,), max_refl=4, city_seed=7, panels=2,
                    complex_gamma=True)
    P0, _ = oracle.scene_forward(sc)
    rng = np.random.default_rng(0)
    perm_r = rng.permutation(sc.table.n_rays)
    Pr, _ = oracle.forward(sc.table.subset_rays(perm_r), sc.gamma, sc.rcv, sc.freqs, sc.eps)
    assert np.max(np.abs(Pr - P0) / np.abs(P0)) <= 1e-11
    perm_x = rng.permutation(len(sc.rcv))
    Px, _ = oracle.forward(sc.table, sc.gamma, sc.rcv[perm_x], sc.freqs, sc.eps)
    assert np.array_equal(Px[:, :], P0[:, perm_x])


def test_interval_split_tie_break():
    """Splitting a segment into [0, L) and [L, 2L) on the same axis changes
    nothing, also for receivers exactly on the split plane (counted once)."""
    L = 32.0
    whole = single_ray_table(a=[0, 0, 0], t=[1, 0, 0], s0=5.0, lo=0.0, hi=2 * L, faces=[])
    split = single_ray_table(a=[[0, 0, 0], [L, 0, 0]], t=[[1, 0, 0], [1, 0, 0]], s0=[5.0, 5.0 + L],
                             lo=[0.0, 0.0], hi=[L, L], faces=[[], []])
    R = np.array([[L, 1.0, 0.5], [L, -2.0, 1.0], [10.0, 1.0, 1.0], [50.0, 0.5, -1.0], [0.0, 0.3, 0.0]])
    Pw, _ = oracle.forward(whole, np.ones(4, complex), R, [300.0], [6.0])
    Ps, _ = oracle.forward(split, np.ones(4, complex), R, [300.0], [6.0])
    assert np.all(np.abs(Pw) > 0)
    assert np.max(np.abs(Ps - Pw) / np.abs(Pw)) <= 1e-13
    # sigma == hi is excluded, sigma == lo included
    edge = single_ray_table(a=[0, 0, 0], t=[1, 0, 0], s0=5.0, lo=0.0, hi=L, faces=[])
    Pe, _ = oracle.forward(edge, np.ones(4, complex), np.array([[L, 0.5, 0.0], [0.0, 0.5, 0.0]]), [300.0], [6.0])
    assert Pe[0, 0] == 0 and Pe[0, 1] != 0


def test_gate_threshold_placed_analytically():
    """A pair is kept iff its Gaussian factor exp(-(k eps / 2) n^2/(s^2+eps^2))
    is >= exp(-G): receivers placed just inside / outside the gate radius."""
    f, eps, G, s = 500.0, 8.0, 9.21, 60.0
    k = 2 * np.pi * f / C
    n_gate = np.sqrt(2 * G * (s * s + eps * eps) / (k * eps))
    table = single_ray_table(a=[0, 0, 0], t=[0, 0, 1], s0=0.0, lo=0.0, hi=200.0, faces=[])
    R = np.array([[n_gate * (1 - 1e-7), 0, s], [n_gate * (1 + 1e-7), 0, s], [0, n_gate * 0.5, s]])
    P, _ = oracle.forward(table, np.ones(4, complex), R, [f], [eps], gate=G)
    assert P[0, 0] != 0 and P[0, 1] == 0 and P[0, 2] != 0
    # the kept boundary value has Gaussian magnitude exp(-G) relative to the axis value
    Pax, _ = oracle.forward(table, np.ones(4, complex), np.array([[0, 0, s]]), [f], [eps], gate=G)
    assert abs(abs(P[0, 0]) / abs(Pax[0, 0]) - np.exp(-G)) <= 1e-5 * np.exp(-G)


def test_on_axis_beam():
    """On the axis the Gaussian factor is one and the term is the paraxial
    on-axis beam w k eps / (8 pi^2) exp(iks)/(s - i eps): as eps -> 0 the
    beam weight times the beam's 2 pi/(k eps) solid-angle footprint gives
    the monopole 1/(4 pi s)."""
    w = 1e-3
    table = single_ray_table(a=[0, 0, 0], t=[0, 1, 0], s0=12.0, lo=-100, hi=100.0, faces=[], w=w)
    f, eps = 700.0, 3.0
    k = 2 * np.pi * f / C
    R = np.array([[0, 25.0, 0]])
    P, _ = oracle.forward(table, np.ones(4, complex), R, [f], [eps])
    s = 37.0
    expect = w * k * eps / (8 * np.pi ** 2) * np.exp(1j * k * s) / (s - 1j * eps)
    assert abs(P[0, 0] - expect) <= 1e-13 * abs(expect)
    footprint = 2 * np.pi / (k * eps)   # integral of the Gaussian over solid angle, far field
    assert abs(abs(expect) * footprint / w - 1 / (4 * np.pi * s)) <= 0.01 / (4 * np.pi * s)


# -------------------------------------------------------------- hand adjoint
def _adjoint_case():
    sc = city_scene(n_blocks=2, n_rays=400, grid=3, freqs=(400.0, 900.0), max_refl=4, city_seed=5, panels=2,
                    complex_gamma=True)
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((sc.n_jobs, len(sc.rcv))) + 1j * rng.standard_normal((sc.n_jobs, len(sc.rcv)))
    return sc, lam


def _loss(sc, lam, gamma, rcv, eps, mask):
    P, _ = oracle.forward(sc.table, gamma, rcv, sc.freqs, eps, mask_mode=2, mask=mask)
    return float(np.real(np.sum(lam * P)))


def test_adjoint_matches_finite_differences(oracle_lib):
    """Central differences with the active set frozen (the almost-everywhere
    derivative) agree with the hand adjoint for Gamma, receivers and eps."""
    sc, lam = _adjoint_case()
    n_jobs, n_rcv, n_segs = sc.n_jobs, len(sc.rcv), sc.table.n_segs
    mask = np.zeros((n_jobs, n_rcv, n_segs), np.uint8)
    oracle.forward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, mask_mode=1, mask=mask)
    assert mask.sum() > 50
    dG, dR, dE = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam)
    # faces that are actually used
    used = np.unique(sc.table.face_ids)
    rng = np.random.default_rng(1)
    for f in rng.choice(used, size=min(6, len(used)), replace=False):
        for comp, unit in ((0, 1.0), (1, 1j)):
            h = 1e-6
            gp = sc.gamma.copy(); gp[f] += h * unit
            gm = sc.gamma.copy(); gm[f] -= h * unit
            fd = (_loss(sc, lam, gp, sc.rcv, sc.eps, mask) - _loss(sc, lam, gm, sc.rcv, sc.eps, mask)) / (2 * h)
            assert abs(fd - dG[f, comp]) <= 1e-6 * max(1.0, abs(fd)), (f, comp, fd, dG[f, comp])
    for r in range(n_rcv):
        for d in range(3):
            h = 1e-6 * max(1.0, abs(sc.rcv[r, d]))
            Rp = sc.rcv.copy(); Rp[r, d] += h
            Rm = sc.rcv.copy(); Rm[r, d] -= h
            fd = (_loss(sc, lam, sc.gamma, Rp, sc.eps, mask) - _loss(sc, lam, sc.gamma, Rm, sc.eps, mask)) / (2 * h)
            assert abs(fd - dR[r, d]) <= 1e-5 * max(1e-3, np.abs(dR).max()), (r, d, fd, dR[r, d])
    for j in range(n_jobs):
        h = 1e-6 * sc.eps.reshape(-1)[j]
        ep = sc.eps.reshape(-1).copy(); ep[j] += h
        em = sc.eps.reshape(-1).copy(); em[j] -= h
        fd = (_loss(sc, lam, sc.gamma, sc.rcv, ep, mask) - _loss(sc, lam, sc.gamma, sc.rcv, em, mask)) / (2 * h)
        assert abs(fd - dE[j]) <= 1e-6 * max(1e-3, abs(fd)), (j, fd, dE[j])


def test_adjoint_frozen_mask_matches_gate(oracle_lib):
    """Mask mode 2 with the recorded mask reproduces mode 0 exactly."""
    sc, lam = _adjoint_case()
    mask = np.zeros((sc.n_jobs, len(sc.rcv), sc.table.n_segs), np.uint8)
    P1, _ = oracle.forward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, mask_mode=1, mask=mask)
    P2, _ = oracle.forward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, mask_mode=2, mask=mask)
    P0, _ = oracle.forward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps)
    assert np.array_equal(P0, P1) and np.array_equal(P0, P2)


# ---------------------------------------------------------- FP64 accuracy
def test_fp64_accuracy_against_high_precision():
    """The FP64 evaluation loses no accuracy to cancellation: a tiny random
    case evaluated with 40-digit arithmetic agrees to 1e-12."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    rng = np.random.default_rng(4)
    n = 5
    a = rng.uniform(-20, 20, (n, 3))
    t = rng.standard_normal((n, 3)); t /= np.linalg.norm(t, axis=1, keepdims=True)
    s0 = rng.uniform(0, 30, n)
    table = single_ray_table(a=a, t=t, s0=s0, lo=np.full(n, -50.0), hi=np.full(n, 80.0),
                             faces=[[1], [], [2, 1], [3], []], w=0.01)
    gam = np.array([1.0, 0.9 - 0.1j, 0.7 + 0.2j, -0.5 + 0.5j])
    R = rng.uniform(-30, 30, (6, 3))
    f, eps = 250.0, 12.0
    P, _ = oracle.forward(table, gam, R, [f], [eps], gate=50.0)
    k = 2 * mp.pi * mp.mpf(f) / mp.mpf(C)
    for r in range(len(R)):
        acc = mp.mpc(0)
        for j in range(n):
            v = [mp.mpf(R[r, d]) - mp.mpf(a[j, d]) for d in range(3)]
            sig = sum(v[d] * mp.mpf(t[j, d]) for d in range(3))
            if not (-50 <= sig < 80):
                continue
            n2 = sum(x * x for x in v) - sig * sig
            q = mp.mpf(s0[j]) + sig - 1j * mp.mpf(eps)
            E = 1j * k * (mp.mpf(s0[j]) + sig + n2 / (2 * q))
            if mp.re(E) < -50:
                continue
            g = mp.mpc(1)
            for fi in table.face_ids[table.face_ptr[j]:table.face_ptr[j + 1]]:
                g *= mp.mpc(gam[fi].real, gam[fi].imag)
            acc += 1j * k * mp.mpf(0.01) / (8 * mp.pi ** 2) * g * (-1j * mp.mpf(eps)) / q * mp.exp(E)
        ref = complex(acc)
        assert abs(P[0, r] - ref) <= 1e-12 * abs(ref)
