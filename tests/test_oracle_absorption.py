"""Pins of the oracle's atmospheric absorption.

The paper fixes the atmosphere of its runs (Tables 2 and 3: 20 deg C, 70 %
relative humidity, 1 atm) but not how it attenuates sound; the reading is
the pure-tone attenuation of ISO 9613-1 applied to each beam's pressure
amplitude as exp(-alpha s) along its arc length.  Pinned by:

  * the octave-band attenuation table the standard publishes (fixture in
    tests/golden/, with its citation), to its printed rounding;
  * the free-field monopole exp(ikr - alpha r)/(4 pi r) and Lloyd's mirror
    with each path attenuated by its own length (closed forms);
  * exact factorisation: one beam segment's term scales by exp(-alpha s);
  * central finite differences of the hand adjoint with absorption on.
"""
import json
import os

import numpy as np
import pytest

import oracle
from scenes import city_scene, eps_rule, fibonacci_fan, open_plane_2k, trace_open_plane
from tests.test_oracle_pins import C, monopole, single_ray_table

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "iso9613_octave_attenuation.json")


def test_attenuation_matches_the_published_table(oracle_lib):
    ref = json.load(open(GOLDEN))
    f = 1000.0 * 10.0 ** (np.arange(-12, 10, 3) / 10.0)
    for row in ref["rows"]:
        got = oracle.air_absorption_db(f, row["temperature_c"], row["humidity_pct"], 1.0) * 1e3
        want = np.asarray(row["alpha"], float)
        # printed to 0.1 dB/km (3 significant digits from 100 dB/km)
        assert np.all(np.abs(got - want) <= 0.06 + 0.005 * want), (row, np.round(got, 2))


def test_attenuation_physics(oracle_lib):
    f = np.geomspace(20.0, 20000.0, 40)
    a = oracle.air_absorption_db(f, 20.0, 70.0, 1.0)
    assert np.all(np.diff(a) > 0)                                 # rises with frequency
    lo = oracle.air_absorption_db([1.0, 2.0], 20.0, 70.0, 1.0)    # ~ f^2 far below relaxation
    assert abs(lo[1] / lo[0] - 4.0) < 1e-3
    np.testing.assert_allclose(oracle.air_absorption(f), a * np.log(10.0) / 20.0)


def test_free_field_monopole_with_absorption(oracle_lib):
    f = 500.0
    k = 2 * np.pi * f / C
    alpha = 0.01                                                  # Np/m: exp(-1.4) at the farthest receiver
    rng = np.random.default_rng(11)
    d = rng.standard_normal((48, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(10.0, 140.0, 48)
    S = np.array([0.0, 0.0, 10.0])
    R = S + d * r[:, None]
    dirs, w = fibonacci_fan(20000)
    table = trace_open_plane(S, dirs, w, s_max=180.0, policy="EC")
    eps = eps_rule([f], 150.0)
    P, TL = oracle.forward(table, np.array([0.0 + 0j]), R, [f], eps, alpha=[alpha])
    ref = monopole(R, S, k) * np.exp(-alpha * r)
    rel = np.abs(P[0] - ref) / np.abs(ref)
    assert np.abs(TL[0] + 20 * np.log10(np.abs(ref))).max() <= 0.1
    assert rel.max() <= 0.05 and np.percentile(rel, 50) <= 0.03
    # and the absorption changes the level by 8.686 alpha r dB
    P0, TL0 = oracle.forward(table, np.array([0.0 + 0j]), R, [f], eps)
    assert np.abs((TL[0] - TL0[0]) - 8.685889638 * alpha * r).max() <= 0.1     # of up to 12 dB


def test_lloyds_mirror_with_absorption(oracle_lib):
    sc = open_plane_2k(eps="rule")
    gamma = 0.8 * np.exp(1j * np.pi / 8)
    sc.gamma = np.array([gamma])
    alpha = 0.004
    k = 2 * np.pi * 500.0 / C
    P, TL = oracle.scene_forward(sc, n_threads=4, alpha=[alpha])
    S = sc.table.src_xyz[0]
    r1 = np.linalg.norm(sc.rcv - S, axis=1)
    r2 = np.linalg.norm(sc.rcv - S * np.array([1, 1, -1]), axis=1)
    Pd = monopole(sc.rcv, S, k) * np.exp(-alpha * r1)
    Pi = gamma * monopole(sc.rcv, S * np.array([1, 1, -1]), k) * np.exp(-alpha * r2)
    ref = Pd + Pi
    err = np.abs(P[0] - ref) / (np.abs(Pd) + np.abs(Pi))
    assert np.percentile(np.abs(TL[0] + 20 * np.log10(np.abs(ref))), 99) <= 0.1
    assert np.percentile(err, 99) <= 0.03


def test_single_segment_factorises(oracle_lib):
    """u(alpha) = u(0) exp(-alpha s) per pair, s the arc length at the receiver's projection."""
    tab = single_ray_table([[0.0, 0.0, 0.0]], [[1.0, 0.0, 0.0]], [7.0], [0.0], [100.0])
    R = np.array([[30.0, 1.0, 0.5], [55.0, -2.0, 0.0], [80.0, 0.0, 3.0]])
    P0, _ = oracle.forward(tab, np.ones(4, complex), R, [800.0], [[12.0]])
    P1, _ = oracle.forward(tab, np.ones(4, complex), R, [800.0], [[12.0]], alpha=[0.02])
    s = 7.0 + R[:, 0]
    np.testing.assert_allclose(P1[0], P0[0] * np.exp(-0.02 * s), rtol=1e-14)


def test_adjoint_with_absorption_matches_finite_differences(oracle_lib):
    sc = city_scene(n_blocks=2, n_rays=400, grid=3, freqs=(400.0, 900.0), max_refl=4, city_seed=5, panels=2,
                    complex_gamma=True)
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((sc.n_jobs, len(sc.rcv))) + 1j * rng.standard_normal((sc.n_jobs, len(sc.rcv)))
    alpha = np.array([0.003, 0.006])
    mask = np.zeros((sc.n_jobs, len(sc.rcv), sc.table.n_segs), np.uint8)
    oracle.forward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, mask_mode=1, mask=mask, alpha=alpha)

    def loss(gamma, rcv):
        P, _ = oracle.forward(sc.table, gamma, rcv, sc.freqs, sc.eps, mask_mode=2, mask=mask, alpha=alpha)
        return float(np.real(np.sum(lam * P)))

    dG, dR, _ = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam, alpha=alpha)
    dG0, dR0, _ = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam)
    assert np.abs(dR - dR0).max() > 1e-3 * np.abs(dR0).max()        # the absorption term matters
    for r in range(len(sc.rcv)):
        for d in range(3):
            h = 1e-6 * max(1.0, abs(sc.rcv[r, d]))
            Rp = sc.rcv.copy(); Rp[r, d] += h
            Rm = sc.rcv.copy(); Rm[r, d] -= h
            fd = (loss(sc.gamma, Rp) - loss(sc.gamma, Rm)) / (2 * h)
            assert abs(fd - dR[r, d]) <= 1e-5 * max(1e-3, np.abs(dR).max()), (r, d, fd, dR[r, d])
    f = int(np.unique(sc.table.face_ids)[-1])
    h = 1e-6
    gp = sc.gamma.copy(); gp[f] += h
    gm = sc.gamma.copy(); gm[f] -= h
    fd = (loss(gp, sc.rcv) - loss(gm, sc.rcv)) / (2 * h)
    assert abs(fd - dG[f, 0]) <= 1e-6 * max(1.0, abs(fd))
