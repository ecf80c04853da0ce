"""Pins of the oracle's broadband synthesis (impulse response).

  * the FFT route against the defining sum over bins, written out directly
    (transform sign, scale, bin offset, window, truncation);
  * free field: one arrival at t = r/c whose peak is 2 df sum(w_n)/(4 pi r)
    and whose shape is the closed-form band-limited pulse;
  * Lloyd's mirror: two arrivals at r1/c and r2/c, the second scaled by the
    ground coefficient (real here).
"""
import numpy as np

import oracle
from scenes import fibonacci_fan, open_plane_2k, trace_open_plane
from tests.test_oracle_pins import C, single_ray_table


def test_fft_route_matches_the_defining_sum(oracle_lib):
    tab = single_ray_table([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0]], [[1.0, 0.2, 0.0], [1.0, -0.3, 0.1]], [3.0, 9.0],
                           [0.0, 0.0], [80.0, 80.0])
    rcv = np.array([[20.0, 2.0, 0.5], [50.0, -8.0, 1.0]])
    df, bin0, n_bins, n_fft, n_t = 4.0, 3, 40, 256, 200
    freqs = (bin0 + np.arange(n_bins)) * df
    eps = np.full((1, n_bins), 15.0)
    w = 0.5 - 0.5 * np.cos(2 * np.pi * (np.arange(n_bins) + 0.5) / n_bins)
    h = oracle.impulse_response(tab, np.ones(4, complex), rcv, df, bin0, n_bins, eps, n_fft, n_t, window=w)
    P, _ = oracle.forward(tab, np.ones(4, complex), rcv, freqs, eps)
    dt = 1.0 / (n_fft * df)
    t = np.arange(n_t) * dt
    for r in range(2):
        direct = 2 * df * np.real(np.sum(w[:, None] * P[:, r][:, None] * np.exp(-2j * np.pi * freqs[:, None] * t[None, :]),
                                         axis=0))
        np.testing.assert_allclose(h[0, r], direct, rtol=0, atol=1e-12 * np.abs(direct).max())


def _pulse(t, r, df, bin0, n_bins, w, amp):
    f = (bin0 + np.arange(n_bins)) * df
    return 2 * df * amp * np.real(np.sum(w[:, None] * np.exp(2j * np.pi * f[:, None] * (r / C - t[None, :])), axis=0))


def test_free_field_arrival(oracle_lib):
    S = np.array([0.0, 0.0, 10.0])
    rcv = S + np.array([[60.0, 10.0, -5.0], [-30.0, 80.0, 2.0]])
    r = np.linalg.norm(rcv - S, axis=1)
    d, wr = fibonacci_fan(20000)
    table = trace_open_plane(S, d, wr, s_max=180.0, policy="EC")
    df, bin0, n_bins, n_fft = 2.0, 64, 160, 1024          # 128 - 446 Hz; period 1/df = 0.5 s > r/c
    freqs = (bin0 + np.arange(n_bins)) * df
    eps = (6.0 * np.sqrt(150.0 / (2 * np.pi * freqs / C)))[None, :]
    w = np.hanning(n_bins + 2)[1:-1]
    h = oracle.impulse_response(table, np.array([0.0 + 0j]), rcv, df, bin0, n_bins, eps, n_fft, n_fft, window=w)
    dt = 1.0 / (n_fft * df)
    t = np.arange(n_fft) * dt
    for k in range(2):
        ref = _pulse(t, r[k], df, bin0, n_bins, w, 1.0 / (4 * np.pi * r[k]))
        assert abs(np.argmax(h[0, k]) - np.argmax(ref)) <= 1
        assert abs(np.argmax(ref) * dt - r[k] / C) <= dt
        assert np.abs(h[0, k] - ref).max() <= 0.05 * np.abs(ref).max()


def test_lloyds_mirror_two_arrivals(oracle_lib):
    sc = open_plane_2k(eps="rule")
    sc.gamma = np.array([0.7 + 0j])
    idx = np.array([5, 700, 2100, 4000])
    rcv = sc.rcv[idx]
    S = sc.table.src_xyz[0]
    r1 = np.linalg.norm(rcv - S, axis=1)
    r2 = np.linalg.norm(rcv - S * np.array([1, 1, -1]), axis=1)
    df, bin0, n_bins, n_fft = 4.0, 100, 50, 1024          # 400 - 596 Hz; period 0.25 s > r2/c
    freqs = (bin0 + np.arange(n_bins)) * df
    eps = (6.0 * np.sqrt(sc.meta["r_ref"] / (2 * np.pi * freqs / C)))[None, :]
    w = np.hanning(n_bins + 2)[1:-1]
    h = oracle.impulse_response(sc.table, sc.gamma, rcv, df, bin0, n_bins, eps, n_fft, n_fft, window=w)
    t = np.arange(n_fft) / (n_fft * df)
    for k in range(len(idx)):
        ref = _pulse(t, r1[k], df, bin0, n_bins, w, 1 / (4 * np.pi * r1[k])) + \
            _pulse(t, r2[k], df, bin0, n_bins, w, 0.7 / (4 * np.pi * r2[k]))
        assert np.abs(h[0, k] - ref).max() <= 0.05 * np.abs(ref).max(), k
