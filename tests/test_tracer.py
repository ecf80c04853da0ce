"""Checks on the seeded input tracer (data, not summation arithmetic)."""
import numpy as np

from scenes import (city_10x10, city_5x5_panels, city_batched, fibonacci_fan, open_plane_2k, theta_phi_fan,
                    trace_open_plane)


def test_fibonacci_weights_and_unit_dirs():
    d, w = fibonacci_fan(1001)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    assert abs(w.sum() - 4 * np.pi) < 1e-12
    # equal-area: mean direction ~ 0
    assert np.linalg.norm(d.mean(axis=0)) < 1e-2


def test_theta_phi_weights():
    d, w = theta_phi_fan(60, 48)
    assert abs(w.sum() - 4 * np.pi) < 4 * np.pi * 1e-3


def test_open_plane_table_structure():
    sc = open_plane_2k()
    t = sc.table
    t.validate()
    assert t.n_segs == 2 * t.n_rays          # direct + (real or completed) image segment
    assert np.all(np.diff(t.ray_ptr) == 2)
    # every second segment carries the ground
    assert np.array_equal(np.diff(t.face_ptr), np.tile([0, 1], t.n_rays))
    # image segments are straight lines from the image source
    img = t.src_xyz[0] * np.array([1, 1, -1])
    a, tt, s0 = t.seg_a[1::2], t.seg_t[1::2], t.seg_s0[1::2]
    virt = a - s0[:, None] * tt
    assert np.allclose(virt, img, atol=1e-9)
    # image beams span [0, s_max] in arc length
    assert np.allclose(s0 + t.seg_lo[1::2], 0.0, atol=1e-9)
    assert np.allclose(s0 + t.seg_hi[1::2], sc.meta["s_max"], atol=1e-9)


def _check_path_continuity(t):
    for i in range(t.n_rays):
        j0, j1 = t.ray_ptr[i], t.ray_ptr[i + 1]
        assert t.seg_s0[j0] == 0.0
        assert np.allclose(t.seg_a[j0], t.src_xyz[t.ray_src[i]])
        for j in range(j0, j1 - 1):
            L = t.seg_s0[j + 1] - t.seg_s0[j]
            assert L > 0
            end = t.seg_a[j] + L * t.seg_t[j]
            assert np.allclose(end, t.seg_a[j + 1], atol=1e-6)
            # specular reflection: the tangential part is kept, |t| preserved
            dt = t.seg_t[j + 1] - t.seg_t[j]
            ax = np.argmax(np.abs(dt))
            assert np.allclose(np.delete(dt, ax), 0.0, atol=1e-12)
            assert abs(t.seg_t[j + 1][ax] + t.seg_t[j][ax]) < 1e-12
            # face history grows by one face per reflection
            assert t.face_ptr[j + 2] - t.face_ptr[j + 1] == t.face_ptr[j + 1] - t.face_ptr[j] + 1


def test_city_paths():
    sc = city_10x10(n_rays=3000, grid=16)
    t = sc.table
    t.validate()
    counts = np.diff(t.ray_ptr)
    assert counts.min() >= 1 and counts.max() <= 11
    assert 2.5 < counts.mean() < 4.5
    _check_path_continuity(t.subset_rays(np.arange(0, t.n_rays, 7)))
    # segments do not start inside a building
    city = sc.meta["city"]
    a = t.seg_a
    for x0, x1, y0, y1, h in city.boxes:
        inside = (a[:, 0] > x0 + 1e-6) & (a[:, 0] < x1 - 1e-6) & (a[:, 1] > y0 + 1e-6) & (a[:, 1] < y1 - 1e-6) \
            & (a[:, 2] < h - 1e-6)
        assert not np.any(inside)


def test_city_ground_chain_extents():
    """A segment ending on the ground keeps its beam through the reflected
    segment; the reflected one reaches back to the incoming one's start."""
    sc = city_10x10(n_rays=2000, grid=16)
    t = sc.table
    for i in range(t.n_rays):
        j0, j1 = t.ray_ptr[i], t.ray_ptr[i + 1]
        for j in range(j0, j1 - 1):
            if t.face_ids[t.face_ptr[j + 2] - 1] == 0:      # segment j ends on the ground
                L = t.seg_s0[j + 1] - t.seg_s0[j]
                end_next = t.seg_s0[j + 1] + (t.seg_hi[j + 1] if t.seg_lo[j + 1] < 0 else 0)
                assert abs(t.seg_lo[j + 1] + L) < 1e-9
                assert t.seg_hi[j] > L


def test_panel_city_faces():
    sc = city_5x5_panels(n_rays=3000, grid=16)
    t = sc.table
    t.validate()
    assert t.n_faces == 501
    assert len(np.unique(t.face_ids)) > 100
    assert sc.gamma[0] == 1.0 and np.all(np.abs(sc.gamma[1:]) <= 0.95 + 1e-12)


def test_batched_city_sorted_by_source():
    sc = city_batched(n_src=3, ray_lo=300, ray_hi=900, grid=8)
    t = sc.table
    t.validate()
    assert t.n_src == 3 and sc.eps.shape == (3, 4)
    assert np.all(np.diff(t.ray_src) >= 0)


def test_transported_frame_mirrors_the_launch_frame():
    """The frame carried along each ray stays a unit vector normal to every
    axis; with launch angle psi it makes angle psi with the horizontal frame
    after an even number of reflections and -psi after an odd number (a
    mirror reverses orientation), and psi = 0 gives the horizontal frame."""
    from scenes import city_scene, normal_frame, transported_frame
    sc = city_scene(n_blocks=2, n_rays=600, grid=3, freqs=(400.0,), max_refl=5, city_seed=5, panels=2)
    T = sc.table
    psi = 0.4
    e = transported_frame(T, psi, panels=2)
    assert np.allclose(np.linalg.norm(e, axis=1), 1.0, atol=1e-14)
    assert np.abs((e * T.seg_t).sum(1)).max() <= 1e-14
    h = normal_frame(T.seg_t)
    cosang = (e * h).sum(1)
    sinang = (e * np.cross(T.seg_t, h)).sum(1)
    nref = np.diff(T.face_ptr)
    ang = np.arctan2(sinang, cosang)
    # the horizontal frame of a reflected axis may be the mirror image up to sign: compare modulo pi
    d_even = np.angle(np.exp(2j * (ang - psi))) / 2
    d_odd = np.angle(np.exp(2j * (ang + psi))) / 2
    assert np.abs(d_even[nref % 2 == 0]).max() <= 1e-12
    assert np.abs(d_odd[nref % 2 == 1]).max() <= 1e-12
    assert (nref % 2 == 1).any() and (nref >= 2).any()
    e0 = transported_frame(T, 0.0, panels=2)
    assert np.abs(np.abs((e0 * h).sum(1)) - 1.0).max() <= 1e-14
