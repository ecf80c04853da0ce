"""Pins of the ray-tracing oracle (oracle/tracer.py) to closed forms and
geometric invariants of specular reflection, plus its agreement with the
vectorised input generator that writes the beam-summation tables.

The pins: the image-source construction (every reflected segment's axis
passes through the source mirrored in the planes of the faces it hit, in
order: Sec. 1), hit points lying on the face cell named by the face id,
closed-form paths off a single box and the ground, path continuity and the
arc-length budget, and the open plane's image completion.
"""
import math

import numpy as np
import pytest

from oracle import tracer as ot
from scenes import fibonacci_fan, grid_city, trace_city, trace_open_plane


def _face_plane(face, boxes, panels):
    """(axis, coordinate, cell rectangle) of a face: axis 2 / z = 0 for the
    ground; walls -x, +x, -y, +y and the roof of box b otherwise."""
    if face == 0:
        return 2, 0.0, None
    b, rest = divmod(face - 1, 5 * panels * panels)
    wall, cell = divmod(rest, panels * panels)
    x0, x1, y0, y1, h = boxes[b]
    iu, iv = divmod(cell, panels)
    if wall in (0, 1):
        u0, u1, v0, v1 = y0, y1, 0.0, h
        axis, coord = 0, (x0, x1)[wall]
        ru, rv = 1, 2
    elif wall in (2, 3):
        u0, u1, v0, v1 = x0, x1, 0.0, h
        axis, coord = 1, (y0, y1)[wall - 2]
        ru, rv = 0, 2
    else:
        u0, u1, v0, v1 = x0, x1, y0, y1
        axis, coord = 2, h
        ru, rv = 0, 1
    du, dv = (u1 - u0) / panels, (v1 - v0) / panels
    rect = (ru, u0 + iu * du, u0 + (iu + 1) * du, rv, v0 + iv * dv, v0 + (iv + 1) * dv)
    return axis, coord, rect


def _mirror(pt, axis, coord):
    q = np.array(pt, dtype=np.float64)
    q[axis] = 2.0 * coord - q[axis]
    return q


@pytest.fixture(scope="module")
def small_city():
    city = grid_city(3, 40.0, 20.0, 10.0, 40.0, seed=11, panels=2)
    src = np.array([50.0, 50.0, 6.0])
    d, w = fibonacci_fan(400)
    tab = ot.trace(src[None], d, w, boxes=city.boxes, panels=2, s_max=500.0, max_refl=6)
    return city, src, d, w, tab


def test_image_source_of_every_segment(small_city):
    """a - s0 t is the source mirrored successively in the planes of the
    history's faces (image-source geometry)."""
    city, src, _, _, tab = small_city
    fp, fi = tab["face_ptr"], tab["face_ids"]
    n_refl = 0
    for j in range(len(tab["seg_s0"])):
        img = src.copy()
        for f in fi[fp[j]:fp[j + 1]]:
            axis, coord, _ = _face_plane(int(f), city.boxes, 2)
            img = _mirror(img, axis, coord)
        virt = tab["seg_a"][j] - tab["seg_s0"][j] * tab["seg_t"][j]
        assert np.allclose(virt, img, rtol=0, atol=1e-9 * max(1.0, tab["seg_s0"][j])), j
        n_refl += fp[j + 1] - fp[j] > 0
    assert n_refl > 200                      # the fan does reflect, off walls, roofs and the ground
    assert set(np.unique(fi)) >= {0} and len(np.unique(fi)) > 20


def test_hit_points_lie_on_the_named_face_cell(small_city):
    city, _, _, _, tab = small_city
    fp, fi = tab["face_ptr"], tab["face_ids"]
    for j in range(len(tab["seg_s0"])):
        if fp[j + 1] == fp[j]:
            continue
        f = int(fi[fp[j + 1] - 1])                 # the face this segment starts on
        axis, coord, rect = _face_plane(f, city.boxes, 2)
        a = tab["seg_a"][j]
        assert abs(a[axis] - coord) <= 1e-9 * max(1.0, abs(coord))
        if rect is not None:
            ru, u0, u1, rv, v0, v1 = rect
            assert u0 - 1e-9 <= a[ru] <= u1 + 1e-9 and v0 - 1e-9 <= a[rv] <= v1 + 1e-9, (j, f)
        # the reflected direction leaves the face
        t = tab["seg_t"][j]
        assert abs(np.linalg.norm(t) - 1.0) < 1e-15


def test_path_continuity_and_arc_budget(small_city):
    """Each segment starts where the previous one ended (a ground start
    carries lo = -L_prev; a wall or roof start follows a truncated hi = L),
    arc lengths add up, and the last segment ends at s_max."""
    _, src, _, _, tab = small_city
    rp, a, t, s0, lo, hi = (tab[k] for k in ("ray_ptr", "seg_a", "seg_t", "seg_s0", "seg_lo", "seg_hi"))
    for i in range(len(rp) - 1):
        j0, j1 = rp[i], rp[i + 1]
        assert 1 <= j1 - j0 <= 7                    # at most max_refl + 1 segments
        assert np.array_equal(a[j0], src) and s0[j0] == 0.0 and lo[j0] == 0.0
        for j in range(j0, j1 - 1):
            on_ground = lo[j + 1] < 0.0
            L = -lo[j + 1] if on_ground else hi[j]
            if on_ground:
                assert a[j + 1][2] == 0.0 and hi[j] == L + hi[j + 1]
            assert s0[j + 1] == s0[j] + L
            assert np.allclose(a[j + 1], a[j] + L * t[j], rtol=0, atol=1e-9)
        assert s0[j1 - 1] + hi[j1 - 1] == pytest.approx(500.0, abs=1e-9)


def test_single_box_closed_forms():
    """Paths worked out by hand off one box x in [10, 20], y in [-5, 5],
    height 10, standing on the ground."""
    box = np.array([[10.0, 20.0, -5.0, 5.0, 10.0]])
    s2 = math.sqrt(0.5)
    src = np.array([[0.0, 0.0, 5.0]])
    dirs = np.array([[1.0, 0.0, 0.0],          # straight at the -x wall
                     [s2, 0.0, -s2],           # ground at (5, 0, 0), then the -x wall at (10, 0, 5)
                     [0.0, 1.0, 0.0]])         # misses everything
    tab = ot.trace(src, dirs, np.ones(3), boxes=box, s_max=100.0, max_refl=4)
    rp, a, t, s0, lo, hi = (tab[k] for k in ("ray_ptr", "seg_a", "seg_t", "seg_s0", "seg_lo", "seg_hi"))
    fp, fi = tab["face_ptr"], tab["face_ids"]
    assert list(rp) == [0, 2, 5, 6]
    # ray 0: 10 m to the wall (face 1 = box 0, wall -x), then back along -x
    assert hi[0] == 10.0 and lo[0] == 0.0
    assert np.allclose(a[1], [10.0, 0.0, 5.0]) and np.allclose(t[1], [-1.0, 0.0, 0.0])
    assert s0[1] == 10.0 and hi[1] == 90.0 and list(fi[fp[1]:fp[2]]) == [1]
    # ray 1: ground after 5 sqrt 2 (transparent extent), wall after another 5 sqrt 2
    L = 5.0 * math.sqrt(2.0)
    assert hi[2] == pytest.approx(2 * L, rel=1e-15) and lo[2] == 0.0
    assert np.allclose(a[3], [5.0, 0.0, 0.0]) and a[3][2] == 0.0
    assert np.allclose(t[3], [s2, 0.0, s2])
    assert lo[3] == pytest.approx(-L, rel=1e-15) and hi[3] == pytest.approx(L, rel=1e-15)
    assert np.allclose(a[4], [10.0, 0.0, 5.0]) and np.allclose(t[4], [-s2, 0.0, s2])
    assert list(fi[fp[3]:fp[4]]) == [0] and list(fi[fp[4]:fp[5]]) == [0, 1]
    assert s0[4] == pytest.approx(2 * L, rel=1e-15) and hi[4] == pytest.approx(100.0 - 2 * L, rel=1e-14)
    # ray 2: one segment of the full budget
    assert hi[5] == 100.0 and fp[6] == fp[5]


def test_roof_and_panel_cells():
    box = np.array([[10.0, 20.0, -5.0, 5.0, 10.0]])
    src = np.array([[12.0, -4.0, 30.0]])
    dirs = np.array([[0.0, 0.0, -1.0]])        # onto the roof cell (iu = 0, iv = 0)
    tab = ot.trace(src, dirs, np.ones(1), boxes=box, panels=2, s_max=60.0, max_refl=3)
    assert list(tab["ray_ptr"]) == [0, 2]
    assert tab["seg_hi"][0] == 20.0
    assert list(tab["face_ids"]) == [1 + 4 * 4 + 0]
    assert np.allclose(tab["seg_t"][1], [0.0, 0.0, 1.0])
    tab2 = ot.trace(np.array([[18.0, 4.0, 30.0]]), dirs, np.ones(1), boxes=box, panels=2, s_max=60.0,
                    max_refl=3)
    assert list(tab2["face_ids"]) == [1 + 4 * 4 + 1 * 2 + 1]


def test_reflection_budget_ends_the_path():
    """Between two parallel walls a ray bounces until R_max, then runs out
    its arc length on the last segment."""
    boxes = np.array([[-20.0, -10.0, -50.0, 50.0, 30.0], [10.0, 20.0, -50.0, 50.0, 30.0]])
    tab = ot.trace(np.array([[0.0, 0.0, 5.0]]), np.array([[1.0, 0.0, 0.0]]), np.ones(1), boxes=boxes,
                   s_max=1000.0, max_refl=5)
    assert list(tab["ray_ptr"]) == [0, 6]
    # box 1's -x wall (face 1 + 5 + 0), box 0's +x wall (face 1 + 0 + 1), ...
    assert list(tab["face_ids"][tab["face_ptr"][5]:]) == [6, 2, 6, 2, 6]
    assert tab["seg_s0"][5] == 90.0 and tab["seg_hi"][5] == 910.0


def test_open_plane_image_completion():
    """No boxes: every ray has its direct segment and either the ground
    reflection or the completed image segment; both lines pass through the
    image source (0, 0, -h)."""
    d, w = fibonacci_fan(300)
    src = np.array([[0.0, 0.0, 10.0]])
    tab = ot.trace(src, d, w, s_max=300.0, max_refl=4, image_complete=True)
    assert np.all(np.diff(tab["ray_ptr"]) == 2)
    second = tab["ray_ptr"][:-1] + 1
    virt = tab["seg_a"][second] - tab["seg_s0"][second][:, None] * tab["seg_t"][second]
    assert np.allclose(virt, [0.0, 0.0, -10.0], atol=1e-9)
    assert np.array_equal(np.diff(tab["face_ptr"]), np.tile([0, 1], 300))
    assert np.all(tab["face_ids"] == 0)
    # the two beams of a ray span the whole budget: direct [0, s_max), second [-s0, s_max - s0)
    assert np.allclose(tab["seg_hi"][second - 1], 300.0)
    assert np.allclose(tab["seg_s0"][second] + tab["seg_lo"][second], 0.0, atol=1e-12)
    assert np.allclose(tab["seg_s0"][second] + tab["seg_hi"][second], 300.0, atol=1e-9)
    with pytest.raises(ValueError):
        ot.trace(src, d, w, boxes=np.array([[1.0, 2.0, 1.0, 2.0, 3.0]]), s_max=10.0, image_complete=True)


def _same_table(ref, tab):
    for k in ("ray_ptr", "seg_a", "seg_t", "seg_s0", "seg_lo", "seg_hi", "face_ptr", "face_ids"):
        assert np.array_equal(np.asarray(ref[k]), np.asarray(getattr(tab, k))), k


def test_input_generator_agrees_with_the_oracle():
    """The vectorised tracer that writes the summation inputs produces the
    oracle's table bit for bit (city with panels, and the open plane)."""
    city = grid_city(3, 40.0, 20.0, 10.0, 40.0, seed=3, panels=2)
    d, w = fibonacci_fan(500)
    src = np.array([50.0, 110.0, 4.0])
    ref = ot.trace(src[None], d, w, boxes=city.boxes, panels=2, s_max=400.0, max_refl=5)
    _same_table(ref, trace_city(src, d, w, city, 400.0, 5))
    ref = ot.trace(np.array([[0.0, 0.0, 10.0]]), d, w, s_max=200.0, max_refl=1, image_complete=True)
    tab = trace_open_plane(np.array([0.0, 0.0, 10.0]), d, w, 200.0, policy="EC")
    # the open-plane generator writes the direct segment's extent as s_max
    # directly; the general tracer adds the two lengths (equal to rounding)
    assert np.allclose(ref["seg_hi"], tab.seg_hi, rtol=1e-15, atol=0)
    ref["seg_hi"] = tab.seg_hi
    _same_table(ref, tab)


def test_per_source_budgets():
    """A budget per source: each ray's path ends at its own source's s_max,
    and a single source's rays match a one-source trace exactly."""
    city = grid_city(2, 40.0, 20.0, 10.0, 40.0, seed=4)
    src = np.array([[30.0, 30.0, 5.0], [90.0, 40.0, 8.0]])
    d, w = fibonacci_fan(120)
    rs = np.repeat(np.arange(2, dtype=np.int32), 60)
    tab = ot.trace(src, np.concatenate([d[:60], d[60:]]), w, ray_src=rs, boxes=city.boxes, s_max=[200.0, 333.0],
                   max_refl=4)
    last = tab["ray_ptr"][1:] - 1
    np.testing.assert_allclose(tab["seg_s0"][last] + tab["seg_hi"][last], np.array([200.0, 333.0])[rs],
                               rtol=1e-12)
    one = ot.trace(src[1:], d[60:], w[60:], boxes=city.boxes, s_max=333.0, max_refl=4)
    k0 = tab["ray_ptr"][60]
    for key in ("seg_a", "seg_t", "seg_s0", "seg_lo", "seg_hi"):
        assert np.array_equal(tab[key][k0:], one[key]), key


def test_frame_transport_matches_the_history_rule():
    """The oracle tracer's frame, mirrored at every reflection along the path,
    equals the launch frame with the components flipped by the parity of the
    face normals in each segment's history (an independent construction from
    the finished table), and stays a unit vector normal to every axis."""
    from scenes import fibonacci_fan, grid_city, normal_frame
    from scenes.tracer import face_normal_axis
    city = grid_city(2, 40.0, 20.0, 10.0, 40.0, seed=3, panels=2)
    d, w = fibonacci_fan(300)
    psi = np.random.default_rng(2).uniform(0, np.pi, len(d))
    h = normal_frame(d)
    e0 = np.cos(psi)[:, None] * h + np.sin(psi)[:, None] * np.cross(d, h)
    tab = ot.trace(np.array([[50.0, 50.0, 6.0]]), d, w, boxes=city.boxes, panels=2, s_max=300.0, max_refl=5, e1=e0)
    e = tab["seg_e1"]
    lens = np.diff(tab["ray_ptr"])
    expect = e0[np.repeat(np.arange(len(d)), lens)].copy()
    flips = np.zeros((len(e), 3), np.int64)
    seg_of_face = np.repeat(np.arange(len(e)), np.diff(tab["face_ptr"]))
    np.add.at(flips, (seg_of_face, face_normal_axis(tab["face_ids"], 2)), 1)
    expect *= np.where(flips % 2 == 1, -1.0, 1.0)
    assert np.array_equal(e, expect)
    assert np.abs((e * tab["seg_t"]).sum(1)).max() <= 1e-14
    assert (np.diff(tab["face_ptr"]) >= 2).any()
    # the open plane's image segments carry the launch frame mirrored in z = 0
    tab2 = ot.trace(np.array([[0.0, 0.0, 10.0]]), d, w, s_max=200.0, max_refl=1, image_complete=True, e1=e0)
    two = np.where(np.diff(tab2["ray_ptr"]) == 2)[0]
    img = tab2["ray_ptr"][two] + 1
    assert np.array_equal(tab2["seg_e1"][img], e0[two] * np.array([1.0, 1.0, -1.0]))
