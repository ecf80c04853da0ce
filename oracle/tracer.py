"""FP64 CPU oracle of the ray-tracing stage: one ray at a time, plain Python.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may use this module; the library under test never does.

Gaussian beam tracing runs in two stages (paper Sec. 3.1): ray tracing (RT)
finds each ray's propagation path and the faces it reflects from, then beam
summation (GBS) adds the beams up at the observers.  Sec. 3.3 gives every ray
its own thread; here every ray is one iteration of a Python loop, and every
floating-point step is one IEEE double operation (no fused multiply-add), so
a device tracer that performs the same operations in the same order produces
the same bits.

What is traced (the paper leaves the environment model open; these are the
readings used throughout):
  * the ground plane z = 0 is face 0; buildings are axis-aligned boxes
    (x0, x1, y0, y1, height) standing on it, each with four walls (-x, +x,
    -y, +y) and a roof, every face split into panels x panels cells;
  * reflection is specular: the component of the direction along the face
    normal flips sign (image-source geometry, Sec. 1);
  * a ray reflects at most R_max times (Tables 2 and 3) and ends when its
    arc length reaches s_max;
  * a box is found by the slab test on its three coordinate intervals; a
    hit needs an entry distance greater than EPS (no self-hits), the entry
    axis is the first coordinate whose slab entry equals the entry distance,
    and a box is never entered through its floor;
  * the ground wins ties with a box at equal distance; between boxes at
    equal distance the lower box index wins.

The beam extent of every segment (its interval [lo, hi) along the axis) and
the face history follow the table conventions of the beam summation:
  * walls and roofs truncate a beam at the reflection point (lo = 0, hi = L);
  * the ground is transparent for the extent: a segment that ends on the
    ground extends by the length of the next one (hi = L + L_next) and the
    segment that starts there reaches back by the previous one's length
    (lo = -L_prev);
  * face history of segment j = the end faces of segments 0..j-1;
  * image completion (open plane only, no boxes): a ray that never reflects
    from the ground gets a second, virtual segment from the image source
    (source mirrored in z = 0) along the mirrored direction, with lo = 0,
    hi = s_max and face history [0].

With a launch frame per ray (the unit vector e1 normal to the launch
direction along which an anisotropic beam has its first width), each
segment also carries that frame transported along the path: a specular
reflection mirrors e1 in the face's plane like the direction, flipping the
same component (an exact sign change); the image segment carries the launch
frame mirrored in z = 0.
"""
from __future__ import annotations

import math

import numpy as np

EPS = 1e-7          # minimum hit distance after a reflection (m)
INF = math.inf


def _slab(p, d, lo_b, hi_b):
    """Entry/exit distances of the ray p + t d through the box [lo_b, hi_b]
    (per axis: the interval of t inside the slab), the entry distance, the
    exit distance and the per-axis entry values."""
    tmin = [0.0, 0.0, 0.0]
    tmax = [0.0, 0.0, 0.0]
    for j in range(3):
        if d[j] == 0.0:
            inside = lo_b[j] <= p[j] <= hi_b[j]
            tmin[j] = -INF if inside else INF
            tmax[j] = INF if inside else -INF
        else:
            inv = 1.0 / d[j]
            t1 = (lo_b[j] - p[j]) * inv
            t2 = (hi_b[j] - p[j]) * inv
            tmin[j] = t1 if t1 < t2 else t2
            tmax[j] = t1 if t1 > t2 else t2
    tnear = max(max(tmin[0], tmin[1]), tmin[2])
    tfar = min(min(tmax[0], tmax[1]), tmax[2])
    return tnear, tfar, tmin


def _face_id(box_idx, box, axis, side, hit, panels):
    """Face index of a hit: 0 is the ground; box b owns 5 * panels^2 faces
    starting at 1 + b * 5 * panels^2, walls -x, +x, -y, +y then the roof."""
    x0, x1, y0, y1, h = box
    if axis == 0:
        wall = 0 if side == 0 else 1
    elif axis == 1:
        wall = 2 if side == 0 else 3
    else:
        wall = 4
    cell = 0
    if panels > 1:
        u = (hit[1] - y0) / (y1 - y0) if axis == 0 else (hit[0] - x0) / (x1 - x0)
        v = (hit[1] - y0) / (y1 - y0) if axis == 2 else hit[2] / h
        iu = min(max(int(u * panels), 0), panels - 1)
        iv = min(max(int(v * panels), 0), panels - 1)
        cell = iu * panels + iv
    return 1 + box_idx * 5 * panels * panels + wall * panels * panels + cell


def trace_ray(src, d0, boxes, panels, s_max, max_refl, e0=(0.0, 0.0, 0.0)):
    """Path of one ray: a list of segments (a, t, s0, L, end_face, ends_on_ground,
    e); end_face is -1 for the last segment; e is the launch frame e0
    transported to the segment."""
    p = [float(src[0]), float(src[1]), float(src[2])]
    d = [float(d0[0]), float(d0[1]), float(d0[2])]
    e = [float(e0[0]), float(e0[1]), float(e0[2])]
    s = 0.0
    out = []
    for k in range(max_refl + 1):
        # the ground plane z = 0
        tg = -p[2] / d[2] if d[2] < 0.0 else INF
        if not tg > EPS:
            tg = INF
        best, best_box, best_axis, best_side = tg, -1, 0, 0
        if k < max_refl:
            for b, box in enumerate(boxes):
                x0, x1, y0, y1, h = (float(v) for v in box)
                tnear, tfar, tmin = _slab(p, d, (x0, y0, 0.0), (x1, y1, h))
                if not (tnear <= tfar and tnear > EPS):
                    continue
                if tmin[0] >= tmin[1] and tmin[0] >= tmin[2]:
                    axis = 0
                elif tmin[1] >= tmin[2]:
                    axis = 1
                else:
                    axis = 2
                if axis == 2 and d[2] > 0.0:
                    continue                       # through the floor: not a hit
                if tnear < best:                   # strict: ground and lower index win ties
                    best, best_box, best_axis = tnear, b, axis
                    best_side = 0 if d[axis] > 0.0 else 1
        remaining = s_max - s
        ends = best >= remaining or k == max_refl
        L = remaining if ends else best
        hp = [p[0] + L * d[0], p[1] + L * d[1], p[2] + L * d[2]]
        ground = (not ends) and best_box < 0
        if ends:
            face = -1
        elif ground:
            face = 0
        else:
            face = _face_id(best_box, tuple(float(v) for v in boxes[best_box]), best_axis, best_side, hp, panels)
        out.append((tuple(p), tuple(d), s, L, face, ground, tuple(e)))
        if ends:
            break
        axis = 2 if ground else best_axis
        d[axis] = -d[axis]
        e[axis] = -e[axis]
        if ground:
            hp[2] = 0.0
        p = hp
        s = s + L
    return out


def ray_segments(src, d0, boxes, panels, s_max, max_refl, image_complete, e0=(0.0, 0.0, 0.0)):
    """Table rows of one ray: a list of (a, t, s0, lo, hi, face_history, e1)."""
    path = trace_ray(src, d0, boxes, panels, s_max, max_refl, e0)
    rows = []
    for j, (a, t, s0, L, _face, ground, e) in enumerate(path):
        lo, hi = 0.0, L
        if ground and j + 1 < len(path):
            hi = L + path[j + 1][3]
        if j > 0 and path[j - 1][5]:
            lo = -path[j - 1][3]
        rows.append((a, t, s0, lo, hi, [path[m][4] for m in range(j)], e))
    if image_complete and not any(seg[5] for seg in path):
        img = (float(src[0]), float(src[1]), -float(src[2]))
        tm = (float(d0[0]), float(d0[1]), -float(d0[2]))
        em = (float(e0[0]), float(e0[1]), -float(e0[2]))
        rows.append((img, tm, 0.0, 0.0, float(s_max), [0], em))
    return rows


def trace(src_xyz, dirs, weights, ray_src=None, boxes=None, panels=1, s_max=1.0, max_refl=10,
          image_complete=False, rays=None, e1=None):
    """Ray table (dict of numpy arrays in the beam-summation table layout)
    of the given rays, or of the subset `rays` (indices, kept in order).
    s_max: one arc-length budget, or one per source.  e1: launch frame per
    ray ([n_rays, 3]); the table then also holds seg_e1, the frame carried to
    every segment."""
    src_xyz = np.asarray(src_xyz, np.float64).reshape(-1, 3)
    dirs = np.asarray(dirs, np.float64).reshape(-1, 3)
    weights = np.asarray(weights, np.float64).reshape(-1)
    ray_src = np.zeros(len(dirs), np.int32) if ray_src is None else np.asarray(ray_src, np.int32)
    boxes = np.zeros((0, 5)) if boxes is None else np.asarray(boxes, np.float64).reshape(-1, 5)
    if image_complete and len(boxes):
        raise ValueError("image completion is defined for the open plane only")
    idx = np.arange(len(dirs)) if rays is None else np.asarray(rays, np.int64)
    s_max_src = np.broadcast_to(np.asarray(s_max, np.float64), (len(src_xyz),))
    frames = None if e1 is None else np.asarray(e1, np.float64).reshape(-1, 3)
    ray_ptr, face_ptr = [0], [0]
    A, T, S0, LO, HI, F, E = [], [], [], [], [], [], []
    for i in idx:
        e0 = (0.0, 0.0, 0.0) if frames is None else frames[i]
        for a, t, s0, lo, hi, hist, e in ray_segments(src_xyz[ray_src[i]], dirs[i], boxes, panels,
                                                      float(s_max_src[ray_src[i]]), max_refl, image_complete, e0):
            E.append(e)
            A.append(a)
            T.append(t)
            S0.append(s0)
            LO.append(lo)
            HI.append(hi)
            F.extend(hist)
            face_ptr.append(face_ptr[-1] + len(hist))
        ray_ptr.append(len(S0))
    n_faces = 1 + len(boxes) * 5 * panels * panels
    out = dict(src_xyz=src_xyz.copy(), ray_ptr=np.asarray(ray_ptr, np.int64), ray_w=weights[idx].copy(),
               ray_src=ray_src[idx].copy(), seg_a=np.asarray(A, np.float64).reshape(-1, 3),
               seg_t=np.asarray(T, np.float64).reshape(-1, 3), seg_s0=np.asarray(S0, np.float64),
               seg_lo=np.asarray(LO, np.float64), seg_hi=np.asarray(HI, np.float64),
               face_ptr=np.asarray(face_ptr, np.int64), face_ids=np.asarray(F, np.int32), n_faces=n_faces)
    if frames is not None:
        out["seg_e1"] = np.asarray(E, np.float64).reshape(-1, 3)
    return out
