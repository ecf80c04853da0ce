"""Seeded CPU ray tracer that writes the ray table consumed by beam summation.

This module is an input generator.  It performs the ray-tracing (RT) stage
that precedes Gaussian beam summation (paper Sec. 3.1, Fig. 2: rays are traced
first, their paths and reflections are stored, and only then are beams summed
at the observers).  It holds none of the summation arithmetic: it writes
straight segments, their arc-length bookkeeping, the faces each ray has hit and
the solid angle each ray represents.  Both the oracle and the HIP library read
the table it produces as plain data.

Ray table layout (all numpy, float64 unless noted):

  src_xyz  [n_src, 3]        source positions
  ray_ptr  [n_rays + 1] i64  CSR: segments of ray i are ray_ptr[i]:ray_ptr[i+1]
  ray_w    [n_rays]          solid angle of each ray's launch cell (sr)
  ray_src  [n_rays] i32      source index of each ray, non-decreasing
  seg_a    [n_segs, 3]       segment start point
  seg_t    [n_segs, 3]       unit direction of the segment's axis
  seg_s0   [n_segs]          arc length from the (virtual) source at seg_a
  seg_lo   [n_segs]          beam interval start, in sigma = (R - a).t
  seg_hi   [n_segs]          beam interval end (exclusive)
  face_ptr [n_segs + 1] i64  CSR into face_ids: faces hit before the segment
  face_ids [nnz] i32         face indices, in hit order

Extent policy (the segment interval [lo, hi)):
  * finite faces (walls, roofs) truncate a beam at the reflection point;
  * the ground plane is treated as transparent for the beam extent: a segment
    that ends on the ground keeps its beam up to the end of the reflected
    segment, and the reflected segment reaches back to the start of the
    incoming one, so the pair reproduces the image-source field near the
    reflection point;
  * "EC" (open plane only) also completes the image fan: every ray that never
    reaches the ground gets a virtual mirrored segment launched from the image
    source, carrying the ground's reflection coefficient.  The direct fan and
    the image fan are then both complete spheres of rays.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

GOLDEN_ANGLE = np.pi * (3.0 - np.sqrt(5.0))


@dataclass
class RayTable:
    src_xyz: np.ndarray
    ray_ptr: np.ndarray
    ray_w: np.ndarray
    ray_src: np.ndarray
    seg_a: np.ndarray
    seg_t: np.ndarray
    seg_s0: np.ndarray
    seg_lo: np.ndarray
    seg_hi: np.ndarray
    face_ptr: np.ndarray
    face_ids: np.ndarray
    n_faces: int
    meta: dict = field(default_factory=dict)

    @property
    def n_src(self) -> int:
        return int(self.src_xyz.shape[0])

    @property
    def n_rays(self) -> int:
        return int(self.ray_w.shape[0])

    @property
    def n_segs(self) -> int:
        return int(self.seg_s0.shape[0])

    def validate(self) -> None:
        """Structural checks on the table (raises ValueError)."""
        n_rays, n_segs = self.n_rays, self.n_segs
        if self.ray_ptr.shape != (n_rays + 1,) or self.ray_ptr[0] != 0 or self.ray_ptr[-1] != n_segs:
            raise ValueError("ray_ptr is not a CSR over the segments")
        if np.any(np.diff(self.ray_ptr) < 0):
            raise ValueError("ray_ptr not monotone")
        if np.any(np.diff(self.ray_src) < 0):
            raise ValueError("rays must be sorted by source")
        if n_rays and (self.ray_src.min() < 0 or self.ray_src.max() >= self.n_src):
            raise ValueError("ray_src out of range")
        tn = np.linalg.norm(self.seg_t, axis=1)
        if n_segs and np.max(np.abs(tn - 1.0)) > 1e-9:
            raise ValueError("segment directions are not unit vectors")
        if np.any(self.seg_lo > self.seg_hi):
            raise ValueError("lo > hi")
        if self.face_ptr.shape != (n_segs + 1,) or self.face_ptr[0] != 0 or self.face_ptr[-1] != self.face_ids.shape[0]:
            raise ValueError("face_ptr is not a CSR over face_ids")
        if self.face_ids.size and (self.face_ids.min() < 0 or self.face_ids.max() >= self.n_faces):
            raise ValueError("face id out of range")

    def subset_rays(self, ray_idx) -> "RayTable":
        """Table restricted to the given rays (kept in the given order)."""
        ray_idx = np.asarray(ray_idx, dtype=np.int64)
        lens = self.ray_ptr[ray_idx + 1] - self.ray_ptr[ray_idx]
        seg_idx = np.concatenate([np.arange(self.ray_ptr[i], self.ray_ptr[i + 1]) for i in ray_idx]) \
            if len(ray_idx) else np.zeros(0, np.int64)
        flens = self.face_ptr[seg_idx + 1] - self.face_ptr[seg_idx]
        fidx = np.concatenate([np.arange(self.face_ptr[j], self.face_ptr[j + 1]) for j in seg_idx]) \
            if len(seg_idx) else np.zeros(0, np.int64)
        return RayTable(
            src_xyz=self.src_xyz.copy(),
            ray_ptr=np.concatenate([[0], np.cumsum(lens)]).astype(np.int64),
            ray_w=self.ray_w[ray_idx].copy(),
            ray_src=self.ray_src[ray_idx].copy(),
            seg_a=self.seg_a[seg_idx].copy(), seg_t=self.seg_t[seg_idx].copy(),
            seg_s0=self.seg_s0[seg_idx].copy(), seg_lo=self.seg_lo[seg_idx].copy(),
            seg_hi=self.seg_hi[seg_idx].copy(),
            face_ptr=np.concatenate([[0], np.cumsum(flens)]).astype(np.int64),
            face_ids=self.face_ids[fidx].astype(np.int32),
            n_faces=self.n_faces, meta=dict(self.meta))

    @staticmethod
    def concat(tables) -> "RayTable":
        """Stack tables of distinct sources into one multi-source table."""
        src = np.concatenate([t.src_xyz for t in tables])
        ray_ptr = [np.zeros(1, np.int64)]
        face_ptr = [np.zeros(1, np.int64)]
        seg_off = 0
        face_off = 0
        src_off = 0
        ray_src = []
        for t in tables:
            ray_ptr.append(t.ray_ptr[1:] + seg_off)
            face_ptr.append(t.face_ptr[1:] + face_off)
            ray_src.append(t.ray_src + src_off)
            seg_off += t.n_segs
            face_off += int(t.face_ids.shape[0])
            src_off += t.n_src
        n_faces = max(t.n_faces for t in tables)
        return RayTable(
            src_xyz=src, ray_ptr=np.concatenate(ray_ptr), ray_w=np.concatenate([t.ray_w for t in tables]),
            ray_src=np.concatenate(ray_src).astype(np.int32),
            seg_a=np.concatenate([t.seg_a for t in tables]), seg_t=np.concatenate([t.seg_t for t in tables]),
            seg_s0=np.concatenate([t.seg_s0 for t in tables]), seg_lo=np.concatenate([t.seg_lo for t in tables]),
            seg_hi=np.concatenate([t.seg_hi for t in tables]), face_ptr=np.concatenate(face_ptr),
            face_ids=np.concatenate([t.face_ids for t in tables]).astype(np.int32), n_faces=n_faces,
            meta={"parts": [t.meta for t in tables]})


# --------------------------------------------------------------------------
# Launch fans.  The paper launches rays over the full sphere of elevation and
# azimuth (Tables 2 and 3: elevation 0..180 degrees, azimuth 0..360 degrees).
# --------------------------------------------------------------------------

def fibonacci_fan(n: int):
    """Fibonacci sphere: z_i = 1 - (2i+1)/n, azimuth i * golden angle.

    Returns (dirs [n,3], weights [n]) with equal solid angle 4*pi/n per ray.
    """
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * GOLDEN_ANGLE
    d = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d, np.full(n, 4.0 * np.pi / n)


def theta_phi_fan(n_theta: int, n_phi: int):
    """Product fan: polar cell centres theta_i = (i + 1/2) pi / n_theta,
    azimuths phi_m = 2 pi m / n_phi.  Weight = sin(theta) dtheta dphi.

    The fan is invariant under rotation by 2 pi / n_phi about the z axis and
    under the mirror phi -> -phi, which the symmetry tests rely on.
    """
    th = (np.arange(n_theta) + 0.5) * np.pi / n_theta
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    st = np.sin(T)
    d = np.stack([st * np.cos(Ph), st * np.sin(Ph), np.cos(T)], axis=-1).reshape(-1, 3)
    w = (st * (np.pi / n_theta) * (2.0 * np.pi / n_phi)).reshape(-1)
    return d, w


# --------------------------------------------------------------------------
# Open plane: homogeneous medium above a flat ground z = 0 (face 0).
# --------------------------------------------------------------------------

def trace_open_plane(src, dirs, weights, s_max: float, policy: str = "EC") -> RayTable:
    """Trace a fan over a single reflecting ground plane z = 0.

    policy: "EC" (extend through the ground + image completion), "E" (extend
    only), "T" (truncate at the reflection point).  Every ray gets at most one
    ground reflection: in a homogeneous medium an up-going ray never returns.
    """
    src = np.asarray(src, dtype=np.float64)
    if src[2] <= 0:
        raise ValueError("source must be above the ground")
    n = dirs.shape[0]
    h = src[2]
    down = dirs[:, 2] < 0.0
    mirror = dirs * np.array([1.0, 1.0, -1.0])
    s_g = np.where(down, h / np.where(down, -dirs[:, 2], 1.0), np.inf)

    segs = []  # (ray, order, a, t, s0, lo, hi, faces)
    a0 = np.broadcast_to(src, (n, 3))
    if policy == "T":
        hi0 = np.where(down, np.minimum(s_g, s_max), s_max)
    else:
        hi0 = np.full(n, s_max)
    segs.append((np.arange(n), np.zeros(n, np.int64), a0, dirs, np.zeros(n), np.zeros(n), hi0, np.zeros(n, bool)))

    # real reflections
    idx = np.nonzero(down & (s_g < s_max))[0]
    g = src + s_g[idx, None] * dirs[idx]
    g[:, 2] = 0.0
    s0 = s_g[idx]
    lo = np.zeros_like(s0) if policy == "T" else -s0
    segs.append((idx, np.ones(len(idx), np.int64), g, mirror[idx], s0, lo, s_max - s0, np.ones(len(idx), bool)))

    if policy == "EC":
        img = src * np.array([1.0, 1.0, -1.0])
        idx2 = np.nonzero(~(down & (s_g < s_max)))[0]
        m = len(idx2)
        segs.append((idx2, np.ones(m, np.int64), np.broadcast_to(img, (m, 3)), mirror[idx2],
                     np.zeros(m), np.zeros(m), np.full(m, s_max), np.ones(m, bool)))

    ray = np.concatenate([s[0] for s in segs])
    order = np.concatenate([s[1] for s in segs])
    perm = np.lexsort((order, ray))
    cat = lambda k: np.concatenate([np.asarray(s[k], dtype=np.float64) for s in segs])[perm]
    seg_a = np.concatenate([np.asarray(s[2]) for s in segs])[perm]
    seg_t = np.concatenate([np.asarray(s[3]) for s in segs])[perm]
    hit_ground = np.concatenate([s[7] for s in segs])[perm]
    counts = np.bincount(ray, minlength=n)
    ray_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    face_ptr = np.concatenate([[0], np.cumsum(hit_ground.astype(np.int64))]).astype(np.int64)
    face_ids = np.zeros(int(face_ptr[-1]), np.int32)
    return RayTable(
        src_xyz=src[None, :].copy(), ray_ptr=ray_ptr, ray_w=np.asarray(weights, np.float64).copy(),
        ray_src=np.zeros(n, np.int32), seg_a=np.ascontiguousarray(seg_a, dtype=np.float64),
        seg_t=np.ascontiguousarray(seg_t, dtype=np.float64), seg_s0=cat(4), seg_lo=cat(5), seg_hi=cat(6),
        face_ptr=face_ptr, face_ids=face_ids, n_faces=1,
        meta={"kind": "open_plane", "policy": policy, "s_max": s_max})


# --------------------------------------------------------------------------
# City: ground plane plus axis-aligned box buildings with specular faces.
# --------------------------------------------------------------------------

@dataclass
class City:
    boxes: np.ndarray        # [B, 5]: x0, x1, y0, y1, height
    panels: int = 1          # faces split into panels x panels (1 or 2)

    @property
    def faces_per_box(self) -> int:
        return 5 * self.panels * self.panels

    @property
    def n_faces(self) -> int:
        return 1 + self.boxes.shape[0] * self.faces_per_box


def grid_city(n: int, footprint: float, street: float, h_lo: float, h_hi: float, seed: int,
              panels: int = 1) -> City:
    """n x n blocks of footprint x footprint, separated by `street`; the first
    block starts at x = street.  Heights drawn U(h_lo, h_hi) with the seed."""
    rng = np.random.default_rng(seed)
    pitch = footprint + street
    boxes = []
    for i in range(n):
        for j in range(n):
            x0 = street + pitch * i
            y0 = street + pitch * j
            boxes.append([x0, x0 + footprint, y0, y0 + footprint, 0.0])
    boxes = np.array(boxes)
    boxes[:, 4] = rng.uniform(h_lo, h_hi, size=len(boxes))
    return City(boxes=boxes, panels=panels)


def _box_face_id(city: City, b, axis, side, hit):
    """Face index of a hit on box b.  Faces: 0 ground; per box walls
    (-x, +x, -y, +y) then roof, each split into panels x panels cells."""
    P = city.panels
    bx = city.boxes[b]
    x0, x1, y0, y1, h = bx[:, 0], bx[:, 1], bx[:, 2], bx[:, 3], bx[:, 4]
    wall = np.where(axis == 0, np.where(side == 0, 0, 1), np.where(axis == 1, np.where(side == 0, 2, 3), 4))
    if P == 1:
        cell = np.zeros_like(wall)
    else:
        # along-wall coordinate u and height/second coordinate v, each split in halves
        u = np.where(axis == 0, (hit[:, 1] - y0) / (y1 - y0), (hit[:, 0] - x0) / (x1 - x0))
        v = np.where(axis == 2, (hit[:, 1] - y0) / (y1 - y0), hit[:, 2] / h)
        iu = np.clip((u * P).astype(np.int64), 0, P - 1)
        iv = np.clip((v * P).astype(np.int64), 0, P - 1)
        cell = iu * P + iv
    return 1 + b * city.faces_per_box + wall * P * P + cell


_TRACE_CHUNK = 16384


def _nearest_box(B, p, dd, eps, best, best_box, best_axis, best_side):
    """Slab test of rays (p, dd) against every box; updates, in place, the
    nearest hit closer than `best` (distance, box, axis and side of entry).
    Works on one coordinate at a time (1-D arrays are much faster to reduce)."""
    P = [np.ascontiguousarray(p[:, j]) for j in range(3)]
    D = [np.ascontiguousarray(dd[:, j]) for j in range(3)]
    with np.errstate(divide="ignore"):
        inv = [np.where(D[j] != 0, 1.0 / np.where(D[j] != 0, D[j], 1.0), np.inf) for j in range(3)]
    par = [D[j] == 0 for j in range(3)]
    up = D[2] > 0
    for b in range(B.shape[0]):
        x0, x1, y0, y1, hb = B[b]
        lo_b = (x0, y0, 0.0)
        hi_b = (x1, y1, hb)
        tmin, tmax = [], []
        with np.errstate(invalid="ignore", over="ignore"):
            for j in range(3):
                t1 = (lo_b[j] - P[j]) * inv[j]
                t2 = (hi_b[j] - P[j]) * inv[j]
                # rays parallel to a slab: inside -> (-inf, inf), outside -> empty
                inside = (P[j] >= lo_b[j]) & (P[j] <= hi_b[j])
                tmin.append(np.where(par[j], np.where(inside, -np.inf, np.inf), np.minimum(t1, t2)))
                tmax.append(np.where(par[j], np.where(inside, np.inf, -np.inf), np.maximum(t1, t2)))
        tnear = np.maximum(np.maximum(tmin[0], tmin[1]), tmin[2])
        tfar = np.minimum(np.minimum(tmax[0], tmax[1]), tmax[2])
        hit = (tnear <= tfar) & (tnear > eps) & (tnear < best)
        if not np.any(hit):
            continue
        # entry axis: the first coordinate attaining tnear
        axis = np.where((tmin[0] >= tmin[1]) & (tmin[0] >= tmin[2]), 0, np.where(tmin[1] >= tmin[2], 1, 2))
        # a box is never entered from below: z = 0 is the ground
        hit &= ~((axis == 2) & up)
        if np.any(hit):
            best[hit] = tnear[hit]
            best_box[hit] = b
            best_axis[hit] = axis[hit]
            d_ax = np.where(axis == 0, D[0], np.where(axis == 1, D[1], D[2]))
            best_side[hit] = np.where(d_ax > 0, 0, 1)[hit]


def trace_city(src, dirs, weights, city: City, s_max: float, max_refl: int) -> RayTable:
    """Specular tracing among boxes and the ground plane, up to max_refl
    reflections; the path ends at arc length s_max.  Walls and roofs truncate
    the beam interval; ground reflections extend it (see the module doc)."""
    src = np.asarray(src, dtype=np.float64)
    n = dirs.shape[0]
    B = city.boxes
    eps = 1e-7

    pos = np.broadcast_to(src, (n, 3)).copy()
    d = dirs.astype(np.float64).copy()
    s = np.zeros(n)
    alive = np.ones(n, bool)
    rec = []  # per bounce: (ray, k, a, t, s0, L, end_face, end_is_ground)
    for k in range(max_refl + 1):
        ids = np.nonzero(alive)[0]
        if len(ids) == 0:
            break
        p = pos[ids]
        dd = d[ids]
        best = np.full(len(ids), np.inf)
        best_box = np.full(len(ids), -1, np.int64)
        best_axis = np.zeros(len(ids), np.int64)
        best_side = np.zeros(len(ids), np.int64)
        # ground
        with np.errstate(divide="ignore", invalid="ignore"):
            tg = np.where(dd[:, 2] < 0, -p[:, 2] / dd[:, 2], np.inf)
        tg = np.where(tg > eps, tg, np.inf)
        best = tg.copy()
        if k < max_refl:
            # in chunks of rays so that the per-box temporaries stay in cache
            for c0 in range(0, len(ids), _TRACE_CHUNK):
                c1 = min(c0 + _TRACE_CHUNK, len(ids))
                _nearest_box(B, p[c0:c1], dd[c0:c1], eps, best[c0:c1], best_box[c0:c1], best_axis[c0:c1],
                             best_side[c0:c1])
        remaining = s_max - s[ids]
        ends = (best >= remaining) | (k == max_refl)
        L = np.where(ends, remaining, best)
        hp = p + L[:, None] * dd
        is_ground = (~ends) & (best_box < 0)
        face = np.full(len(ids), -1, np.int64)
        face[is_ground] = 0
        wb = (~ends) & (best_box >= 0)
        if np.any(wb):
            face[wb] = _box_face_id(city, best_box[wb], best_axis[wb], best_side[wb], hp[wb])
        rec.append((ids, np.full(len(ids), k), p.copy(), dd.copy(), s[ids].copy(), L, face, is_ground))
        # reflect and advance
        cont = ~ends
        nd = dd.copy()
        ax = np.where(is_ground, 2, best_axis)
        rows = np.nonzero(cont)[0]
        nd[rows, ax[rows]] *= -1.0
        hp[is_ground, 2] = 0.0
        pos[ids] = hp
        d[ids] = nd
        s[ids] = s[ids] + L
        alive[ids[ends]] = False

    ray = np.concatenate([r[0] for r in rec])
    kk = np.concatenate([r[1] for r in rec])
    perm = np.lexsort((kk, ray))
    ray = ray[perm]
    kk = kk[perm]
    A = np.concatenate([r[2] for r in rec])[perm]
    T = np.concatenate([r[3] for r in rec])[perm]
    S0 = np.concatenate([r[4] for r in rec])[perm]
    L = np.concatenate([r[5] for r in rec])[perm]
    F = np.concatenate([r[6] for r in rec])[perm]
    G = np.concatenate([r[7] for r in rec])[perm]
    counts = np.bincount(ray, minlength=n)
    ray_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    nseg = len(ray)
    lo = np.zeros(nseg)
    hi = L.copy()
    first = np.zeros(nseg, bool)
    first[ray_ptr[:-1][counts > 0]] = True
    # ground chains: a segment ending on the ground extends through the next one;
    # a segment starting on the ground reaches back to the start of the previous.
    ends_ground = G
    nxt = np.arange(nseg) + 1
    has_next = np.zeros(nseg, bool)
    has_next[:-1] = ray[1:] == ray[:-1]
    e = np.nonzero(ends_ground & has_next)[0]
    hi[e] = L[e] + L[nxt[e]]
    starts_ground = np.zeros(nseg, bool)
    starts_ground[1:] = ends_ground[:-1] & (ray[1:] == ray[:-1])
    sg = np.nonzero(starts_ground)[0]
    lo[sg] = -L[sg - 1]
    # face history: faces hit before each segment (end faces of the previous ones)
    hist_len = kk.astype(np.int64)
    face_ptr = np.concatenate([[0], np.cumsum(hist_len)]).astype(np.int64)
    total = int(face_ptr[-1])
    within = np.arange(total, dtype=np.int64) - np.repeat(face_ptr[:-1], hist_len)
    src_seg = np.repeat(np.arange(nseg, dtype=np.int64) - hist_len, hist_len) + within
    face_ids = F[src_seg].astype(np.int32)
    return RayTable(
        src_xyz=src[None, :].copy(), ray_ptr=ray_ptr, ray_w=np.asarray(weights, np.float64).copy(),
        ray_src=np.zeros(n, np.int32), seg_a=np.ascontiguousarray(A), seg_t=np.ascontiguousarray(T),
        seg_s0=S0, seg_lo=lo, seg_hi=hi, face_ptr=face_ptr, face_ids=face_ids, n_faces=city.n_faces,
        meta={"kind": "city", "s_max": s_max, "max_refl": max_refl})


def normal_frame(t, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Unit vector e1 normal to each axis t ([n, 3]): up x t normalised, or,
    where t is parallel to `up`, the coordinate axis least aligned with t made
    normal to it.  With the default up = z this is the horizontal normal
    (-t_y, t_x, 0) / |(t_x, t_y)|, which a reflection on a vertical wall, a roof
    or the ground maps to plus or minus the horizontal normal of the reflected
    axis: the frame of anisotropic beams in the box scenes."""
    t = np.asarray(t, np.float64).reshape(-1, 3)
    u = np.broadcast_to(np.asarray(up, np.float64), t.shape)
    e = np.cross(u, t)
    n = np.linalg.norm(e, axis=1)
    bad = ~(n > 0.0)
    if bad.any():
        ax = np.eye(3)[np.argmin(np.abs(t[bad]), axis=1)]
        e[bad] = ax - (ax * t[bad]).sum(1, keepdims=True) * t[bad]
        n[bad] = np.linalg.norm(e[bad], axis=1)
    return e / n[:, None]


def face_normal_axis(face_ids, panels: int = 1) -> np.ndarray:
    """Coordinate axis of each face's normal in the box scenes: z (2) for the
    ground (face 0) and the roofs, x (0) for the -x and +x walls, y (1) for
    the -y and +y walls (face layout of _box_face_id)."""
    f = np.asarray(face_ids, np.int64)
    wall = ((f - 1) // (panels * panels)) % 5
    ax = np.where(wall < 2, 0, np.where(wall < 4, 1, 2))
    return np.where(f == 0, 2, ax)


def transported_frame(table: RayTable, psi=0.0, panels: int = 1) -> np.ndarray:
    """The ray frame of anisotropic beams carried along every ray ([n_segs, 3]).

    At launch e1 = cos(psi) h + sin(psi) (t x h), with t the ray's first axis
    and h = normal_frame(t) (psi, one value or one per ray, turns the frame
    onto the principal axes of the beam's initial width matrix); at every
    reflection e1 is mirrored in the face's plane like the axis itself, so it
    stays a unit vector normal to the axis.  The box scenes' faces are normal
    to a coordinate axis: a mirror flips that component of e1, and segment j
    carries the flips of the faces in its history (the open plane's image
    segments carry the ground's)."""
    n_rays = table.n_rays
    lens = np.diff(table.ray_ptr)
    ray_of_seg = np.repeat(np.arange(n_rays), lens)
    first = table.ray_ptr[:-1][lens > 0]
    t0 = np.zeros((n_rays, 3))
    t0[lens > 0] = table.seg_t[first]
    h = normal_frame(t0)
    ps = np.broadcast_to(np.asarray(psi, np.float64), (n_rays,))
    e0 = np.cos(ps)[:, None] * h + np.sin(ps)[:, None] * np.cross(t0, h)
    e = e0[ray_of_seg].copy()
    flen = np.diff(table.face_ptr)
    seg_of_face = np.repeat(np.arange(table.n_segs), flen)
    ax = face_normal_axis(table.face_ids, panels)
    flips = np.zeros((table.n_segs, 3), np.int64)
    np.add.at(flips, (seg_of_face, ax), 1)
    e *= np.where(flips % 2 == 1, -1.0, 1.0)
    return e


def rotate_table(table: RayTable, rot) -> RayTable:
    """The same table in coordinates turned by the rotation matrix `rot`
    (points and axes map by rot; arc lengths, intervals and histories are
    unchanged): e.g. an open plane over a tilted ground."""
    R = np.asarray(rot, np.float64)
    return RayTable(src_xyz=table.src_xyz @ R.T, ray_ptr=table.ray_ptr.copy(), ray_w=table.ray_w.copy(),
                    ray_src=table.ray_src.copy(), seg_a=table.seg_a @ R.T, seg_t=table.seg_t @ R.T,
                    seg_s0=table.seg_s0.copy(), seg_lo=table.seg_lo.copy(), seg_hi=table.seg_hi.copy(),
                    face_ptr=table.face_ptr.copy(), face_ids=table.face_ids.copy(), n_faces=table.n_faces,
                    meta=dict(table.meta))


def receiver_grid(nx: int, ny: int, x0: float, x1: float, y0: float, y1: float, z: float) -> np.ndarray:
    """Row-major grid (x fastest) of receivers at height z."""
    xs = x0 + (x1 - x0) * np.arange(nx) / max(nx - 1, 1)
    ys = y0 + (y1 - y0) * np.arange(ny) / max(ny - 1, 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1)


def inside_buildings(city: City, rcv: np.ndarray) -> np.ndarray:
    m = np.zeros(len(rcv), bool)
    for x0, x1, y0, y1, h in city.boxes:
        m |= (rcv[:, 0] > x0) & (rcv[:, 0] < x1) & (rcv[:, 1] > y0) & (rcv[:, 1] < y1) & (rcv[:, 2] < h)
    return m
