"""Seeded synthetic workloads for Gaussian beam summation.

The paper's own scenes (its city model and GIS inputs, Tables 2 and 3) are not
public, so these seeded synthetic scenes stand in for its "free field" (open
plane over a rigid ground) and "city" cases.  Each builder returns a Scene:
a ray table (data), receivers, band frequencies, the beam parameter epsilon
per (source, band) job and the reflection coefficient of every face.

Every builder takes scale-down arguments (ray count, receiver grid) so that
tests can run the same scene at sizes a CPU finishes in seconds.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .tracer import (City, RayTable, fibonacci_fan, grid_city, inside_buildings, receiver_grid,
                     trace_city, trace_open_plane)

C_AIR = 343.0
GATE_G = 9.21            # keep a pair while its Gaussian factor is >= exp(-9.21) ~ 1e-4
EPS_RULE_C = 6.0         # epsilon_b = C * sqrt(r_ref / k_b)
OCTAVES_8 = (63.0, 125.0, 250.0, 500.0, 1000.0, 2000.0, 4000.0, 8000.0)


@dataclass
class Scene:
    name: str
    table: RayTable
    rcv: np.ndarray                 # [n_rcv, 3] float64
    freqs: np.ndarray               # [n_freq] Hz
    eps: np.ndarray                 # [n_src, n_freq] beam parameter (m)
    gamma: np.ndarray               # [n_faces] complex128 reflection coefficients
    c: float = C_AIR
    gate: float = GATE_G
    meta: dict = field(default_factory=dict)

    @property
    def n_jobs(self) -> int:
        return self.table.n_src * len(self.freqs)

    @property
    def dense_pairs(self) -> int:
        """Segment x receiver x band evaluations a dense sum performs."""
        segs_per_src = np.bincount(self.table.ray_src, weights=np.diff(self.table.ray_ptr),
                                   minlength=self.table.n_src)
        return int(segs_per_src.sum()) * len(self.rcv) * len(self.freqs)


def eps_rule(freqs, r_ref: float, c: float = C_AIR, C: float = EPS_RULE_C) -> np.ndarray:
    """epsilon_b = C sqrt(r_ref / k_b): keeps the paraxial phase error, which
    grows like r / (k epsilon^2), small out to range r_ref."""
    k = 2.0 * np.pi * np.asarray(freqs, dtype=np.float64) / c
    return C * np.sqrt(r_ref / k)


def eps_literal(freqs, c: float = C_AIR, frac: float = 0.5) -> np.ndarray:
    """epsilon = frac * wavelength."""
    return frac * c / np.asarray(freqs, dtype=np.float64)


def open_plane(n_rays=2000, grid=64, half=100.0, src=(0.0, 0.0, 10.0), freqs=(500.0,),
               gamma_ground=1.0 + 0j, eps="rule", policy="EC", z_rcv=1.5, name="open_plane") -> Scene:
    """Homogeneous air (c = 343 m/s) above a reflecting ground z = 0 (face 0);
    Fibonacci fan from `src`; grid x grid receivers over [-half, half]^2."""
    rcv = receiver_grid(grid, grid, -half, half, -half, half, z_rcv)
    S = np.asarray(src, dtype=np.float64)
    img = S * np.array([1.0, 1.0, -1.0])
    r_ref = float(np.max(np.linalg.norm(rcv - img, axis=1)))
    s_max = 1.2 * r_ref
    d, w = fibonacci_fan(n_rays)
    table = trace_open_plane(S, d, w, s_max, policy=policy)
    freqs = np.asarray(freqs, dtype=np.float64)
    e = eps_rule(freqs, r_ref) if eps == "rule" else (eps_literal(freqs) if eps == "literal" else
                                                       np.broadcast_to(np.asarray(eps, float), freqs.shape))
    return Scene(name=name, table=table, rcv=rcv, freqs=freqs, eps=np.asarray(e, float)[None, :].copy(),
                 gamma=np.array([complex(gamma_ground)]),
                 meta={"r_ref": r_ref, "s_max": s_max, "policy": policy})


def open_plane_2k(eps="rule", **kw) -> Scene:
    """2,000 rays, rigid ground, source at 10 m, 500 Hz, 64 x 64 receivers at
    1.5 m over 200 x 200 m.  eps="literal" uses epsilon = lambda / 2."""
    kw.setdefault("name", "open_plane_2k_" + str(eps))
    return open_plane(n_rays=kw.pop("n_rays", 2000), grid=kw.pop("grid", 64), half=100.0, freqs=(500.0,),
                      gamma_ground=1.0, eps=eps, **kw)


def open_plane_100k(n_rays=100_000, grid=512, freqs=OCTAVES_8, **kw) -> Scene:
    """100,000 rays, ground coefficient 0.8 exp(i pi/8), eight octave bands
    63 Hz - 8 kHz, 512 x 512 receivers at 1.5 m over 2 x 2 km."""
    kw.setdefault("name", "open_plane_100k_8band")
    return open_plane(n_rays=n_rays, grid=grid, half=1000.0, freqs=freqs,
                      gamma_ground=0.8 * np.exp(1j * np.pi / 8), eps="rule", **kw)


def _city_gamma(city: City, rng, complex_phase: bool) -> np.ndarray:
    nf = city.n_faces
    g = np.empty(nf, np.complex128)
    g[0] = 1.0   # hard ground
    mag = rng.uniform(0.6, 0.95, size=nf - 1)
    if complex_phase:
        g[1:] = mag * np.exp(1j * rng.uniform(-np.pi / 8, np.pi / 8, size=nf - 1))
    else:
        g[1:] = mag
    return g


def city_scene(n_blocks=10, n_rays=1_000_000, grid=1024, freqs=(1000.0,), src=None, max_refl=10,
               city_seed=1, panels=1, complex_gamma=False, name="city", extent=None, z_rcv=1.5) -> Scene:
    """n_blocks x n_blocks buildings of 40 x 40 m footprint, 20 m streets,
    heights U(10, 60) m; walls and roofs with reflection coefficient
    U(0.6, 0.95) (complex phase U(-pi/8, pi/8) when complex_gamma); ground 1.0."""
    city = grid_city(n_blocks, 40.0, 20.0, 10.0, 60.0, seed=city_seed, panels=panels)
    L = extent if extent is not None else 20.0 + 60.0 * n_blocks
    rcv = receiver_grid(grid, grid, 0.0, L, 0.0, L, z_rcv)
    if src is None:
        src = (L / 2.0, L / 2.0, 5.0)
    S = np.asarray(src, dtype=np.float64)
    s_max = 2.0 * float(np.max(np.linalg.norm(rcv - S, axis=1)))
    d, w = fibonacci_fan(n_rays)
    table = trace_city(S, d, w, city, s_max, max_refl)
    freqs = np.asarray(freqs, dtype=np.float64)
    rng = np.random.default_rng(city_seed + 1000)
    gamma = _city_gamma(city, rng, complex_gamma)
    e = eps_rule(freqs, s_max)
    return Scene(name=name, table=table, rcv=rcv, freqs=freqs, eps=e[None, :].copy(), gamma=gamma,
                 meta={"s_max": s_max, "city": city, "inside": inside_buildings(city, rcv)})


def city_10x10(n_rays=1_000_000, grid=1024, **kw) -> Scene:
    """10 x 10 blocks, source at 5 m in the central intersection, up to ten
    specular reflections, 1 kHz, 1024 x 1024 receivers at 1.5 m."""
    kw.setdefault("name", "city_10x10")
    return city_scene(n_blocks=10, n_rays=n_rays, grid=grid, freqs=(1000.0,), max_refl=10, city_seed=1, **kw)


def city_5x5_panels(n_rays=200_000, grid=256, **kw) -> Scene:
    """5 x 5 blocks with every wall and roof split into 2 x 2 panels (500 faces
    plus the ground), each with its own complex coefficient; up to eight
    reflections, 1 kHz, 256 x 256 receivers; source (130, 130, 5)."""
    kw.setdefault("name", "city_5x5_panels")
    return city_scene(n_blocks=5, n_rays=n_rays, grid=grid, freqs=(1000.0,), max_refl=8, city_seed=3,
                      panels=2, complex_gamma=True, src=(130.0, 130.0, 5.0), extent=320.0, **kw)


def perturbed_gamma(gamma: np.ndarray, seed: int = 4, scale: float = 0.1) -> np.ndarray:
    """Target coefficients Gamma* = Gamma (1 + scale xi), xi complex normal,
    clipped to |Gamma*| <= 1; the ground (face 0) is left unchanged."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(gamma.shape) + 1j * rng.standard_normal(gamma.shape)
    g = gamma * (1.0 + scale * xi)
    mag = np.abs(g)
    g = np.where(mag > 1.0, g / mag, g)
    g[0] = gamma[0]
    return g


def city_batched(n_src=16, ray_lo=10_000, ray_hi=500_000, grid=1024, freqs=(125.0, 500.0, 2000.0, 8000.0),
                 seed=2, max_refl=10, name="city_batched_16src") -> Scene:
    """The 10 x 10 city with n_src sources placed uniformly over the streets at
    heights U(2, 30) m, each with U(ray_lo, ray_hi) rays (ragged), four bands."""
    rng = np.random.default_rng(seed)
    city = grid_city(10, 40.0, 20.0, 10.0, 60.0, seed=1)
    L = 620.0
    rcv = receiver_grid(grid, grid, 0.0, L, 0.0, L, 1.5)
    srcs = []
    while len(srcs) < n_src:
        p = np.array([rng.uniform(0, L), rng.uniform(0, L), rng.uniform(2.0, 30.0)])
        if not inside_buildings(city, p[None, :])[0]:
            srcs.append(p)
    n_rays = rng.integers(ray_lo, ray_hi + 1, size=n_src)
    tables = []
    eps = []
    freqs = np.asarray(freqs, dtype=np.float64)
    for S, nr in zip(srcs, n_rays):
        s_max = 2.0 * float(np.max(np.linalg.norm(rcv - S, axis=1)))
        d, w = fibonacci_fan(int(nr))
        tables.append(trace_city(S, d, w, city, s_max, max_refl))
        eps.append(eps_rule(freqs, s_max))
    table = RayTable.concat(tables)
    gamma = _city_gamma(city, np.random.default_rng(1001), False)
    return Scene(name=name, table=table, rcv=rcv, freqs=freqs, eps=np.array(eps), gamma=gamma,
                 meta={"n_rays": n_rays.tolist(), "city": city})


def receiver_subsample(n_total: int, n: int = 4096, seed: int = 5) -> np.ndarray:
    """Seeded sorted subset of receiver indices used where the oracle cannot
    afford every receiver."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=min(n, n_total), replace=False))
