"""Python surface of libgbs: argument marshalling onto the C ABI.

Every step of the computation runs in the HIP library; this module only
moves arrays into torch device memory, passes pointers and the current HIP
stream, and shapes the outputs.  Torch is used for memory and streams only.
"""
from __future__ import annotations

import ctypes
import json
import os
import math

import numpy as np
import torch

from . import _lib

_contexts: dict = {}


def _device_index(device) -> int:
    d = torch.device(device)
    if d.type != "cuda":
        raise ValueError("libgbs runs on a HIP device (torch 'cuda' device)")
    return d.index if d.index is not None else torch.cuda.current_device()


class Context:
    """A libgbs context bound to one device; calls enqueue on torch's current stream."""

    def __init__(self, device="cuda"):
        self.device = torch.device("cuda", _device_index(device))
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(self.lib.gbs_create(ctypes.byref(h), self.device.index, None), None)
        self.handle = h

    def bind_stream(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _lib.check(self.lib.gbs_set_stream(self.handle, ctypes.c_void_p(s.cuda_stream)), self.handle)

    def stats(self) -> dict:
        st = _lib.GbsStats()
        _lib.check(self.lib.gbs_get_stats(self.handle, ctypes.byref(st)), self.handle)
        return st.as_dict()

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.lib.gbs_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def context(device="cuda") -> Context:
    idx = _device_index(device)
    if idx not in _contexts:
        _contexts[idx] = Context(torch.device("cuda", idx))
    return _contexts[idx]


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _as_tensor(x, dtype, device, pin=False):
    if isinstance(x, torch.Tensor):
        t = x.to(dtype=dtype)
        t = t.to(device) if device is not None else t
    else:
        t = torch.as_tensor(np.ascontiguousarray(x), dtype=dtype)
        if device is not None:
            t = t.to(device)
    t = t.contiguous()
    if pin and device is None and not t.is_pinned():
        p = torch.empty(t.shape, dtype=dtype, pin_memory=True)
        p.copy_(t)
        t = p
    return t


class Table:
    """A ray table held as torch tensors, on the device or in pinned host
    memory (host tables are streamed by the library in chunks).

    `src` is any object with the ray-table fields: src_xyz, ray_ptr, ray_w,
    ray_src, seg_a, seg_t, seg_s0, seg_lo, seg_hi, face_ptr, face_ids,
    n_faces (numpy arrays or tensors), and optionally seg_e1 (the ray frame
    of anisotropic beams, [n_segs, 3]; or the `seg_e1` argument)."""

    def __init__(self, src, device="cuda", on_host=False, seg_e1=None):
        dev = None if on_host else torch.device("cuda", _device_index(device))
        self.on_host = on_host
        self.device = torch.device("cuda", _device_index(device))
        self.n_src = int(len(src.src_xyz))
        self.n_faces = int(src.n_faces)
        f64, i64, i32 = torch.float64, torch.int64, torch.int32
        self.ray_ptr = _as_tensor(src.ray_ptr, i64, dev, on_host)
        self.ray_w = _as_tensor(src.ray_w, f64, dev, on_host)
        self.ray_src = _as_tensor(src.ray_src, i32, dev, on_host)
        self.seg_a = _as_tensor(src.seg_a, f64, dev, on_host).reshape(-1, 3)
        self.seg_t = _as_tensor(src.seg_t, f64, dev, on_host).reshape(-1, 3)
        self.seg_s0 = _as_tensor(src.seg_s0, f64, dev, on_host)
        self.seg_lo = _as_tensor(src.seg_lo, f64, dev, on_host)
        self.seg_hi = _as_tensor(src.seg_hi, f64, dev, on_host)
        self.face_ptr = _as_tensor(src.face_ptr, i64, dev, on_host)
        self.face_ids = _as_tensor(src.face_ids, i32, dev, on_host)
        self.n_rays = int(self.ray_w.numel())
        self.n_segs = int(self.seg_s0.numel())
        e1 = seg_e1 if seg_e1 is not None else getattr(src, "seg_e1", None)
        self.seg_e1 = None if e1 is None else _as_tensor(e1, f64, dev, on_host).reshape(-1, 3)
        if self.seg_e1 is not None and self.seg_e1.shape[0] != self.n_segs:
            raise ValueError("seg_e1 needs one frame vector per segment")

    def structs(self):
        rays = _lib.GbsRays(self.n_src, self.n_rays, _ptr(self.ray_ptr), _ptr(self.ray_w), _ptr(self.ray_src))
        segs = _lib.GbsSegs(self.n_segs, _ptr(self.seg_a), _ptr(self.seg_t), _ptr(self.seg_s0), _ptr(self.seg_lo),
                            _ptr(self.seg_hi), _ptr(self.face_ptr), _ptr(self.face_ids),
                            _ptr(self.seg_e1) if self.seg_e1 is not None else None)
        return rays, segs


def _gamma_ri(gamma, device):
    if isinstance(gamma, torch.Tensor) and gamma.is_complex():
        g = torch.view_as_real(gamma.detach().to(device=device, dtype=torch.complex128).contiguous())
    elif isinstance(gamma, torch.Tensor):
        g = gamma.detach().to(device=device, dtype=torch.float64).reshape(-1, 2)
    else:
        a = np.asarray(gamma)
        if np.iscomplexobj(a) or a.ndim == 1:
            a = np.stack([np.real(a), np.imag(a)], axis=-1)
        g = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
    return g.contiguous()


# Shapes chosen by autotune() (or read from its JSON cache), per (device, mode);
# used where a call leaves rcv_per_lane / work_chunk at 0.
_TUNED = {}


def _params(c, gate, mode, flags, chunk_segs, rcv_per_lane, work_chunk, device, alpha=None, eps_e2=None):
    if mode not in _lib.MODES:
        raise ValueError(f"mode must be one of {sorted(_lib.MODES)}")
    tuned = _TUNED.get((_device_index(device), mode), {})
    nr = int(rcv_per_lane) or int(tuned.get("rcv_per_lane", 0))
    wc = int(work_chunk) or int(tuned.get("work_chunk", 0))
    return _lib.GbsParams(float(c), float(gate), _lib.MODES[mode], int(flags), int(chunk_segs), nr, wc,
                          _ptr(alpha) if alpha is not None else None, _ptr(eps_e2) if eps_e2 is not None else None)


class _Call:
    """Marshalled arguments of one forward/backward call."""

    def __init__(self, table, rcv, freqs, eps, gamma, c, gate, mode, chunk_segs, rcv_per_lane, count_active,
                 time_kernels=False, work_chunk=0, alpha=None, eps_e2=None):
        if not isinstance(table, Table):
            raise TypeError("table must be a gbs.Table")
        dev = table.device
        self.table = table
        self.rcv = _as_tensor(rcv, torch.float64, dev).reshape(-1, 3)
        self.freqs = _as_tensor(freqs, torch.float64, dev).reshape(-1)
        self.eps = _as_tensor(eps, torch.float64, dev).reshape(-1)
        if self.eps.numel() != table.n_src * self.freqs.numel():
            raise ValueError("eps must hold one value per (source, band)")
        self.gamma = _gamma_ri(gamma, dev)
        if self.gamma.shape[0] != table.n_faces:
            raise ValueError("gamma must hold one coefficient per face")
        flags = (_lib.FLAG_TABLE_HOST if table.on_host else 0) | \
            (_lib.FLAG_COUNT_ACTIVE if count_active else 0) | (_lib.FLAG_TIME_KERNELS if time_kernels else 0)
        self.alpha = None
        if alpha is not None:
            self.alpha = _as_tensor(alpha, torch.float64, dev).reshape(-1)
            if self.alpha.numel() != self.eps.numel():
                raise ValueError("alpha must hold one value per (source, band)")
        self.eps_e2 = None
        if eps_e2 is not None:
            self.eps_e2 = _as_tensor(eps_e2, torch.float64, dev).reshape(-1)
            if self.eps_e2.numel() != self.eps.numel():
                raise ValueError("eps_e2 must hold one value per (source, band)")
        self.params = _params(c, gate, mode, flags, chunk_segs, rcv_per_lane, work_chunk, dev, self.alpha,
                              self.eps_e2)
        self.rays, self.segs = table.structs()
        self.faces = _lib.GbsFaces(table.n_faces, _ptr(self.gamma))
        self.n_rcv = int(self.rcv.shape[0])
        self.n_freq = int(self.freqs.numel())
        self.shape = (table.n_src, self.n_freq, self.n_rcv)

    def common(self, ctx):
        return (ctx.handle, ctypes.byref(self.rays), ctypes.byref(self.segs), ctypes.byref(self.faces),
                _ptr(self.rcv), self.n_rcv, _ptr(self.freqs), self.n_freq, _ptr(self.eps), ctypes.byref(self.params))


def forward(table: Table, rcv, freqs, eps, gamma, *, c=343.0, gate=9.21, mode="mix", chunk_segs=0,
            rcv_per_lane=0, work_chunk=0, count_active=False, time_kernels=False, want_tl=True,
            alpha=None, eps_e2=None):
    """Beam summation.  Returns (P complex128 [n_src, n_freq, n_rcv],
    TL float64 of the same shape or None).  count_active / time_kernels fill
    the statistics returned by stats().  alpha: atmospheric absorption per
    (source, band) in Np/m (see air_absorption), or None.  eps_e2: beam
    parameter along e2 per (source, band) for anisotropic beams (eps is then
    the one along the horizontal frame vector e1), or None."""
    return _forward("gbs_forward", table, rcv, freqs, eps, gamma, c, gate, mode, chunk_segs, rcv_per_lane,
                    work_chunk, count_active, time_kernels, want_tl, alpha, eps_e2)


def forward_noalloc(table: Table, rcv, freqs, eps, gamma, *, c=343.0, gate=9.21, mode="mix", rcv_per_lane=0,
                    work_chunk=0, count_active=False, time_kernels=False, want_tl=True, alpha=None, eps_e2=None,
                    out=None):
    """forward() through gbs_forward_noalloc: the library allocates no device
    memory (its scratch is a static 128 MiB array per GPU, shared by every
    call on that GPU; stats()["scratch_bytes"] is what the call used).
    Device tables only.  `out` = (P float64 [n_src, n_freq, n_rcv, 2],
    TL float64 [n_src, n_freq, n_rcv] or None) reuses caller-owned outputs."""
    return _forward("gbs_forward_noalloc", table, rcv, freqs, eps, gamma, c, gate, mode, 0, rcv_per_lane,
                    work_chunk, count_active, time_kernels, want_tl, alpha, eps_e2, out)


def _forward(entry, table, rcv, freqs, eps, gamma, c, gate, mode, chunk_segs, rcv_per_lane, work_chunk,
             count_active, time_kernels, want_tl, alpha, eps_e2, out=None):
    ctx = context(table.device)
    ctx.bind_stream()
    call = _Call(table, rcv, freqs, eps, gamma, c, gate, mode, chunk_segs, rcv_per_lane, count_active,
                 time_kernels, work_chunk, alpha, eps_e2)
    if out is not None:
        P, TL = out
        if P.dtype != torch.float64 or tuple(P.shape) != call.shape + (2,) or not P.is_contiguous():
            raise ValueError("out P must be contiguous float64 of shape (n_src, n_freq, n_rcv, 2)")
        if TL is not None and (TL.dtype != torch.float64 or tuple(TL.shape) != call.shape or
                               not TL.is_contiguous()):
            raise ValueError("out TL must be contiguous float64 of shape (n_src, n_freq, n_rcv)")
    else:
        P = torch.empty(call.shape + (2,), dtype=torch.float64, device=table.device)
        TL = torch.empty(call.shape, dtype=torch.float64, device=table.device) if want_tl else None
    rc = getattr(ctx.lib, entry)(*call.common(ctx), _ptr(P), _ptr(TL))
    _lib.check(rc, ctx.handle)
    return torch.view_as_complex(P), TL


def backward(table: Table, rcv, freqs, eps, gamma, lam, *, c=343.0, gate=9.21, mode="mix", chunk_segs=0,
             alpha=None, time_kernels=False, eps_e2=None):
    """Adjoint for dL = Re sum lam * dP.  Returns (d_gamma [n_faces, 2] as
    (dL/dRe, dL/dIm), d_rcv [n_rcv, 3], d_eps [n_src, n_freq]); with
    anisotropic beams (eps_e2) also d_eps_e2 [n_src, n_freq]."""
    ctx = context(table.device)
    ctx.bind_stream()
    call = _Call(table, rcv, freqs, eps, gamma, c, gate, mode, chunk_segs, 0, False, time_kernels,
                 alpha=alpha, eps_e2=eps_e2)
    lam_t = lam if isinstance(lam, torch.Tensor) else torch.as_tensor(np.asarray(lam))
    lam_t = lam_t.to(device=table.device, dtype=torch.complex128).reshape(call.shape).contiguous()
    lam_ri = torch.view_as_real(lam_t).contiguous()
    d_gamma = torch.empty((table.n_faces, 2), dtype=torch.float64, device=table.device)
    d_rcv = torch.empty((call.n_rcv, 3), dtype=torch.float64, device=table.device)
    d_eps = torch.empty((table.n_src, call.n_freq), dtype=torch.float64, device=table.device)
    d_eps2 = torch.empty_like(d_eps) if eps_e2 is not None else None
    rc = ctx.lib.gbs_backward(*call.common(ctx), _ptr(lam_ri), _ptr(d_gamma), _ptr(d_rcv), _ptr(d_eps),
                              _ptr(d_eps2) if d_eps2 is not None else None)
    _lib.check(rc, ctx.handle)
    if eps_e2 is not None:
        return d_gamma, d_rcv, d_eps, d_eps2
    return d_gamma, d_rcv, d_eps


class _Traced:
    """Fields of a traced table (device tensors) in the layout Table reads."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def trace(src_xyz, dirs, weights, *, ray_src=None, boxes=None, panels=1, s_max, max_refl=10,
          image_complete=False, e1=None, device="cuda") -> Table:
    """Ray tracing on the device (gbs_trace): the fan `dirs` [n, 3] (unit) from
    the sources `src_xyz` [n_src, 3] (ray i from source ray_src[i], default 0)
    through the ground plane and `boxes` [n_boxes, 5] (x0, x1, y0, y1, h),
    each ray until its arc length reaches s_max (a number, or one per source);
    returns the ray table as a device Table with the given ray weights.
    e1: launch frame per ray ([n, 3], unit, normal to the direction) for
    anisotropic beams; the table then carries the frame of every segment
    (mirrored at each reflection) as seg_e1."""
    ctx = context(device)
    ctx.bind_stream()
    dev = ctx.device
    f64 = torch.float64
    src = _as_tensor(src_xyz, f64, dev).reshape(-1, 3)
    d = _as_tensor(dirs, f64, dev).reshape(-1, 3)
    w = _as_tensor(weights, f64, dev).reshape(-1)
    n = int(d.shape[0])
    if w.numel() != n:
        raise ValueError("one weight per ray")
    rs = _as_tensor(ray_src, torch.int32, dev).reshape(-1) if ray_src is not None else \
        torch.zeros(n, dtype=torch.int32, device=dev)
    if rs.numel() != n:
        raise ValueError("one source index per ray")
    bx = _as_tensor(np.zeros((0, 5)) if boxes is None else boxes, f64, dev).reshape(-1, 5)
    sm = np.asarray(s_max, np.float64)
    sm_src = None
    if sm.ndim > 0:
        sm_src = _as_tensor(sm, f64, dev).reshape(-1)
        if sm_src.numel() != src.shape[0]:
            raise ValueError("s_max: one value, or one per source")
    scene = _lib.GbsScene(int(bx.shape[0]), int(panels), _ptr(bx), float(sm.max()) if sm.size else 0.0,
                          int(max_refl), 1 if image_complete else 0)
    e1t = None if e1 is None else _as_tensor(e1, f64, dev).reshape(-1, 3)
    if e1t is not None and e1t.shape[0] != n:
        raise ValueError("e1: one launch frame per ray")
    fan = _lib.GbsFan(int(src.shape[0]), _ptr(src), n, _ptr(d), _ptr(rs), _ptr(sm_src) if sm_src is not None else None,
                      _ptr(e1t) if e1t is not None else None)
    ns, nf, token = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _lib.check(ctx.lib.gbs_trace_count(ctx.handle, ctypes.byref(scene), ctypes.byref(fan), ctypes.byref(ns),
                                       ctypes.byref(nf), ctypes.byref(token)), ctx.handle)
    S, F = int(ns.value), int(nf.value)
    out = _Traced(src_xyz=src, ray_w=w, ray_src=rs, n_faces=1 + int(bx.shape[0]) * 5 * int(panels) ** 2,
                  ray_ptr=torch.empty(n + 1, dtype=torch.int64, device=dev),
                  seg_a=torch.empty((S, 3), dtype=f64, device=dev), seg_t=torch.empty((S, 3), dtype=f64, device=dev),
                  seg_s0=torch.empty(S, dtype=f64, device=dev), seg_lo=torch.empty(S, dtype=f64, device=dev),
                  seg_hi=torch.empty(S, dtype=f64, device=dev),
                  face_ptr=torch.empty(S + 1, dtype=torch.int64, device=dev),
                  face_ids=torch.empty(F, dtype=torch.int32, device=dev),
                  seg_e1=torch.empty((S, 3), dtype=f64, device=dev) if e1t is not None else None)
    # the count just taken is reused (same arguments, inputs untouched in between)
    rc = ctx.lib.gbs_trace(ctx.handle, ctypes.byref(scene), ctypes.byref(fan), token.value, S, F,
                           _ptr(out.ray_ptr), _ptr(out.seg_a), _ptr(out.seg_t), _ptr(out.seg_s0), _ptr(out.seg_lo),
                           _ptr(out.seg_hi), _ptr(out.face_ptr), _ptr(out.face_ids),
                           _ptr(out.seg_e1) if out.seg_e1 is not None else None, ctypes.byref(ns), ctypes.byref(nf))
    _lib.check(rc, ctx.handle)
    return Table(out, device=dev)


def _tune_key(table: Table, call, mode: str) -> str:
    """Cache key: GPU architecture, mode and a size bucket of the problem
    (log2 of the dense pair count, bands, sources)."""
    arch = torch.cuda.get_device_properties(table.device).gcnArchName.split(":")[0]
    dense = max(1, table.n_segs * call.n_rcv * call.n_freq)
    return f"{arch}|{mode}|2^{int(math.log2(dense))}|bands{call.n_freq}|src{table.n_src}"


def autotune(table: Table, rcv, freqs, eps, gamma, *, c=343.0, gate=9.21, mode="mix", cache=None, alpha=None,
             eps_e2=None):
    """Times the pair-kernel shapes (receivers per lane x work-unit size) on
    this problem; later calls in `mode` that leave rcv_per_lane / work_chunk
    at 0 use the fastest.  With `cache` (a JSON file path) a stored choice for
    the same architecture, mode and size bucket is reused without timing, and
    a new one is stored.  Returns {"rcv_per_lane": .., "work_chunk": ..}."""
    ctx = context(table.device)
    ctx.bind_stream()
    call = _Call(table, rcv, freqs, eps, gamma, c, gate, mode, 0, 0, False, alpha=alpha, eps_e2=eps_e2)
    key = _tune_key(table, call, mode)
    store = {}
    if cache is not None and os.path.exists(cache):
        with open(cache) as f:
            store = json.load(f)
        if key in store:
            _TUNED[(_device_index(table.device), mode)] = dict(store[key])
            return dict(store[key])
    P = torch.empty(call.shape + (2,), dtype=torch.float64, device=table.device)
    nr, wc = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = ctx.lib.gbs_autotune(*call.common(ctx), _ptr(P), ctypes.byref(nr), ctypes.byref(wc))
    _lib.check(rc, ctx.handle)
    choice = {"rcv_per_lane": int(nr.value), "work_chunk": int(wc.value)}
    _TUNED[(_device_index(table.device), mode)] = choice
    if cache is not None:
        store[key] = choice
        tmp = f"{cache}.tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(store, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(choice)


def impulse_response(table: Table, rcv, df, bin0, n_bins, eps, gamma, *, n_fft, n_t=None, window=None, c=343.0,
                     gate=9.21, mode="mix", alpha=None, chunk_segs=0):
    """Broadband synthesis (gbs_impulse_response): the time signal
    h [n_src, n_rcv, n_t] at dt = 1 / (n_fft df) from the forward sum at
    f_n = (bin0 + n) df, n < n_bins, with the real taper `window` [n_bins].
    eps (and alpha) per (source, bin)."""
    ctx = context(table.device)
    ctx.bind_stream()
    n_t = n_fft if n_t is None else int(n_t)
    freqs = (int(bin0) + np.arange(int(n_bins))) * float(df)
    call = _Call(table, rcv, freqs, eps, gamma, c, gate, mode, chunk_segs, 0, False, alpha=alpha)
    win = None if window is None else _as_tensor(window, torch.float64, table.device).reshape(-1)
    if win is not None and win.numel() != int(n_bins):
        raise ValueError("one window value per bin")
    h = torch.empty((table.n_src, call.n_rcv, n_t), dtype=torch.float64, device=table.device)
    rays, segs = call.rays, call.segs
    rc = ctx.lib.gbs_impulse_response(ctx.handle, ctypes.byref(rays), ctypes.byref(segs), ctypes.byref(call.faces),
                                      _ptr(call.rcv), call.n_rcv, float(df), int(bin0), int(n_bins), _ptr(call.eps),
                                      _ptr(win), ctypes.byref(call.params), int(n_fft), n_t, _ptr(h))
    _lib.check(rc, ctx.handle)
    return h


def air_absorption(freqs, temp_c=20.0, rh_pct=70.0, pressure_atm=1.0) -> np.ndarray:
    """Atmospheric absorption (ISO 9613-1, gbs_air_absorption_db) as the
    amplitude decay rate alpha in Np/m for each frequency; the defaults are
    the paper's atmosphere (Tables 2 and 3)."""
    lib = _lib.load()
    f = np.atleast_1d(np.asarray(freqs, np.float64))
    db = np.array([lib.gbs_air_absorption_db(float(x), float(temp_c), float(rh_pct), float(pressure_atm))
                   for x in f])
    if not np.all(np.isfinite(db)):
        raise ValueError("atmosphere or frequency out of range")
    return db * (math.log(10.0) / 20.0)


def stats(device="cuda") -> dict:
    return context(device).stats()


class Graph:
    """One captured forward (all jobs, one persistent launch per pass over the
    table; a host table is streamed by the replay) that can be replayed; the
    coefficient tensor may be updated in place between replays."""

    def __init__(self, table: Table, rcv, freqs, eps, gamma, *, c=343.0, gate=9.21, mode="mix", rcv_per_lane=0,
                 chunk_segs=0, alpha=None, eps_e2=None):
        self.ctx = context(table.device)
        self.stream = torch.cuda.Stream(device=table.device)
        self.call = _Call(table, rcv, freqs, eps, gamma, c, gate, mode, chunk_segs, rcv_per_lane, False,
                          alpha=alpha, eps_e2=eps_e2)
        self.gamma = self.call.gamma          # [n_faces, 2] device buffer read at every replay
        self.P = torch.empty(self.call.shape + (2,), dtype=torch.float64, device=table.device)
        self.TL = torch.empty(self.call.shape, dtype=torch.float64, device=table.device)
        torch.cuda.current_stream(table.device).synchronize()
        self.ctx.bind_stream(self.stream)
        h = ctypes.c_void_p()
        try:
            rc = self.ctx.lib.gbs_graph_create(*self.call.common(self.ctx), _ptr(self.P), _ptr(self.TL),
                                               ctypes.byref(h))
            _lib.check(rc, self.ctx.handle)
        finally:
            self.ctx.bind_stream()
        self.handle = h

    def set_gamma(self, gamma):
        g = _gamma_ri(gamma, self.P.device)
        with torch.cuda.stream(self.stream):
            self.gamma.copy_(g)

    def launch(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.P.device))
        self.ctx.bind_stream(self.stream)
        try:
            _lib.check(self.ctx.lib.gbs_graph_launch(self.handle), self.ctx.handle)
        finally:
            self.ctx.bind_stream()
        torch.cuda.current_stream(self.P.device).wait_stream(self.stream)
        return torch.view_as_complex(self.P), self.TL

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.ctx.lib.gbs_graph_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


LN10 = math.log(10.0)


class GBSFunction(torch.autograd.Function):
    """Differentiable beam summation with the ray geometry held fixed.

    apply(gamma [n_faces] complex128, rcv [n_rcv, 3] float64,
          eps [n_src, n_freq] float64, table, freqs, opts dict,
          eps_e2 [n_src, n_freq] float64 or None) -> (P, TL)

    Gradients flow to the reflection coefficients (torch's complex
    convention: dL/dRe + i dL/dIm), the receiver positions, eps and, with
    anisotropic beams, eps_e2 (the table's frame held fixed).
    """

    @staticmethod
    def forward(ctx, gamma, rcv, eps, table, freqs, opts, eps_e2=None):
        opts = dict(opts or {})
        if "eps_e2" in opts:
            raise ValueError("pass eps_e2 as GBSFunction's last input, not in opts")
        e2 = eps_e2.detach() if eps_e2 is not None else None
        P, TL = forward(table, rcv.detach(), freqs, eps.detach(), gamma.detach(), eps_e2=e2, **opts)
        ctx.save_for_backward(gamma, rcv, eps, P, e2 if e2 is not None else torch.empty(0))
        ctx.table, ctx.freqs, ctx.opts, ctx.aniso = table, freqs, opts, eps_e2 is not None
        ctx.mark_non_differentiable()
        return P, TL

    @staticmethod
    def backward(ctx, gP, gTL):
        gamma, rcv, eps, P, e2 = ctx.saved_tensors
        lam = torch.zeros_like(P)
        if gP is not None:
            lam = lam + torch.conj(gP)
        if gTL is not None:
            # TL = -20 log10|P|: dTL = -(20/ln10) Re(dP/P); receivers with P = 0
            # (TL = inf) take no gradient
            g = gTL.to(P.dtype)
            live = (g != 0) & (P != 0)
            lam = lam - (20.0 / LN10) * torch.where(live, g / torch.where(live, P, torch.ones_like(P)),
                                                     torch.zeros_like(P))
        opts = {k: v for k, v in ctx.opts.items() if k in ("c", "gate", "mode", "chunk_segs", "alpha")}
        out = backward(ctx.table, rcv.detach(), ctx.freqs, eps.detach(), gamma.detach(), lam,
                       eps_e2=e2 if ctx.aniso else None, **opts)
        dG, dR, dE = out[:3]
        g_gamma = torch.complex(dG[:, 0], dG[:, 1]).to(gamma.dtype) if ctx.needs_input_grad[0] else None
        g_rcv = dR.to(rcv.dtype).reshape(rcv.shape) if ctx.needs_input_grad[1] else None
        g_eps = dE.to(eps.dtype).reshape(eps.shape) if ctx.needs_input_grad[2] else None
        g_e2 = None
        if ctx.aniso and len(ctx.needs_input_grad) > 6 and ctx.needs_input_grad[6]:
            g_e2 = out[3].to(e2.dtype).reshape(e2.shape)
        return g_gamma, g_rcv, g_eps, None, None, None, g_e2
