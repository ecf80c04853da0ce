"""Benchmark: Gaussian beam summation throughput on one MI355X.

Workload: the 100,000-ray open plane (Fibonacci fan from 10 m over a ground
with coefficient 0.8 exp(i pi/8), eight octave bands 63 Hz - 8 kHz, 512 x 512
receivers at 1.5 m over 2 x 2 km), seeded and synthetic.  One step is one
full forward call of the library (receiver ordering, segment records, culled
work lists, persistent pair kernel, TL) in the FP32 + FP64-phase mode with
the table resident in HBM.  `value` = dense segment x receiver x band
evaluations per second (the dense sum the culled kernel reproduces).

Also reported: the pair kernel's roofline (the survey's algorithmic FLOPs
per pair times the listed and kept pairs of one launch, over its
HIP-event-timed duration, against the FP32 VALU peak; the kernel's own count
against its FP64/FP32 mixed peak beside it; the launch's HBM traffic from
rocprofv3 counters while the pair kernel's source is the one they were
measured on), the all-FP64 mode on the same GPU, the forward
captured as a hipGraph and replayed, the table
streamed from pinned host memory in four overlapped passes (PCIe-inclusive,
never `value`), the adjoint call on the same workload, the error against the
FP64 oracle on 16,384 seeded receivers, the oracle timed on this host's
cores on that sample (and single-threaded on a smaller one), and the device
ray tracer re-tracing the workload's fan (with the per-ray oracle tracer
timed on a sample of rays), the forward with atmospheric absorption in
the paper's atmosphere, the forward with anisotropic beams (beam parameter
along e2 twice the one along e1), and broadband synthesis (an impulse
response per receiver from 1,751 frequency bins) on a receiver subsample.
Two more workloads run on the same clock (`workloads`): the 10 x 10 city
with 1,000,000 rays over 1024 x 1024 receivers at 1 kHz, and the batched
city (16 sources with U(10k, 500k) rays, four bands, 1024 x 1024 receivers),
each with its forward, pair-kernel roofline, graph replay and a sampled
oracle check.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per pair of the pair kernel, counted from the evaluated
# formulas (an FMA counts 2; a transcendental, a reciprocal or a fract 1;
# compares count 0):
#   every listed pair: arc length s (3 FMA), |R-o|^2 - |o|^2 (3 FMA) and the
#     gate's right-hand side c1 s^2 + c2 - |o|^2 (mul, FMA)                 -> 15 FP64
#   every kept pair: n^2 (add, FMA), the leading phase (f/c) s + arg(w Gamma)/2pi
#     (FMA) and its fract, accumulation (2 adds)                           -> 8 FP64
#     den (FMA), rcp, a = n^2/den, the phase correction (mul, FMA), fract,
#     sin, cos, Gaussian exponent with log2|w Gamma| (FMA), exp2, weight,
#     (s + i eps) w (2 mul), rotation (2 x (mul, FMA)), pair sum            -> 23 FP32
FLOP_LISTED_F64 = 15
FLOP_KEPT_F64 = 8
FLOP_KEPT_F32 = 23
# The survey's algorithmic count per pair (what the method must do, FMA = 2):
# a pre-gate of ~20 flops on every listed (not culled) pair; per kept pair ~30
# FP64 flops (arc length, normal distance, denominator, reciprocal, phase and
# its reduction), ~40 FP32 flops (Gaussian, amplitude, complex rotation,
# compensated accumulation) and 3 transcendentals (counted 1 each, as FP32).
# The adjoint kernel per kept pair (the forward gate per listed pair as above):
# 29 FP64 flops (n^2, den, Newton reciprocal, a, phase, fract, Gaussian
# exponent: 15; the receiver-gradient sums V, W, G and the eps sum: 14) and
# 69 FP32 (rcp, sin, cos, exp2 and the weight; d ln u/dR and d ln u/deps: 25;
# the beam term, lambda u, the gradient coefficients and the segment and eps
# sums).
ADJ_FLOP_KEPT_F64 = 29
ADJ_FLOP_KEPT_F32 = 69
SURVEY_FLOP_LISTED = 20
SURVEY_FLOP_KEPT_F64 = 30
SURVEY_FLOP_KEPT_F32 = 43
# The anisotropic variant (same 15 FP64 per listed pair):
#   every kept pair: n1^2 + n2^2 (add, FMA), n1 (2 FMA), n1^2, n2^2, two
#     denominators (2 FMA), two Newton reciprocals (4 FMA), a1, a2, the gate
#     sum (mul, FMA), cycles (add, FMA, mul), fract, Gaussian exponent,
#     accumulation (2 adds)                                                -> 34 FP64
#     2 rcp, sin, cos, exp2, 2 sqrt, b1, b2, s^2, b1 b2 - s^2 (2 FMA, rcp,
#     mul; eps1 eps2, 2 FMA, add), s (b1 + b2) (add, mul), prefactor (5 mul,
#     rsq), weights (2 x (mul, FMA, mul)), rotation (2 x (mul, FMA)), pair sum -> 45 FP32
ANI_FLOP_KEPT_F64 = 34
ANI_FLOP_KEPT_F32 = 45
# Vector peaks from unit counts and clock: 256 CUs x 2.4 GHz x 64 FMA lanes x 2
# = 78.6 TFLOP/s FP64; FP32 157.3 TFLOP/s (vendor figure).
PEAK_F64 = 256 * 2.4e9 * 64 * 2
PEAK_F32 = 157.3e12

# HBM bytes per launch of the pair kernel on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy and fill (the summary in
# profiles/k_pairs_mix_open_plane_100k.md).  Valid only for the pair-kernel
# source it was measured on: the MD5 of the "pair kernels" section of
# gbs_kernels.hip (from its section rule up to the adjoint's) and of
# gbs_internal.h; reported as null once either changes.
PAIR_TRAFFIC_BYTES = 4.303e9
PAIR_TRAFFIC_SOURCE_MD5 = {"pair_section": "2ed9bfcb852261f25f3264a7d5b1ff82", "gbs_internal.h": "69bc0b9e3ee1e33c6f3bc1b81db3b8c2"}


def pair_source_md5():
    """MD5s of the pair kernel's source: its section of gbs_kernels.hip and gbs_internal.h."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2501_13382_amd", "csrc")
    text = open(os.path.join(csrc, "gbs_kernels.hip")).read()
    i = text.find("// " + "-" * 61 + " pair kernels")
    j = text.find("// " + "-" * 65 + " adjoint")
    section = text[i:j] if 0 <= i < j else text
    with open(os.path.join(csrc, "gbs_internal.h"), "rb") as f:
        internal = f.read()
    return {"pair_section": hashlib.md5(section.encode()).hexdigest(),
            "gbs_internal.h": hashlib.md5(internal).hexdigest()}


def pair_traffic():
    if PAIR_TRAFFIC_BYTES is None or pair_source_md5() != PAIR_TRAFFIC_SOURCE_MD5:
        return None
    return PAIR_TRAFFIC_BYTES


def _open_plane_100k():
    from scenes import open_plane_100k
    return open_plane_100k()


def _city_1m():
    from scenes import city_10x10
    return city_10x10(n_rays=1_000_000, grid=1024)


def _city_batched():
    from scenes import city_batched
    return city_batched(grid=1024)


WORKLOADS = {"open_plane_100k": ("open_plane_100k_8band", _open_plane_100k),
             "city_1m": ("city_10x10_1m_rays_1024sq", _city_1m),
             "city_batched": ("city_batched_16src_4band_1024sq", _city_batched)}


def oracle_threads() -> int:
    """Threads for the oracle: every CPU this process may run on
    (sched_getaffinity), capped by OMP_NUM_THREADS where the host sets it
    to its CPU share."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    return max(1, min(n, int(env))) if env else n


def host_cpus() -> dict:
    return {"nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def roofline(listed, kept, ms, kernel, f64_listed=FLOP_LISTED_F64, f64_kept=FLOP_KEPT_F64, f32_kept=FLOP_KEPT_F32,
             survey=True):
    """The pair kernel's roofline from its listed and kept pair counts and its
    HIP-event time.  `achieved` counts the survey's algorithmic work per pair
    of the forward sum (20 flops per listed pair, 30 FP64 + 43 FP32 per kept
    pair) and `frac` sets it against the FP32 VALU peak, the metric's
    denominator; beside it, the same time with the kernel's own per-pair
    count (the formulas it evaluates) against the peak for its FP64/FP32 mix
    (time at peak = f64/PEAK_F64 + f32/PEAK_F32).  For kernels the survey
    gives no count for (survey=False: the adjoint, anisotropic beams) the
    kernel's own count is the algorithmic one."""
    if survey:
        s64 = SURVEY_FLOP_LISTED * listed + SURVEY_FLOP_KEPT_F64 * kept
        s32 = SURVEY_FLOP_KEPT_F32 * kept
    else:
        s64 = f64_listed * listed + f64_kept * kept
        s32 = f32_kept * kept
    s_ach = (s64 + s32) / (ms * 1e-3)
    s_mixed = (s64 + s32) / (s64 / PEAK_F64 + s32 / PEAK_F32)
    f64 = f64_listed * listed + f64_kept * kept
    f32 = f32_kept * kept
    k_ach = (f64 + f32) / (ms * 1e-3)
    k_mixed = (f64 + f32) / (f64 / PEAK_F64 + f32 / PEAK_F32)
    return {"bound": "alu", "kernel": kernel, "achieved": s_ach / 1e12, "peak": PEAK_F32 / 1e12, "unit": "TFLOP/s",
            "frac": s_ach / PEAK_F32, "frac_of_mixed_peak": s_ach / s_mixed, "mixed_peak": s_mixed / 1e12,
            "flop_per_listed_pair": SURVEY_FLOP_LISTED if survey else {"f64": f64_listed},
            "flop_per_kept_pair": ({"f64": SURVEY_FLOP_KEPT_F64, "f32": SURVEY_FLOP_KEPT_F32} if survey else
                                   {"f64": f64_kept, "f32": f32_kept}),
            "count": "survey" if survey else "kernel",
            "ms_per_launch": ms, "listed_pairs": int(listed), "kept_pairs": int(kept),
            "kernel_count": {"achieved": k_ach / 1e12, "mixed_peak": k_mixed / 1e12, "frac_of_mixed_peak": k_ach / k_mixed,
                             "frac_of_fp32_peak": k_ach / PEAK_F32,
                             "flop_per_listed_pair": {"f64": f64_listed},
                             "flop_per_kept_pair": {"f64": f64_kept, "f32": f32_kept}}}


def cpu_model() -> str:
    """The host CPU's model name (first entry of /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def absorption_bench(sc, dev, table, rcv, freqs, eps, gamma, args, sec_step):
    """The same forward with atmospheric absorption in the paper's atmosphere
    (Tables 2 and 3: 20 deg C, 70 % relative humidity, 1 atm; ISO 9613-1 per
    band): time per step, and the error against the oracle with the same
    absorption on a small seeded receiver sample."""
    import torch

    import paper_2501_13382_amd as gbs
    from scenes import receiver_subsample
    alpha_band = gbs.air_absorption(sc.freqs, 20.0, 70.0, 1.0)
    alpha = np.tile(alpha_band, (sc.table.n_src, 1))
    a_dev = torch.as_tensor(alpha, device=dev)
    call = lambda: gbs.forward(table, rcv, freqs, eps, gamma, c=sc.c, gate=sc.gate, mode="mix", alpha=a_dev)
    call()
    torch.cuda.synchronize()
    n = max(2, args.steps // 2)
    t = time.perf_counter()
    for _ in range(n):
        P, TL = call()
    torch.cuda.synchronize()
    s_ab = (time.perf_counter() - t) / n
    leg = {"value": sc.dense_pairs / s_ab, "ms_per_step": s_ab * 1e3, "overhead_vs_value": s_ab / sec_step - 1.0,
           "atmosphere": {"temperature_c": 20.0, "humidity_pct": 70.0, "pressure_atm": 1.0},
           "alpha_db_per_km": [float(a) * 20.0 / np.log(10.0) * 1e3 for a in alpha_band]}
    print(f"# absorption: {s_ab * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    if not args.no_cpu:
        import oracle
        n_cpu = int(min(1024, max(16, 4e9 / (sc.table.n_segs * len(sc.freqs)))))
        idx = receiver_subsample(len(sc.rcv), n=n_cpu, seed=8)
        threads = oracle_threads()
        P_ref, TL_ref, ab = oracle.scene_forward(sc, rcv=sc.rcv[idx], n_threads=threads, return_absum=True,
                                                 alpha=alpha)
        Pg = P.cpu().numpy().reshape(-1, len(sc.rcv))[:, idx]
        TLg = TL.cpu().numpy().reshape(-1, len(sc.rcv))[:, idx]
        ok = ab / np.maximum(np.abs(P_ref), 1e-300) <= 1e4
        leg["accuracy_vs_oracle"] = {
            "tl_err_db_max": float(np.abs(TLg - TL_ref)[ok].max()),
            "rel_err_max": float((np.abs(Pg - P_ref) / np.maximum(np.abs(P_ref), 1e-300))[ok].max()),
            "receivers": int(len(idx))}
    return leg


def aniso_bench(sc, dev, table, rcv, freqs, eps, gamma, args, sec_step):
    """The same forward with anisotropic beams (Q = diag(q1, q2); the beam
    parameter along e2 twice the one along the horizontal e1): time per
    step, the pair kernel's time, and the error against the oracle's
    anisotropic sum on a small seeded receiver sample."""
    import torch

    import paper_2501_13382_amd as gbs
    from scenes import normal_frame, receiver_subsample
    e2 = 2.0 * np.asarray(sc.eps, np.float64).reshape(-1)
    e2_dev = torch.as_tensor(e2, device=dev)
    call = lambda tk=False: gbs.forward(table, rcv, freqs, eps, gamma, c=sc.c, gate=sc.gate, mode="mix",
                                        eps_e2=e2_dev, time_kernels=tk)
    call()
    torch.cuda.synchronize()
    n = max(2, args.steps // 2)
    t = time.perf_counter()
    for _ in range(n):
        P, TL = call()
    torch.cuda.synchronize()
    s_an = (time.perf_counter() - t) / n
    ms_pairs = []
    for _ in range(3):
        call(True)
        torch.cuda.synchronize()
        ms_pairs.append(gbs.stats()["ms_pairs"])
    ms_pairs = float(np.mean(ms_pairs))
    gbs.forward(table, rcv, freqs, eps, gamma, c=sc.c, gate=sc.gate, mode="mix", eps_e2=e2_dev, count_active=True)
    torch.cuda.synchronize()
    st = gbs.stats()
    listed, active = st["listed_pairs"], st["active_pairs"]
    leg = {"value": sc.dense_pairs / s_an, "ms_per_step": s_an * 1e3, "overhead_vs_value": s_an / sec_step - 1.0,
           "eps_e2_over_eps": 2.0,
           "roofline": roofline(listed, active, ms_pairs, "k_pairs<MIX|aniso>", f64_kept=ANI_FLOP_KEPT_F64,
                                f32_kept=ANI_FLOP_KEPT_F32, survey=False)}
    print(f"# anisotropic: {s_an * 1e3:.2f} ms/step, pair kernel {ms_pairs:.2f} ms", file=sys.stderr,
          flush=True)
    if not args.no_cpu:
        import oracle
        n_cpu = int(min(1024, max(16, 4e9 / (sc.table.n_segs * len(sc.freqs)))))
        idx = receiver_subsample(len(sc.rcv), n=n_cpu, seed=9)
        threads = oracle_threads()
        P_ref, TL_ref, ab = oracle.forward(sc.table, sc.gamma, sc.rcv[idx], sc.freqs, sc.eps, c=sc.c, gate=sc.gate,
                                           n_threads=threads, return_absum=True, eps_e2=e2,
                                           seg_e1=normal_frame(sc.table.seg_t))
        Pg = P.cpu().numpy().reshape(-1, len(sc.rcv))[:, idx]
        TLg = TL.cpu().numpy().reshape(-1, len(sc.rcv))[:, idx]
        ok = ab / np.maximum(np.abs(P_ref), 1e-300) <= 1e4
        leg["accuracy_vs_oracle"] = {
            "tl_err_db_max": float(np.abs(TLg - TL_ref)[ok].max()),
            "rel_err_max": float((np.abs(Pg - P_ref) / np.maximum(np.abs(P_ref), 1e-300))[ok].max()),
            "receivers": int(len(idx))}
    return leg


def impulse_bench(sc, dev, table, gamma, args):
    """Broadband synthesis on the open plane: the time signal at 4,096 seeded
    receivers from 1,751 frequency bins (50-400 Hz every 0.2 Hz: a 5 s period
    that holds the longest path), Hann taper, 4,096-point transforms (1.22 ms
    samples); eps by the workload's rule per bin.  Timed once after a warm-up
    call; a few receivers against the oracle's impulse response."""
    import torch

    import paper_2501_13382_amd as gbs
    from scenes import receiver_subsample
    df, bin0, n_bins, n_fft = 0.2, 250, 1751, 4096
    freqs = (bin0 + np.arange(n_bins)) * df
    eps = (6.0 * np.sqrt(sc.meta["r_ref"] / (2 * np.pi * freqs / sc.c)))[None, :]
    win = np.hanning(n_bins + 2)[1:-1]
    idx = receiver_subsample(len(sc.rcv), n=4096, seed=9)
    rcv = torch.as_tensor(sc.rcv[idx], device=dev)
    call = lambda: gbs.impulse_response(table, rcv, df, bin0, n_bins, eps, gamma, n_fft=n_fft, window=win,
                                        c=sc.c, gate=sc.gate, mode="mix")
    call()
    torch.cuda.synchronize()
    t = time.perf_counter()
    h = call()
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    dense = table.n_segs * len(idx) * n_bins
    leg = {"ms": el * 1e3, "receivers": int(len(idx)), "bins": n_bins, "df_hz": df, "band_hz": [freqs[0], freqs[-1]],
           "n_fft": n_fft, "dt_ms": 1e3 / (n_fft * df), "dense_evals_per_s": dense / el}
    print(f"# impulse response: {el * 1e3:.1f} ms for {len(idx)} receivers x {n_bins} bins", file=sys.stderr,
          flush=True)
    if not args.no_cpu:
        import oracle
        k = np.array([0, 1000, 2000, 3000])
        threads = oracle_threads()
        ref = oracle.impulse_response(sc.table, sc.gamma, sc.rcv[idx[k]], df, bin0, n_bins, eps, n_fft, n_fft,
                                      window=win, c=sc.c, gate=sc.gate, n_threads=threads)
        got = h.cpu().numpy()[:, k, :]
        peak = np.abs(ref).max(axis=-1)
        leg["max_err_rel_to_peak"] = float((np.abs(got - ref).max(axis=-1) / peak).max())
        leg["receivers_checked"] = int(len(k))
    return leg


def trace_bench(sc, dev, args):
    """The ray-tracing stage on the device for the workload's own fan (the
    launch directions are the first segment's axis of every ray): wall time
    of gbs.trace (count pass, prefix sums, write pass, host reads of the
    sizes), the table compared with the workload's input table, and the
    per-ray oracle tracer on a seeded sample of rays on the host."""
    import torch

    import paper_2501_13382_amd as gbs
    tab = sc.table
    kind = tab.meta.get("kind")
    if kind == "open_plane":
        kw = dict(boxes=None, panels=1, s_max=tab.meta["s_max"], max_refl=1, image_complete=True)
    elif kind == "city":
        city = sc.meta["city"]
        kw = dict(boxes=city.boxes, panels=city.panels, s_max=tab.meta["s_max"], max_refl=tab.meta["max_refl"])
    elif "parts" in tab.meta:             # several sources, each with its own arc-length budget
        city = sc.meta["city"]
        parts = tab.meta["parts"]
        kw = dict(boxes=city.boxes, panels=city.panels, s_max=np.array([p["s_max"] for p in parts]),
                  max_refl=parts[0]["max_refl"])
    else:
        return None
    first = tab.ray_ptr[:-1]
    dirs = torch.as_tensor(tab.seg_t[first], device=dev)
    w = torch.as_tensor(tab.ray_w, device=dev)
    src = tab.src_xyz
    rs = torch.as_tensor(tab.ray_src, device=dev)
    t = gbs.trace(src, dirs, w, ray_src=rs, **kw)
    torch.cuda.synchronize()
    ms = []
    for _ in range(5):
        t0 = time.perf_counter()
        t = gbs.trace(src, dirs, w, ray_src=rs, **kw)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    same = {}
    for k in ("ray_ptr", "seg_a", "seg_t", "seg_s0", "seg_lo", "face_ptr", "face_ids"):
        same[k] = bool(np.array_equal(getattr(t, k).cpu().numpy().reshape(np.shape(getattr(tab, k))),
                                      np.asarray(getattr(tab, k))))
    hi = t.seg_hi.cpu().numpy()
    # the open-plane generator writes s_max for the direct beam's end; the
    # general tracer adds the two lengths: equal to rounding
    same["seg_hi_max_rel"] = float(np.max(np.abs(hi - tab.seg_hi) / np.maximum(np.abs(tab.seg_hi), 1e-300)))
    med = float(np.median(ms))
    leg = {"ms_median": med, "ms_min": float(np.min(ms)), "rays": t.n_rays, "segments": t.n_segs,
           "rays_per_s": t.n_rays / (med * 1e-3), "segments_per_s": t.n_segs / (med * 1e-3),
           "matches_input_table": same,
           "note": "wall time of gbs.trace: count pass, prefix sums, host read of the sizes, write pass"}
    print(f"# trace: {med:.2f} ms for {t.n_rays} rays, {t.n_segs} segments", file=sys.stderr, flush=True)
    del t
    if not args.no_cpu:
        from oracle import tracer as ot
        d_host = tab.seg_t[first]
        rng = np.random.default_rng(7)

        def timed(n_s):
            rays = np.sort(rng.choice(tab.n_rays, size=n_s, replace=False))
            t0 = time.perf_counter()
            ot.trace(src, d_host, tab.ray_w, ray_src=tab.ray_src, boxes=kw["boxes"], panels=kw["panels"],
                     s_max=kw["s_max"], max_refl=kw["max_refl"], image_complete=kw.get("image_complete", False),
                     rays=rays)
            return time.perf_counter() - t0

        # a probe of 200 rays sizes a sample of about 3 s
        n_s = min(200, tab.n_rays)
        el = timed(n_s)
        n_s = int(min(tab.n_rays, max(n_s, 3.0 * n_s / max(el, 1e-6))))
        el = timed(n_s)
        leg["cpu_baseline"] = {"value": n_s / el, "unit": "rays/s", "cores": 1, "kind": "oracle",
                               "sample": f"{n_s} of {tab.n_rays} rays (seed 7), one by one; {el:.1f}s"}
    return leg


def workload_leg(key, dev, args):
    """One more workload on the same clock as the headline: the forward (MIX,
    table resident in HBM) timed over a few steps, the pair kernel's roofline,
    the graph replay, and the error against the oracle on a small seeded
    receiver sample, which also times the oracle."""
    import torch

    import paper_2501_13382_amd as gbs
    from scenes import receiver_subsample
    name, build = WORKLOADS[key]
    t0 = time.time()
    sc = build()
    t_build = time.time() - t0
    table = gbs.Table(sc.table, device=dev)
    rcv = torch.as_tensor(sc.rcv, device=dev)
    freqs = torch.as_tensor(sc.freqs, device=dev)
    eps = torch.as_tensor(sc.eps, device=dev)
    gamma = torch.as_tensor(sc.gamma, device=dev)
    dense = sc.dense_pairs
    print(f"# {key}: built in {t_build:.1f}s, {table.n_rays} rays, {table.n_segs} segments", file=sys.stderr,
          flush=True)
    call = lambda **kw: gbs.forward(table, rcv, freqs, eps, gamma, c=sc.c, gate=sc.gate, mode="mix", **kw)
    call()
    torch.cuda.synchronize()
    n = max(2, args.city_steps)
    t = time.perf_counter()
    for _ in range(n):
        P, TL = call()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t) / n
    ms_pairs = []
    for _ in range(2):
        call(time_kernels=True)
        torch.cuda.synchronize()
        ms_pairs.append(gbs.stats(dev)["ms_pairs"])
    call(count_active=True)
    torch.cuda.synchronize()
    st = gbs.stats(dev)
    leg = {"workload": name, "value": dense / sec, "unit": "evals/s", "ms_per_step": sec * 1e3, "steps": n,
           "dense_pairs": dense, "rays": table.n_rays, "segments": table.n_segs, "receivers": int(len(sc.rcv)),
           "bands": int(len(sc.freqs)), "sources": int(table.n_src),
           "roofline": roofline(st["listed_pairs"], st["active_pairs"], float(np.mean(ms_pairs)), "k_pairs<MIX>"),
           "scene_build_s": t_build}
    print(f"# {key}: {sec * 1e3:.1f} ms/step, pair kernel {np.mean(ms_pairs):.1f} ms", file=sys.stderr, flush=True)
    graph = gbs.Graph(table, rcv, freqs, eps, gamma, c=sc.c, gate=sc.gate, mode="mix")
    graph.launch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(n):
        graph.launch()
    torch.cuda.synchronize()
    s_gr = (time.perf_counter() - t) / n
    leg["graph"] = {"value": dense / s_gr, "ms_per_step": s_gr * 1e3, "replays": n}
    del graph
    if not args.no_cpu:
        import oracle
        threads = oracle_threads()
        # about 1e10 oracle pairs (a few seconds on the host) at most
        n_cpu = int(min(256, max(16, 1e10 / (sc.table.n_segs * len(sc.freqs)))))
        idx = receiver_subsample(len(sc.rcv), n=n_cpu, seed=5)
        t = time.perf_counter()
        P_ref, TL_ref, ab = oracle.scene_forward(sc, rcv=sc.rcv[idx], n_threads=threads, return_absum=True)
        el = time.perf_counter() - t
        pairs = sc.table.n_segs * len(idx) * len(sc.freqs)
        Pg = P.cpu().numpy().reshape(-1, len(sc.rcv))[:, idx]
        TLg = TL.cpu().numpy().reshape(-1, len(sc.rcv))[:, idx]
        ok = ab / np.maximum(np.abs(P_ref), 1e-300) <= 1e4
        leg["accuracy_vs_oracle"] = {
            "tl_err_db_max": float(np.abs(TLg - TL_ref)[ok].max()),
            "rel_err_max": float((np.abs(Pg - P_ref) / np.maximum(np.abs(P_ref), 1e-300))[ok].max()),
            "receivers": int(len(idx)), "masked_fraction": float(1.0 - ok.mean())}
        leg["cpu_baseline"] = {"value": pairs / el, "unit": "evals/s", "cores": threads, "kind": "oracle",
                               "sample": f"{len(idx)} of {len(sc.rcv)} receivers (seed 5), all segments; {el:.1f}s",
                               "extrapolated_full_config_s": dense / (pairs / el)}
    del table, P, TL
    torch.cuda.empty_cache()
    return leg


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-f64", action="store_true", help="skip the all-FP64 comparison")
    ap.add_argument("--cpu-receivers", type=int, default=16384)
    ap.add_argument("--cpu1-receivers", type=int, default=512, help="receivers of the single-thread oracle sample")
    ap.add_argument("--no-stream", action="store_true", help="skip the host-streamed table leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--no-trace", action="store_true", help="skip the device ray-tracing leg")
    ap.add_argument("--no-absorption", action="store_true", help="skip the atmospheric-absorption leg")
    ap.add_argument("--no-impulse", action="store_true", help="skip the broadband (impulse response) leg")
    ap.add_argument("--no-aniso", action="store_true", help="skip the anisotropic-beam leg")
    ap.add_argument("--workload", default="open_plane_100k", choices=sorted(WORKLOADS),
                    help="open_plane_100k (default, the headline); city_1m: 10 x 10 city, 1,000,000 rays, "
                         "1024 x 1024 receivers, 1 kHz; city_batched: 16 sources x 4 bands, ragged ray counts, "
                         "replayed as a captured graph")
    ap.add_argument("--no-cities", action="store_true",
                    help="skip the extra workload legs (the 1M-ray city and the 16-source batched city)")
    ap.add_argument("--city-steps", type=int, default=5, help="timed steps of each extra workload leg")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the steps, run one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only (no multi-GPU sharding is implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2501_13382_amd as gbs
    from scenes import receiver_subsample

    dev = torch.device("cuda", 0)
    t0 = time.time()
    workload_name, build = WORKLOADS[args.workload]
    headline = args.workload == "open_plane_100k"
    sc = build()
    table = gbs.Table(sc.table, device=dev)
    rcv = torch.as_tensor(sc.rcv, device=dev)
    freqs = torch.as_tensor(sc.freqs, device=dev)
    eps = torch.as_tensor(sc.eps, device=dev)
    gamma = torch.as_tensor(sc.gamma, device=dev)
    dense = sc.dense_pairs
    print(f"# workload built in {time.time() - t0:.1f}s: {table.n_rays} rays, {table.n_segs} segments, "
          f"{len(sc.rcv)} receivers, {len(sc.freqs)} bands, dense pairs {dense:.3e}", file=sys.stderr, flush=True)

    def step(mode, timed=False, count=False):
        return gbs.forward(table, rcv, freqs, eps, gamma, c=sc.c, gate=sc.gate, mode=mode, time_kernels=timed,
                           count_active=count)

    def run(mode, steps, warmup):
        """Time `steps` forward calls back to back (no synchronisation inside
        the timed region but the library's own list-length read), each also
        bracketed by events on the stream; then the pair kernel's and the
        cull's durations from a few more calls with the library's kernel
        timers (which synchronise, so they stay outside the timed region)."""
        for _ in range(warmup):
            step(mode)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(dev)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t = time.perf_counter()
        for e0, e1 in evs:
            e0.record(stream)
            out = step(mode)
            e1.record(stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        ms_step = [e0.elapsed_time(e1) for e0, e1 in evs]
        ms_pairs, ms_cull = [], []
        for _ in range(3):
            step(mode, timed=True)
            st = gbs.stats(dev)
            ms_pairs.append(st["ms_pairs"])
            ms_cull.append(st["ms_cull"])
        torch.cuda.synchronize()
        run.last = {"ms_cull": float(np.mean(ms_cull)), "grid": st["grid"], "blocks_per_cu": st["blocks_per_cu"],
                    "ms_step_median": float(np.median(ms_step)), "ms_step_min": float(np.min(ms_step))}
        return el / steps, float(np.mean(ms_pairs)), out

    mode = "mix"
    sec_step, ms_pairs, (P, TL) = run(mode, args.steps, args.warmup)
    launch = dict(run.last)
    print(f"# mix: {sec_step * 1e3:.2f} ms/step, pair kernel {ms_pairs:.2f} ms", file=sys.stderr, flush=True)
    step(mode, count=True)
    st = gbs.stats(dev)
    listed, active = st["listed_pairs"], st["active_pairs"]
    roof = roofline(listed, active, ms_pairs, "k_pairs<MIX>")

    stream_leg = None
    if not args.no_stream:
        # the table in pinned host memory, copied in 4 passes that overlap compute (PCIe-inclusive)
        host_table = gbs.Table(sc.table, device=dev, on_host=True)
        chunk = -(-table.n_segs // 4)
        call = lambda: gbs.forward(host_table, rcv, freqs, eps, gamma, c=sc.c, gate=sc.gate, mode=mode,
                                   chunk_segs=chunk)
        call()
        torch.cuda.synchronize()
        t = time.perf_counter()
        n_st = max(2, args.steps // 2)
        for _ in range(n_st):
            call()
        torch.cuda.synchronize()
        s_st = (time.perf_counter() - t) / n_st
        stream_leg = {"value": dense / s_st, "ms_per_step": s_st * 1e3, "passes": gbs.stats(dev)["n_chunks"],
                      "table_bytes": int(sum(np.asarray(v).nbytes for v in (sc.table.seg_a, sc.table.seg_t,
                                             sc.table.seg_s0, sc.table.seg_lo, sc.table.seg_hi)))}
        del host_table
        print(f"# streamed: {s_st * 1e3:.2f} ms/step", file=sys.stderr, flush=True)

    adj_leg = None
    if not args.no_adjoint:
        g = torch.Generator().manual_seed(11)
        lam = torch.complex(torch.randn(P.shape, generator=g, dtype=torch.float64),
                            torch.randn(P.shape, generator=g, dtype=torch.float64)).to(dev)
        bwd = lambda: gbs.backward(table, rcv, freqs, eps, gamma, lam, c=sc.c, gate=sc.gate, mode=mode)
        bwd()
        torch.cuda.synchronize()
        t = time.perf_counter()
        n_adj = max(2, args.steps // 4)
        for _ in range(n_adj):
            bwd()
        torch.cuda.synchronize()
        s_adj = (time.perf_counter() - t) / n_adj
        gbs.backward(table, rcv, freqs, eps, gamma, lam, c=sc.c, gate=sc.gate, mode=mode, time_kernels=True)
        ms_adj_kernel = gbs.stats(dev)["ms_pairs"]
        adj_leg = {"value": dense / s_adj, "ms_per_call": s_adj * 1e3, "mode": mode,
                   "forward_plus_adjoint_ms": sec_step * 1e3 + s_adj * 1e3,
                   "roofline": roofline(listed, active, ms_adj_kernel, "k_adjoint<MIX>",
                                        f64_kept=ADJ_FLOP_KEPT_F64, f32_kept=ADJ_FLOP_KEPT_F32, survey=False)}
        print(f"# adjoint: {s_adj * 1e3:.2f} ms/call", file=sys.stderr, flush=True)

    # the same forward captured once as a hipGraph and replayed (the lists are
    # planned at capture: a replay re-runs records, pair kernel, reduction, TL)
    graph = gbs.Graph(table, rcv, freqs, eps, gamma, c=sc.c, gate=sc.gate, mode=mode)
    graph.launch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    n_gr = max(2, args.steps // 2)
    for _ in range(n_gr):
        graph.launch()
    torch.cuda.synchronize()
    s_gr = (time.perf_counter() - t) / n_gr
    graph_leg = {"value": dense / s_gr, "ms_per_step": s_gr * 1e3, "replays": n_gr,
                 "note": "culled lists built at capture (fixed geometry); replays re-run records, pairs, reduce, TL"}
    del graph
    print(f"# graph replay: {s_gr * 1e3:.2f} ms/step", file=sys.stderr, flush=True)

    absorption_leg = None
    if not args.no_absorption:
        absorption_leg = absorption_bench(sc, dev, table, rcv, freqs, eps, gamma, args, sec_step)

    aniso_leg = None
    if not args.no_aniso:
        aniso_leg = aniso_bench(sc, dev, table, rcv, freqs, eps, gamma, args, sec_step)

    impulse_leg = None
    if not args.no_impulse and sc.table.meta.get("kind") == "open_plane":
        impulse_leg = impulse_bench(sc, dev, table, gamma, args)

    trace_leg = None
    if not args.no_trace:
        trace_leg = trace_bench(sc, dev, args)

    f64_leg = None
    if not args.no_f64:
        s64, ms64, _ = run("f64", max(2, args.steps // 2), 1)
        f64_leg = {"value": dense / s64, "ms_per_step": s64 * 1e3, "ms_pair_kernel": ms64,
                   "mix_speedup": s64 / sec_step}
        print(f"# f64: {s64 * 1e3:.2f} ms/step", file=sys.stderr, flush=True)

    workloads = {}
    if not args.no_cities:
        for key in ("city_1m", "city_batched"):
            if key != args.workload:
                workloads[key] = workload_leg(key, dev, args)

    result = {
        "metric": "GBS segment x receiver evals/s, % FP32 VALU peak; TL error dB vs FP64 oracle",
        "value": dense / sec_step,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 geometry+phase / f32 beam terms",
        "data": "synthetic (seeded tracer)",
        "config": {"workload": workload_name, "rays": table.n_rays, "segments": table.n_segs,
                   "receivers": int(len(sc.rcv)), "bands": int(len(sc.freqs)), "mode": mode,
                   "dense_pairs": dense, "parallelism": "single GPU"},
        "roofline": dict(roof, traffic=pair_traffic() if headline else None),
        "pair_kernel_share": ms_pairs / (sec_step * 1e3),
        "ms_step_median": launch["ms_step_median"],
        "ms_step_min": launch["ms_step_min"],
        "ms_cull": launch["ms_cull"],
        "pairs": {"listed_per_s": listed / sec_step, "kept_per_s": active / sec_step,
                  "culled_fraction": 1.0 - listed / dense, "kept_fraction_of_listed": active / max(listed, 1)},
        "launch": {"grid": launch["grid"], "blocks_per_cu": launch["blocks_per_cu"], "threads_per_block": 256},
        "f64": f64_leg,
        "graph": graph_leg,
        "streamed": stream_leg,
        "adjoint": adj_leg,
        "trace": trace_leg,
        "absorption": absorption_leg,
        "anisotropic": aniso_leg,
        "impulse_response": impulse_leg,
        "workloads": workloads,
    }

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        dst = src.clone()
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = int(n * 8)
        del src, dst

    # accuracy on a seeded receiver subsample, and the oracle timed on this host
    # about 2.5e10 oracle pairs (10-30 s on the host) at most
    n_cpu = int(min(args.cpu_receivers, max(64, 2.5e10 / (table.n_segs * len(sc.freqs)))))
    idx = receiver_subsample(len(sc.rcv), n=n_cpu, seed=5)
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        threads = oracle_threads()
        print(f"# oracle, {threads} threads, {len(idx)} receivers", file=sys.stderr, flush=True)
        t = time.perf_counter()
        P_ref, TL_ref, ab = oracle.scene_forward(sc, rcv=sc.rcv[idx], n_threads=threads, return_absum=True)
        el = time.perf_counter() - t
        pairs = table.n_segs * len(idx) * len(sc.freqs)
        result["cpu_baseline"] = {"value": pairs / el, "unit": "evals/s", "cores": threads, "kind": "oracle",
                                  "cpu_model": cpu_model(), "host_cpus": host_cpus(),
                                  "sample": f"{len(idx)} of {len(sc.rcv)} receivers (seed 5), all "
                                            f"{table.n_segs} segments, {len(sc.freqs)} bands; {el:.1f}s",
                                  "extrapolated_full_config_s": dense / (pairs / el)}
        if args.cpu1_receivers > 0:
            # about 8e8 oracle pairs (a few seconds on one core) at most
            n1 = int(min(args.cpu1_receivers, max(8, 8e8 / (table.n_segs * len(sc.freqs)))))
            print(f"# oracle, 1 thread, {n1} receivers", file=sys.stderr, flush=True)
            idx1 = receiver_subsample(len(sc.rcv), n=n1, seed=6)
            t = time.perf_counter()
            oracle.scene_forward(sc, rcv=sc.rcv[idx1], n_threads=1)
            el1 = time.perf_counter() - t
            result["cpu_baseline"]["single_thread"] = {
                "value": table.n_segs * len(idx1) * len(sc.freqs) / el1, "cores": 1,
                "sample": f"{len(idx1)} receivers (seed 6); {el1:.1f}s"}
        Pg = P.cpu().numpy().reshape(-1, len(sc.rcv))[:, idx]
        TLg = TL.cpu().numpy().reshape(-1, len(sc.rcv))[:, idx]
        mag = np.abs(P_ref)
        ok = ab / np.maximum(mag, 1e-300) <= 1e4
        dtl = np.abs(TLg - TL_ref)[ok]
        rel = (np.abs(Pg - P_ref) / np.maximum(mag, 1e-300))[ok]
        result["accuracy_vs_oracle"] = {"tl_err_db_max": float(dtl.max()), "tl_err_db_p99": float(
            np.percentile(dtl, 99)), "tl_err_db_median": float(np.median(dtl)), "rel_err_max": float(rel.max()),
            "rel_err_p99": float(np.percentile(rel, 99)), "rel_err_median": float(np.median(rel)),
            "receivers": int(len(idx)), "masked_fraction": float(1.0 - ok.mean())}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
