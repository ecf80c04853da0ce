"""Benchmark: Gaussian beam summation throughput on one MI355X.

Workload: the 100,000-ray open plane (Fibonacci fan from 10 m over a ground
with coefficient 0.8 exp(i pi/8), eight octave bands 63 Hz - 8 kHz, 512 x 512
receivers at 1.5 m over 2 x 2 km), seeded and synthetic.  One step is one
full forward call of the library (receiver ordering, segment records, culled
work lists, persistent pair kernel, TL) in the FP32 + FP64-phase mode with
the table resident in HBM.  `value` = dense segment x receiver x band
evaluations per second (the dense sum the culled kernel reproduces).

Also reported: the pair kernel's roofline (algorithmic FLOPs per launch over
its HIP-event-timed duration), the all-FP64 mode on the same GPU, the error
against the FP64 oracle on 16,384 seeded receivers, and the oracle timed on
this host's cores on that sample.
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
# formulas (an FMA counts 2; a transcendental, a reciprocal or a fract 1):
#   gate, every listed pair:  s (3 FMA), |R-o|^2 (3 FMA), rhs (mul, FMA, add)   -> 16 FP64
#   beam term, every kept pair: n^2, den, Newton reciprocal, phase in cycles,
#       fract, FP64 accumulation                                            -> 17 FP64
#     rcp, sin, cos, exp2, Gaussian, amplitude and complex products         -> 21 FP32
FLOP_LISTED_F64 = 16
FLOP_KEPT_F64 = 17
FLOP_KEPT_F32 = 21
# Vector peaks from unit counts and clock: 256 CUs x 2.4 GHz x 64 FMA lanes x 2
# = 78.6 TFLOP/s FP64; FP32 157.3 TFLOP/s (vendor figure).
PEAK_F64 = 256 * 2.4e9 * 64 * 2
PEAK_F32 = 157.3e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-f64", action="store_true", help="skip the all-FP64 comparison")
    ap.add_argument("--cpu-receivers", type=int, default=16384)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the steps, run one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2501_13382_amd as gbs
    from scenes import open_plane_100k, receiver_subsample

    dev = torch.device("cuda", 0)
    t0 = time.time()
    sc = open_plane_100k()
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
        for _ in range(warmup):
            step(mode)
        torch.cuda.synchronize()
        ms_pairs, ms_cull = [], []
        t = time.perf_counter()
        for _ in range(steps):
            out = step(mode, timed=True)
            st = gbs.stats(dev)
            ms_pairs.append(st["ms_pairs"])
            ms_cull.append(st["ms_cull"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        run.last = {"ms_cull": float(np.mean(ms_cull)), "grid": st["grid"], "blocks_per_cu": st["blocks_per_cu"]}
        return el / steps, float(np.mean(ms_pairs)), out

    mode = "mix"
    sec_step, ms_pairs, (P, TL) = run(mode, args.steps, args.warmup)
    launch = dict(run.last)
    print(f"# mix: {sec_step * 1e3:.2f} ms/step, pair kernel {ms_pairs:.2f} ms", file=sys.stderr, flush=True)
    step(mode, count=True)
    st = gbs.stats(dev)
    listed, active = st["listed_pairs"], st["active_pairs"]
    f64 = FLOP_LISTED_F64 * listed + FLOP_KEPT_F64 * active
    f32 = FLOP_KEPT_F32 * active
    flops = f64 + f32
    achieved = flops / (ms_pairs * 1e-3)
    # peak for this kernel's FP64/FP32 mix: time at peak = f64/PEAK_F64 + f32/PEAK_F32
    peak = flops / (f64 / PEAK_F64 + f32 / PEAK_F32)

    f64_leg = None
    if not args.no_f64:
        s64, ms64, _ = run("f64", max(2, args.steps // 2), 1)
        f64_leg = {"value": dense / s64, "ms_per_step": s64 * 1e3, "ms_pair_kernel": ms64,
                   "mix_speedup": s64 / sec_step}
        print(f"# f64: {s64 * 1e3:.2f} ms/step", file=sys.stderr, flush=True)

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
        "config": {"workload": "open_plane_100k_8band", "rays": table.n_rays, "segments": table.n_segs,
                   "receivers": int(len(sc.rcv)), "bands": int(len(sc.freqs)), "mode": mode,
                   "dense_pairs": dense, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "k_pairs<MIX>", "achieved": achieved / 1e12,
                     "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
                     "frac_of_fp32_peak": achieved / PEAK_F32, "frac_of_fp64_peak": achieved / PEAK_F64,
                     "traffic": None, "ms_per_launch": ms_pairs, "listed_pairs": listed, "kept_pairs": active,
                     "flop_per_listed_pair": {"f64": FLOP_LISTED_F64},
                     "flop_per_kept_pair": {"f64": FLOP_KEPT_F64, "f32": FLOP_KEPT_F32}},
        "pair_kernel_share": ms_pairs / (sec_step * 1e3),
        "ms_cull": launch["ms_cull"],
        "launch": {"grid": launch["grid"], "blocks_per_cu": launch["blocks_per_cu"], "threads_per_block": 256},
        "f64": f64_leg,
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
    idx = receiver_subsample(len(sc.rcv), n=args.cpu_receivers, seed=5)
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        threads = int(os.environ.get("OMP_NUM_THREADS", str(min(16, os.cpu_count() or 1))))
        t = time.perf_counter()
        P_ref, TL_ref, ab = oracle.scene_forward(sc, rcv=sc.rcv[idx], n_threads=threads, return_absum=True)
        el = time.perf_counter() - t
        pairs = table.n_segs * len(idx) * len(sc.freqs)
        result["cpu_baseline"] = {"value": pairs / el, "unit": "evals/s", "cores": threads, "kind": "oracle",
                                  "sample": f"{len(idx)} of {len(sc.rcv)} receivers (seed 5), all "
                                            f"{table.n_segs} segments, {len(sc.freqs)} bands; {el:.1f}s"}
        Pg = P.cpu().numpy().reshape(len(sc.freqs), -1)[:, idx]
        TLg = TL.cpu().numpy().reshape(len(sc.freqs), -1)[:, idx]
        mag = np.abs(P_ref)
        ok = ab / np.maximum(mag, 1e-300) <= 1e4
        dtl = np.abs(TLg - TL_ref)[ok]
        rel = (np.abs(Pg - P_ref) / np.maximum(mag, 1e-300))[ok]
        result["accuracy_vs_oracle"] = {"tl_err_db_max": float(dtl.max()), "tl_err_db_p99": float(
            np.percentile(dtl, 99)), "rel_err_max": float(rel.max()), "receivers": int(len(idx))}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
