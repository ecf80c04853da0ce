"""Helpers shared by the GPU parity tests (not collected)."""
import os

import numpy as np

import oracle

TL_MASK_KAPPA = 1e4        # TL tolerances apply where sum|u| / |P| <= 1e4
TOL = {
    # mode: (max relative complex error, max |dTL| dB)
    "f64": (1e-9, 1e-6),
    "mix": (1e-4, 0.05),
    "f32": (None, 0.2),
}


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "16"))


def reference(sc, rcv=None, table=None, gamma=None, eps=None):
    tab = sc.table if table is None else table
    P, TL, ab = oracle.forward(tab, sc.gamma if gamma is None else gamma, sc.rcv if rcv is None else rcv,
                               sc.freqs, sc.eps if eps is None else eps, c=sc.c, gate=sc.gate,
                               n_threads=oracle_threads(), return_absum=True)
    return P, TL, ab


def compare(P, TL, P_ref, TL_ref, absum):
    """Error statistics of a GPU result against the oracle (job-major arrays)."""
    P = np.asarray(P).reshape(P_ref.shape)
    TL = np.asarray(TL).reshape(TL_ref.shape)
    mag = np.abs(P_ref)
    live = absum > 0
    kappa = np.where(live, absum / np.maximum(mag, 1e-300), 0.0)
    ok = live & (kappa <= TL_MASK_KAPPA)
    d = np.abs(P - P_ref)
    rel = np.where(ok, d / np.maximum(mag, 1e-300), 0.0)
    dtl = np.zeros_like(TL_ref)
    dtl[ok] = np.abs(TL[ok] - TL_ref[ok])
    dead = ~live
    return {
        "rel_max": float(rel.max()) if rel.size else 0.0,
        "dtl_max": float(dtl.max()) if dtl.size else 0.0,
        # share of receivers with a beam whose TL is too cancelled to compare
        "masked_frac": float(1.0 - ok.sum() / max(live.sum(), 1)),
        "dead_ok": bool(np.all(P[dead] == 0)),
    }


def assert_within(stats, mode):
    rel_tol, dtl_tol = TOL[mode]
    assert stats["dead_ok"], "receivers with no beam must get exactly zero"
    if rel_tol is not None:
        assert stats["rel_max"] <= rel_tol, (mode, stats)
    assert stats["dtl_max"] <= dtl_tol, (mode, stats)
    assert stats["masked_frac"] <= 0.01, stats
