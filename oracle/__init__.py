"""FP64 CPU oracle for Gaussian beam summation (ctypes binding).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may use this package; the library under test never does.  The C
source (gbs_oracle.c) is the plain definition of the sum (paper Sec. 2,
Eqs. (1)-(3)), with an optional per-job atmospheric absorption exp(-alpha s)
(the atmosphere of Tables 2 and 3 through ISO 9613-1) and optional
anisotropic beams (a diagonal 2x2 Q in each segment's ray frame); this module only
marshals numpy arrays to it and builds it.  oracle/tracer.py is the oracle
of the ray-tracing stage.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gbs_oracle.c")
_LIB = os.path.join(_HERE, "libgbs_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-Wall", "-shared", "-fPIC", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        common = [i32, i64, P, P, P, i64, P, P, P, P, P, P, P, i32, P, i64, P, i32, P, P, P, f64, f64]
        lib.gbso_forward.argtypes = common + [i32, i32, P, P, P, P]
        lib.gbso_forward.restype = ctypes.c_int
        lib.gbso_forward_aniso.argtypes = common + [P, P, i32, i32, P, P, P, P]
        lib.gbso_forward_aniso.restype = ctypes.c_int
        lib.gbso_backward.argtypes = common + [P, i32, P, P, P, P]
        lib.gbso_backward.restype = ctypes.c_int
        lib.gbso_backward_aniso.argtypes = common + [P, P, P, i32, P, P, P, P, P]
        lib.gbso_backward_aniso.restype = ctypes.c_int
        lib.gbso_air_absorption_db.argtypes = [f64, f64, f64, f64]
        lib.gbso_air_absorption_db.restype = f64
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _table_args(table, gamma, rcv, freqs, eps, c, gate, alpha=None):
    arrs = dict(
        ray_ptr=np.ascontiguousarray(table.ray_ptr, np.int64),
        ray_w=np.ascontiguousarray(table.ray_w, np.float64),
        ray_src=np.ascontiguousarray(table.ray_src, np.int32),
        a=np.ascontiguousarray(table.seg_a, np.float64),
        t=np.ascontiguousarray(table.seg_t, np.float64),
        s0=np.ascontiguousarray(table.seg_s0, np.float64),
        lo=np.ascontiguousarray(table.seg_lo, np.float64),
        hi=np.ascontiguousarray(table.seg_hi, np.float64),
        face_ptr=np.ascontiguousarray(table.face_ptr, np.int64),
        face_ids=np.ascontiguousarray(table.face_ids, np.int32),
        gamma=np.ascontiguousarray(np.stack([np.real(gamma), np.imag(gamma)], axis=-1).reshape(-1), np.float64),
        rcv=np.ascontiguousarray(rcv, np.float64).reshape(-1, 3),
        freqs=np.ascontiguousarray(freqs, np.float64).reshape(-1),
        eps=np.ascontiguousarray(eps, np.float64).reshape(-1),
        alpha=None if alpha is None else np.ascontiguousarray(alpha, np.float64).reshape(-1),
    )
    if arrs["eps"].shape[0] != table.n_src * arrs["freqs"].shape[0]:
        raise ValueError("eps must hold one value per (source, band) job")
    if arrs["alpha"] is not None and arrs["alpha"].shape[0] != arrs["eps"].shape[0]:
        raise ValueError("alpha must hold one value per (source, band) job")
    if len(gamma) != table.n_faces:
        raise ValueError("gamma must hold one coefficient per face")
    args = [table.n_src, table.n_rays, _ptr(arrs["ray_ptr"]), _ptr(arrs["ray_w"]), _ptr(arrs["ray_src"]),
            table.n_segs, _ptr(arrs["a"]), _ptr(arrs["t"]), _ptr(arrs["s0"]), _ptr(arrs["lo"]), _ptr(arrs["hi"]),
            _ptr(arrs["face_ptr"]), _ptr(arrs["face_ids"]), table.n_faces, _ptr(arrs["gamma"]),
            arrs["rcv"].shape[0], _ptr(arrs["rcv"]), arrs["freqs"].shape[0], _ptr(arrs["freqs"]),
            _ptr(arrs["eps"]), _ptr(arrs["alpha"]), float(c), float(gate)]
    return args, arrs


def forward(table, gamma, rcv, freqs, eps, c=343.0, gate=9.21, n_threads=1, mask_mode=0, mask=None,
            return_absum=False, alpha=None, eps_e2=None, seg_e1=None):
    """P [n_jobs, n_rcv] complex128 and TL [n_jobs, n_rcv] float64.

    mask_mode 1 records the active (job, receiver, segment) set into `mask`
    (uint8, shape [n_jobs, n_rcv, n_segs]); mask_mode 2 evaluates with that set
    frozen instead of the gate.  return_absum adds sum |u| per output (the
    scale against which cancellation in P is judged).  alpha: atmospheric
    absorption per job in Np/m (amplitude factor exp(-alpha s)), or None.
    eps_e2 and seg_e1 (given together) select anisotropic beams: eps is then
    the beam parameter along each segment's unit normal e1 (seg_e1, [n_segs, 3])
    and eps_e2 (one per job) the one along e2 = t x e1.
    """
    args, arrs = _table_args(table, gamma, rcv, freqs, eps, c, gate, alpha)
    n_jobs = table.n_src * arrs["freqs"].shape[0]
    n_rcv = arrs["rcv"].shape[0]
    P = np.zeros((n_jobs, n_rcv, 2), np.float64)
    TL = np.zeros((n_jobs, n_rcv), np.float64)
    if mask_mode:
        if mask is None or mask.dtype != np.uint8 or mask.size != n_jobs * n_rcv * table.n_segs:
            raise ValueError("mask must be uint8 [n_jobs, n_rcv, n_segs]")
    absum = np.zeros((n_jobs, n_rcv), np.float64) if return_absum else None
    if (eps_e2 is None) != (seg_e1 is None):
        raise ValueError("eps_e2 and seg_e1 go together")
    if eps_e2 is not None:
        e2 = np.ascontiguousarray(eps_e2, np.float64).reshape(-1)
        f1 = np.ascontiguousarray(seg_e1, np.float64).reshape(-1, 3)
        if e2.shape[0] != n_jobs or f1.shape[0] != table.n_segs:
            raise ValueError("eps_e2 needs one value per job and seg_e1 one frame vector per segment")
        rc = _load().gbso_forward_aniso(*args, _ptr(e2), _ptr(f1), int(n_threads), int(mask_mode), _ptr(mask),
                                        _ptr(P), _ptr(TL), _ptr(absum))
    else:
        rc = _load().gbso_forward(*args, int(n_threads), int(mask_mode), _ptr(mask), _ptr(P), _ptr(TL), _ptr(absum))
    if rc != 0:
        raise RuntimeError(f"gbso_forward failed ({rc})")
    if return_absum:
        return P[..., 0] + 1j * P[..., 1], TL, absum
    return P[..., 0] + 1j * P[..., 1], TL


def backward(table, gamma, rcv, freqs, eps, lam, c=343.0, gate=9.21, mask_mode=0, mask=None, alpha=None,
             eps_e2=None, seg_e1=None):
    """Hand adjoint for dL = Re sum lam * dP.

    Returns (d_gamma [n_faces, 2] = (dL/dRe, dL/dIm), d_rcv [n_rcv, 3],
    d_eps [n_jobs]); with anisotropic beams (eps_e2 and seg_e1 as for
    forward) also d_eps_e2 [n_jobs]."""
    args, arrs = _table_args(table, gamma, rcv, freqs, eps, c, gate, alpha)
    n_jobs = table.n_src * arrs["freqs"].shape[0]
    n_rcv = arrs["rcv"].shape[0]
    lam = np.asarray(lam, np.complex128).reshape(n_jobs, n_rcv)
    lam_ri = np.ascontiguousarray(np.stack([lam.real, lam.imag], axis=-1))
    d_gamma = np.zeros((table.n_faces, 2), np.float64)
    d_rcv = np.zeros((n_rcv, 3), np.float64)
    d_eps = np.zeros(n_jobs, np.float64)
    if (eps_e2 is None) != (seg_e1 is None):
        raise ValueError("eps_e2 and seg_e1 go together")
    if eps_e2 is not None:
        e2 = np.ascontiguousarray(eps_e2, np.float64).reshape(-1)
        f1 = np.ascontiguousarray(seg_e1, np.float64).reshape(-1, 3)
        if e2.shape[0] != n_jobs or f1.shape[0] != table.n_segs:
            raise ValueError("eps_e2 needs one value per job and seg_e1 one frame vector per segment")
        d_eps2 = np.zeros(n_jobs, np.float64)
        rc = _load().gbso_backward_aniso(*args, _ptr(e2), _ptr(f1), _ptr(lam_ri), int(mask_mode), _ptr(mask),
                                         _ptr(d_gamma), _ptr(d_rcv), _ptr(d_eps), _ptr(d_eps2))
        if rc != 0:
            raise RuntimeError(f"gbso_backward_aniso failed ({rc})")
        return d_gamma, d_rcv, d_eps, d_eps2
    rc = _load().gbso_backward(*args, _ptr(lam_ri), int(mask_mode), _ptr(mask), _ptr(d_gamma), _ptr(d_rcv),
                               _ptr(d_eps))
    if rc != 0:
        raise RuntimeError(f"gbso_backward failed ({rc})")
    return d_gamma, d_rcv, d_eps


def scene_forward(scene, rcv=None, gamma=None, eps=None, n_threads=1, return_absum=False, alpha=None):
    """Forward on a scenes.Scene (optionally a receiver subset / other gamma)."""
    return forward(scene.table, scene.gamma if gamma is None else gamma, scene.rcv if rcv is None else rcv,
                   scene.freqs, scene.eps if eps is None else eps, c=scene.c, gate=scene.gate,
                   n_threads=n_threads, return_absum=return_absum, alpha=alpha)


def air_absorption_db(freqs, temp_c=20.0, rh=70.0, p_atm=1.0):
    """Pure-tone atmospheric attenuation (ISO 9613-1) in dB/m per frequency."""
    lib = _load()
    return np.array([lib.gbso_air_absorption_db(float(f), float(temp_c), float(rh), float(p_atm))
                     for f in np.atleast_1d(np.asarray(freqs, np.float64))])


def air_absorption(freqs, temp_c=20.0, rh=70.0, p_atm=1.0):
    """The same as an amplitude decay rate alpha in Np/m: |p| ~ exp(-alpha s)."""
    return air_absorption_db(freqs, temp_c, rh, p_atm) * np.log(10.0) / 20.0


def impulse_response(table, gamma, rcv, df, bin0, n_bins, eps, n_fft, n_t, window=None, c=343.0, gate=9.21,
                     alpha=None, n_threads=1):
    """Broadband synthesis: the time-domain form of the beam sum.  The
    spectrum is the forward sum at f_n = (bin0 + n) df, n < n_bins (eps and
    alpha per (source, bin)); with the exp(-i omega t) convention of Eq. (1)
    the real pressure at time t is (1/pi) Re of the integral of
    P(omega) exp(-i omega t) over omega > 0, discretised as
        h[m] = 2 df Re sum_n w_n P_n exp(-2 pi i f_n m dt),  dt = 1 / (n_fft df),
    for m < n_t.  Evaluated with numpy's FFT of the zero-padded spectrum.
    Returns h [n_src, n_rcv, n_t]."""
    freqs = (bin0 + np.arange(n_bins)) * float(df)
    P, _ = forward(table, gamma, rcv, freqs, eps, c=c, gate=gate, n_threads=n_threads, alpha=alpha)
    n_rcv = np.asarray(rcv).reshape(-1, 3).shape[0]
    P = P.reshape(table.n_src, n_bins, n_rcv)
    w = np.ones(n_bins) if window is None else np.asarray(window, np.float64)
    X = np.zeros((table.n_src, n_rcv, n_fft), np.complex128)
    X[:, :, bin0:bin0 + n_bins] = np.transpose(P, (0, 2, 1)) * w[None, None, :]
    return 2.0 * float(df) * np.real(np.fft.fft(X, axis=-1))[:, :, :n_t]
