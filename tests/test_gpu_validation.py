"""The error contract of the C ABI on the default path: array contents that
break the table's invariants are rejected with GBS_E_INVALID, by the host or
by the kernels that read them (a device status word read before any beam is
evaluated).  Every case here is one the library rejects without reading
outside an array; a valid call on the same context afterwards still matches
the oracle."""
import copy

import numpy as np
import pytest
import torch

import paper_2501_13382_amd as gbs
from paper_2501_13382_amd import _lib
from scenes import city_scene, open_plane
from tests.gpu_util import assert_within, compare, reference

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def city():
    # a small city: face histories of several entries, several rays per source
    return city_scene(n_blocks=2, n_rays=400, grid=6, freqs=(500.0,), max_refl=4, city_seed=5)


def _rejects(tab, sc, rcv=None, **kw):
    t = gbs.Table(tab, device="cuda")
    with pytest.raises(_lib.GbsError) as e:
        gbs.forward(t, sc.rcv if rcv is None else rcv, sc.freqs, sc.eps, kw.pop("gamma", sc.gamma), c=sc.c,
                    gate=sc.gate, mode="mix", **kw)
        torch.cuda.synchronize()
    assert e.value.code == _lib.GBS_E_INVALID, str(e.value)
    return str(e.value)


def _with(tab, **fields):
    t = copy.copy(tab)
    for k, v in fields.items():
        setattr(t, k, v)
    return t


def test_segment_values_rejected(city):
    tab = city.table
    print("case validation: segment values", flush=True)
    assert "segment values" in _rejects(_with(tab, seg_t=tab.seg_t * 1.01), city)
    lo = tab.seg_lo.copy()
    lo[3] = tab.seg_hi[3] + 1.0
    assert "segment values" in _rejects(_with(tab, seg_lo=lo), city)
    a = tab.seg_a.copy()
    a[5, 1] = np.nan
    assert "segment values" in _rejects(_with(tab, seg_a=a), city)
    s0 = tab.seg_s0.copy()
    s0[-1] = np.inf
    assert "segment values" in _rejects(_with(tab, seg_s0=s0), city)


def test_face_histories_rejected(city):
    tab = city.table
    assert len(tab.face_ids) > 10
    print("case validation: face histories", flush=True)
    for bad_id in (tab.n_faces, -1):
        ids = tab.face_ids.copy()
        ids[len(ids) // 2] = bad_id
        assert "face id" in _rejects(_with(tab, face_ids=ids), city)
    # non-decreasing face_ptr: one entry moved past its successor
    fp = tab.face_ptr.copy()
    j = int(np.argmax(np.diff(fp) > 0))
    fp[j + 1] = fp[j + 2] + 1
    assert "face_ptr" in _rejects(_with(tab, face_ptr=fp), city)
    fp = tab.face_ptr.copy()
    fp[0] = 1
    assert "face_ptr" in _rejects(_with(tab, face_ptr=fp), city)
    # histories without faces (n_faces = 0): rejected on the host
    assert "n_faces" in _rejects(_with(tab, n_faces=0), city, gamma=np.zeros(0, np.complex128))


def test_ray_table_rejected(city):
    tab = city.table
    print("case validation: rays", flush=True)
    rp = tab.ray_ptr.copy()
    rp[2], rp[3] = rp[3], rp[2] - 1
    assert "ray_ptr" in _rejects(_with(tab, ray_ptr=rp), city)
    rp = tab.ray_ptr.copy()
    rp[-1] -= 1
    assert "ray_ptr" in _rejects(_with(tab, ray_ptr=rp), city)
    w = tab.ray_w.copy()
    w[7] = np.nan
    assert "ray weight" in _rejects(_with(tab, ray_w=w), city)
    w = tab.ray_w.copy()
    w[7] = -1e-3
    assert "ray weight" in _rejects(_with(tab, ray_w=w), city)
    rs = tab.ray_src.copy()
    rs[4] = 1                      # one source only
    assert "ray_src" in _rejects(_with(tab, ray_src=rs), city)


def test_receivers_rejected(city):
    print("case validation: receivers", flush=True)
    for v in (np.nan, np.inf):
        r = city.rcv.copy()
        r[11, 2] = v
        assert "receiver" in _rejects(city.table, city, rcv=r)


def test_backward_rejects_non_finite_lambda(city):
    print("case validation: lambda", flush=True)
    t = gbs.Table(city.table, device="cuda")
    lam = np.ones((1, len(city.rcv)), np.complex128)
    lam[0, 3] = np.nan
    with pytest.raises(_lib.GbsError) as e:
        gbs.backward(t, city.rcv, city.freqs, city.eps, city.gamma, lam, c=city.c, gate=city.gate, mode="f64")
    assert e.value.code == _lib.GBS_E_INVALID and "lambda" in str(e.value)


def test_valid_call_after_rejections(city):
    """The context stays usable: a valid call right after rejected ones."""
    print("case validation: valid call after rejections", flush=True)
    _rejects(_with(city.table, seg_t=city.table.seg_t * 1.01), city)
    P_ref, TL_ref, ab = reference(city)
    t = gbs.Table(city.table, device="cuda")
    P, TL = gbs.forward(t, city.rcv, city.freqs, city.eps, city.gamma, c=city.c, gate=city.gate, mode="f64")
    torch.cuda.synchronize()
    assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), "f64")


def test_host_table_checks_on_the_host():
    sc = open_plane(n_rays=300, grid=4, half=40.0, freqs=(500.0,))
    tab = sc.table
    fp = tab.face_ptr.copy()
    j = int(np.argmax(np.diff(fp) > 0))
    fp[j + 1] = fp[j + 2] + 1
    t = gbs.Table(_with(tab, face_ptr=fp), device="cuda", on_host=True)
    with pytest.raises(_lib.GbsError) as e:
        gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="mix")
    assert e.value.code == _lib.GBS_E_INVALID and "face_ptr" in str(e.value)
