"""The allocation-free forward (gbs_forward_noalloc) through the C ABI.

Its result is compared with gbs_forward's on the same inputs (bitwise: the
same plan and kernels run, only the scratch memory differs) and with the
FP64 oracle to the parity bar of each mode, on two calls in a row whose
second input is smaller (fewer rays, fewer ragged receivers, more bands),
so that the second call runs on the scratch the first one left behind.
"""
import numpy as np
import pytest
import torch

import paper_2501_13382_amd as gbs
from paper_2501_13382_amd import _lib
from scenes import city_scene, open_plane, receiver_grid
from tests.gpu_util import assert_within, compare, reference

pytestmark = pytest.mark.gpu

SCRATCH_LIMIT = 128 << 20


def _cases():
    big = open_plane(n_rays=3000, grid=64, half=150.0, freqs=(500.0,), gamma_ground=0.8 * np.exp(1j * np.pi / 8))
    small = open_plane(n_rays=1200, grid=2, half=150.0, freqs=(125.0, 1000.0, 4000.0),
                       gamma_ground=0.9 * np.exp(-1j * np.pi / 5))
    rng = np.random.default_rng(23)
    n = 777
    rcv = np.stack([rng.uniform(-150, 150, n), rng.uniform(-150, 150, n), rng.uniform(0.5, 12, n)], 1)
    return (big, big.rcv), (small, rcv)


@pytest.mark.parametrize("mode", ["f64", "mix"])
def test_noalloc_matches_forward_and_oracle_on_two_calls(mode):
    for k, (sc, rcv) in enumerate(_cases()):
        print(f"case noalloc call={k} mode={mode} segs={sc.table.n_segs} rcv={len(rcv)} bands={len(sc.freqs)}",
              flush=True)
        t = gbs.Table(sc.table, device="cuda")
        P0, TL0 = gbs.forward(t, rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode=mode)
        torch.cuda.synchronize()
        held = gbs.stats()["scratch_bytes"]
        P1, TL1 = gbs.forward_noalloc(t, rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode=mode)
        torch.cuda.synchronize()
        used = gbs.stats()["scratch_bytes"]
        print(f"  workspace {held} B, static scratch used {used} B", flush=True)
        assert 0 < used <= SCRATCH_LIMIT
        P0, TL0, P1, TL1 = (x.cpu().numpy() for x in (P0, TL0, P1, TL1))
        assert np.array_equal(P0, P1) and np.array_equal(TL0, TL1)
        P_ref, TL_ref, ab = reference(sc, rcv=rcv)
        assert_within(compare(P1, TL1, P_ref, TL_ref, ab), mode)


def test_noalloc_city_into_caller_outputs():
    """A small city (reflections off walls and roofs, several face ids per
    segment) written into caller-owned outputs, twice: the second call with
    fewer receivers into a smaller output."""
    sc = city_scene(n_blocks=3, n_rays=6000, grid=24, freqs=(250.0, 1000.0), max_refl=4, city_seed=7)
    t = gbs.Table(sc.table, device="cuda")
    for n in (len(sc.rcv), 301):
        rcv = sc.rcv[:n]
        print(f"case noalloc city rcv={n}", flush=True)
        P0, TL0 = gbs.forward(t, rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="mix")
        out = (torch.full((1, len(sc.freqs), n, 2), np.nan, dtype=torch.float64, device="cuda"),
               torch.full((1, len(sc.freqs), n), np.nan, dtype=torch.float64, device="cuda"))
        P1, TL1 = gbs.forward_noalloc(t, rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate, mode="mix",
                                      out=out)
        torch.cuda.synchronize()
        assert P1.data_ptr() == out[0].data_ptr()
        assert torch.equal(torch.view_as_real(P1), torch.view_as_real(P0)) and torch.equal(TL1, TL0)
        P_ref, TL_ref, ab = reference(sc, rcv=rcv)
        assert_within(compare(P1.cpu().numpy(), TL1.cpu().numpy(), P_ref, TL_ref, ab), "mix")


def test_noalloc_rejects_host_tables_and_oversized_calls():
    sc = open_plane(n_rays=800, grid=8, half=100.0)
    host = gbs.Table(sc.table, on_host=True)
    with pytest.raises(_lib.GbsError) as e:
        gbs.forward_noalloc(host, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate)
    assert e.value.code == _lib.GBS_E_UNSUPPORTED
    # 4.2 M receivers need 16 B of Morton keys and values and 36 B of padded
    # coordinates and order each (218 MB) before any list: more than the
    # static scratch, refused while the plan is laid out
    big = torch.as_tensor(receiver_grid(2048, 2048, -100.0, 100.0, -100.0, 100.0, 1.5), device="cuda")
    t = gbs.Table(sc.table, device="cuda")
    with pytest.raises(_lib.GbsError) as e:
        gbs.forward_noalloc(t, big, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate)
    assert e.value.code == _lib.GBS_E_UNSUPPORTED
    assert "static scratch" in str(e.value)
    # the next call on the same scratch is unaffected
    P0, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate)
    P1, _ = gbs.forward_noalloc(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, c=sc.c, gate=sc.gate)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(P0), torch.view_as_real(P1))
