"""Graph capture of a batched forward (all sources x bands in one persistent
launch per pass) and its replay: every replay matches the FP64 oracle (and
equals the eager call bit for bit), also after the reflection coefficients
are changed between replays, over several passes of the table, and with the
table streamed from pinned host memory by the replay itself."""
import numpy as np
import pytest
import torch

import paper_2501_13382_amd as gbs
from scenes import city_batched, perturbed_gamma
from tests.gpu_util import assert_within, compare, reference

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batched():
    sc = city_batched(n_src=3, ray_lo=1500, ray_hi=5000, grid=24)
    g2 = perturbed_gamma(sc.gamma, seed=4)
    return sc, g2, reference(sc), reference(sc, gamma=g2)


def _check(P, TL, ref, mode):
    P_ref, TL_ref, ab = ref
    assert_within(compare(P.cpu().numpy(), TL.cpu().numpy(), P_ref, TL_ref, ab), mode)


@pytest.mark.parametrize("mode", ["mix", "f64"])
def test_graph_replays_match_oracle_and_eager(batched, mode):
    sc, g2, ref, ref2 = batched
    t = gbs.Table(sc.table, device="cuda")
    kw = dict(c=sc.c, gate=sc.gate, mode=mode)
    P_eager, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, **kw)
    P_eager = P_eager.cpu().numpy()
    g = gbs.Graph(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, **kw)
    for rep in range(3):
        print(f"case graph replay mode={mode} {rep}", flush=True)
        P, TL = g.launch()
        torch.cuda.synchronize()
        _check(P, TL, ref, mode)
        assert np.array_equal(P.cpu().numpy(), P_eager)
        # eager work between replays
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
    g.set_gamma(g2)
    P2_eager, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, g2, **kw)
    for rep in range(2):
        print(f"case graph replay after set_gamma mode={mode} {rep}", flush=True)
        P, TL = g.launch()
        torch.cuda.synchronize()
        _check(P, TL, ref2, mode)
        assert np.array_equal(P.cpu().numpy(), P2_eager.cpu().numpy())


@pytest.mark.parametrize("on_host", [False, True])
def test_graph_over_several_passes(batched, on_host):
    """A table split into passes (device-resident, or streamed from pinned host
    memory by the replay itself): replays match the oracle, before and after a
    coefficient change, and equal the eager call bit for bit."""
    sc, g2, ref, ref2 = batched
    t = gbs.Table(sc.table, device="cuda", on_host=on_host)
    chunk = sc.table.seg_s0.shape[0] // 4 + 1
    kw = dict(c=sc.c, gate=sc.gate, mode="mix", chunk_segs=chunk)
    P_eager, _ = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, **kw)
    assert gbs.stats()["n_chunks"] >= 4
    P_eager = P_eager.cpu().numpy()
    g = gbs.Graph(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, **kw)
    for rep in range(3):
        print(f"case graph passes on_host={on_host} replay {rep}", flush=True)
        P, TL = g.launch()
        torch.cuda.synchronize()
        _check(P, TL, ref, "mix")
        assert np.array_equal(P.cpu().numpy(), P_eager)
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
    g.set_gamma(g2)
    for rep in range(2):
        P, TL = g.launch()
        torch.cuda.synchronize()
        _check(P, TL, ref2, "mix")
