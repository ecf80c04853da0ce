"""GPU adjoint: the hand-written adjoint kernel against the oracle's hand
adjoint, finite differences (torch gradcheck through GBSFunction) and the
FP64 / MIX agreement, with the ray geometry held fixed."""
import numpy as np
import pytest
import torch

import oracle
import paper_2501_13382_amd as gbs
from scenes import city_5x5_panels, city_scene, open_plane, perturbed_gamma

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def panel_case():
    sc = city_5x5_panels(n_rays=6000, grid=20)
    sc.freqs = np.array([700.0, 1000.0])
    sc.eps = np.array([[25.0, 30.0]])
    rng = np.random.default_rng(21)
    lam = rng.standard_normal((2, len(sc.rcv))) + 1j * rng.standard_normal((2, len(sc.rcv)))
    ref = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam, c=sc.c, gate=sc.gate)
    return sc, lam, ref


def gpu_backward(sc, lam, mode, **kw):
    t = gbs.Table(sc.table, device="cuda")
    dG, dR, dE = gbs.backward(t, sc.rcv, sc.freqs, sc.eps, sc.gamma, lam, c=sc.c, gate=sc.gate, mode=mode, **kw)
    torch.cuda.synchronize()
    return dG.cpu().numpy(), dR.cpu().numpy(), dE.cpu().numpy().reshape(-1)


def test_f64_adjoint_matches_oracle(panel_case):
    sc, lam, (rG, rR, rE) = panel_case
    print("case adjoint f64 vs oracle", flush=True)
    dG, dR, dE = gpu_backward(sc, lam, "f64")
    assert rel_err(dG, rG) <= 1e-9
    assert rel_err(dR, rR) <= 1e-9
    assert rel_err(dE, rE) <= 1e-9


def test_mix_adjoint_close_to_f64(panel_case):
    sc, lam, (rG, rR, rE) = panel_case
    print("case adjoint mix vs oracle", flush=True)
    dG, dR, dE = gpu_backward(sc, lam, "mix")
    assert rel_err(dG, rG) <= 1e-3
    assert rel_err(dR, rR) <= 1e-3
    assert rel_err(dE, rE) <= 1e-3


def test_chunked_adjoint_matches(panel_case):
    sc, lam, (rG, rR, rE) = panel_case
    dG, dR, dE = gpu_backward(sc, lam, "f64", chunk_segs=4000)
    assert gbs.stats()["n_chunks"] >= 3
    assert rel_err(dG, rG) <= 1e-9 and rel_err(dR, rR) <= 1e-9 and rel_err(dE, rE) <= 1e-9


@pytest.mark.parametrize("mode", ["f64", "mix"])
def test_adjoint_bitwise_repeatable(panel_case, mode):
    """Every adjoint output is bitwise equal over repeated calls (fixed-order
    receiver and beam-parameter sums, exact fixed-point segment and face
    sums), with one pass and with several."""
    sc, lam, (rG, rR, rE) = panel_case
    for chunk in (0, 4000):
        print(f"case adjoint repeat mode={mode} chunk={chunk}", flush=True)
        first = gpu_backward(sc, lam, mode, chunk_segs=chunk)
        for _ in range(2):
            again = gpu_backward(sc, lam, mode, chunk_segs=chunk)
            for x, y in zip(first, again):
                assert np.array_equal(x, y)
        assert rel_err(first[0], rG) <= (1e-9 if mode == "f64" else 1e-3)


def test_gradcheck_through_autograd():
    """torch.autograd.gradcheck of TL with respect to the complex coefficients,
    the receivers and eps (finite differences on the GPU F64 path)."""
    sc = city_scene(n_blocks=2, n_rays=500, grid=3, freqs=(400.0,), max_refl=4, city_seed=5, panels=2,
                    complex_gamma=True)
    t = gbs.Table(sc.table, device="cuda")
    used = np.unique(sc.table.face_ids)
    gamma = torch.tensor(sc.gamma, dtype=torch.complex128, device="cuda", requires_grad=True)
    rcv = torch.tensor(sc.rcv, dtype=torch.float64, device="cuda", requires_grad=True)
    eps = torch.tensor(sc.eps, dtype=torch.float64, device="cuda", requires_grad=True)
    opts = {"mode": "f64", "c": sc.c, "gate": sc.gate}
    freqs = torch.tensor(sc.freqs, dtype=torch.float64, device="cuda")

    def f(g, r, e):
        P, TL = gbs.GBSFunction.apply(g, r, e, t, freqs, opts)
        return TL
    assert len(used) > 3
    assert torch.autograd.gradcheck(f, (gamma, rcv, eps), eps=1e-6, atol=1e-5, rtol=1e-4, nondet_tol=1e-9)


def test_autograd_matches_oracle_adjoint():
    """loss = sum (TL - TL_target)^2: torch's gradient equals the oracle adjoint
    driven by lambda = -(20/ln10) dL/dTL / P."""
    sc = open_plane(n_rays=1500, grid=6, half=80.0, freqs=(500.0,), gamma_ground=0.7 + 0.2j)
    t = gbs.Table(sc.table, device="cuda")
    gamma = torch.tensor(sc.gamma, dtype=torch.complex128, device="cuda", requires_grad=True)
    rcv = torch.tensor(sc.rcv, dtype=torch.float64, device="cuda", requires_grad=True)
    eps = torch.tensor(sc.eps, dtype=torch.float64, device="cuda", requires_grad=True)
    freqs = torch.tensor(sc.freqs, dtype=torch.float64, device="cuda")
    P, TL = gbs.GBSFunction.apply(gamma, rcv, eps, t, freqs, {"mode": "f64"})
    target = TL.detach() + 0.5
    loss = ((TL - target) ** 2).sum()
    loss.backward()
    Pn = P.detach().cpu().numpy().reshape(1, -1)
    gTL = (2 * (TL - target)).detach().cpu().numpy().reshape(1, -1)
    lam = -(20 / np.log(10)) * gTL / Pn
    rG, rR, rE = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam)
    assert rel_err(gamma.grad.cpu().numpy(), rG[:, 0] + 1j * rG[:, 1]) <= 1e-9
    assert rel_err(rcv.grad.cpu().numpy(), rR) <= 1e-9
    assert rel_err(eps.grad.cpu().numpy().reshape(-1), rE) <= 1e-9


@pytest.fixture(scope="module")
def inversion_case():
    """Differentiable 5 x 5 paneled city: 501 faces with their own complex
    coefficients; the target field comes from perturbed coefficients and the
    loss is sum over receivers outside the buildings of (TL - TL_target)^2."""
    sc = city_5x5_panels(n_rays=20000, grid=32)
    target_gamma = perturbed_gamma(sc.gamma, seed=4)
    t = gbs.Table(sc.table, device="cuda")
    freqs = torch.tensor(sc.freqs, dtype=torch.float64, device="cuda")
    _, TLt = gbs.forward(t, sc.rcv, sc.freqs, sc.eps, target_gamma, c=sc.c, gate=sc.gate, mode="f64")
    keep = torch.tensor(~sc.meta["inside"], device="cuda").reshape(1, 1, -1)
    return sc, t, freqs, TLt, keep


def _loss(sc, t, freqs, TLt, keep, gamma, mode):
    rcv = torch.tensor(sc.rcv, dtype=torch.float64, device="cuda")
    eps = torch.tensor(sc.eps, dtype=torch.float64, device="cuda")
    P, TL = gbs.GBSFunction.apply(gamma, rcv, eps, t, freqs, {"mode": mode, "c": sc.c, "gate": sc.gate})
    ok = keep & torch.isfinite(TL) & torch.isfinite(TLt)
    return torch.where(ok, TL - TLt, torch.zeros_like(TL)).pow(2).sum(), P, TL, ok


@pytest.mark.parametrize("mode", ["f64", "mix"])
def test_inversion_gradient_matches_oracle(inversion_case, mode):
    sc, t, freqs, TLt, keep = inversion_case
    print(f"case inversion gradient {mode}", flush=True)
    gamma = torch.tensor(sc.gamma, dtype=torch.complex128, device="cuda", requires_grad=True)
    loss, P, TL, ok = _loss(sc, t, freqs, TLt, keep, gamma, mode)
    loss.backward()
    gTL = torch.where(ok, 2 * (TL - TLt), torch.zeros_like(TL)).detach().cpu().numpy().reshape(1, -1)
    Pn = P.detach().cpu().numpy().reshape(1, -1)
    lam = -(20 / np.log(10)) * gTL / np.where(gTL != 0, Pn, 1.0)
    rG, _, _ = oracle.backward(sc.table, sc.gamma, sc.rcv, sc.freqs, sc.eps, lam, c=sc.c, gate=sc.gate)
    used = np.unique(sc.table.face_ids)
    assert len(used) > 250
    tol = 1e-9 if mode == "f64" else 1e-3
    assert rel_err(gamma.grad.cpu().numpy(), rG[:, 0] + 1j * rG[:, 1]) <= tol


def test_inversion_descends(inversion_case):
    """The negative gradient is a descent direction: a backtracking step along
    it lowers the loss at every iteration of a short inversion."""
    sc, t, freqs, TLt, keep = inversion_case
    gamma = torch.tensor(sc.gamma, dtype=torch.complex128, device="cuda", requires_grad=True)
    losses = []
    for it in range(4):
        gamma.grad = None
        loss, _, _, _ = _loss(sc, t, freqs, TLt, keep, gamma, "mix")
        loss.backward()
        losses.append(float(loss.detach()))
        g = gamma.grad.detach()
        step = 0.05 / float(g.abs().max())
        for _ in range(8):                              # backtracking
            trial = (gamma.detach() - step * g).requires_grad_(True)
            with torch.no_grad():
                lt, _, _, _ = _loss(sc, t, freqs, TLt, keep, trial, "mix")
            if float(lt) < losses[-1]:
                break
            step *= 0.5
        assert float(lt) < losses[-1], (it, losses)
        gamma = trial
    print("case inversion losses", losses, flush=True)
    assert losses[-1] < losses[0]
