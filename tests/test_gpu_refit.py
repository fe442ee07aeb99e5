"""GPU parity of the differentiable Givens-band path (fp32) against the FP64
oracle: forward, adjoint and angle gradients (analytic and finite
differences), bitwise reproducibility, and a short refit that lowers the
loss.  Tolerances: forward per vector |dy| <= 1e-5 |y|_inf; gradients
|dg|_inf <= 1e-4 |g|_inf."""

import numpy as np
import pytest

import synth
from oracle import refit as R

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402
from paper_2505_23618_amd import refit as RF  # noqa: E402

BASES = {"C2": ta.DCT2, "S3": ta.DST3}


@pytest.fixture(scope="module")
def tctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ta.Context(0)


def _vectors(m, n=32, seed=synth.SEED_BASE + 4):
    return synth.ar1_vectors(m, n, 0.85, 0.99, 1.0, seed=seed)


@pytest.mark.parametrize("base", ["C2", "S3"])
@pytest.mark.parametrize("n,taps", [(32, 4), (32, 6), (16, 4)])
def test_forward_and_backward_match_oracle(tctx, base, n, taps):
    rng = np.random.Generator(np.random.PCG64(21))
    m = 1000 + 37
    x = _vectors(m, n)
    th = rng.uniform(-0.5, 0.5, RF.n_angles(n, taps))
    gy = rng.standard_normal((m, n))
    xd = torch.tensor(x, dtype=torch.float32, device="cuda", requires_grad=True)
    thd = torch.tensor(th, dtype=torch.float32, device="cuda", requires_grad=True)
    y = RF.adjusted(xd, thd, tctx, BASES[base], taps)
    yref = R.forward(th, x, base=base, n=n, layers=taps // 2)
    err = np.abs(y.detach().cpu().numpy() - yref).max(axis=1) / np.abs(yref).max(axis=1)
    assert err.max() <= 1e-5
    y.backward(torch.tensor(gy, dtype=torch.float32, device="cuda"))
    dx, dth = R.backward(th, x, gy, base=base, n=n, layers=taps // 2)
    gx = xd.grad.cpu().numpy()
    assert np.abs(gx - dx).max() <= 1e-4 * np.abs(dx).max()
    gth = thd.grad.cpu().numpy()
    assert np.abs(gth - dth).max() <= 1e-4 * np.abs(dth).max()


def test_refit_loss_gradient_full_workload(tctx):
    """131,072 32-point vectors: the torch loss through the library kernels and
    its angle gradient against the FP64 oracle (analytic and central
    differences)."""
    x = _vectors(131072)
    th = np.random.Generator(np.random.PCG64(8)).uniform(-0.3, 0.3, 31)
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    thd = torch.tensor(th, dtype=torch.float32, device="cuda", requires_grad=True)
    loss, basis, energy = RF.refit_loss(xd, thd, tctx)
    lb, le, lt = R.loss_terms(th, x)
    assert abs(loss.item() - lt) <= 1e-5 * max(1.0, abs(lt))
    loss.backward()
    g = thd.grad.cpu().numpy()
    gref = R.grad(th, x)
    assert np.abs(g - gref).max() <= 1e-4 * np.abs(gref).max()
    # FP64 central differences of the oracle loss on a few angles
    for i in (0, 7, 15, 16, 30):
        e = np.zeros(31)
        e[i] = 1e-6
        fd = (R.loss(th + e, x) - R.loss(th - e, x)) / 2e-6
        assert abs(g[i] - fd) <= 1e-4 * np.abs(gref).max()


def test_backward_bitwise_reproducible(tctx):
    x = torch.tensor(_vectors(50000), dtype=torch.float32, device="cuda")
    th = torch.tensor(np.linspace(-0.2, 0.3, 31), dtype=torch.float32, device="cuda")
    grads = []
    for _ in range(3):
        t = th.clone().requires_grad_(True)
        loss, _, _ = RF.refit_loss(x, t, tctx)
        loss.backward()
        grads.append(t.grad.clone())
    assert torch.equal(grads[0], grads[1]) and torch.equal(grads[1], grads[2])


def test_refit_lowers_the_loss(tctx):
    x = torch.tensor(_vectors(131072), dtype=torch.float32, device="cuda")
    th = torch.zeros(31, dtype=torch.float32, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([th], lr=0.02)
    losses = []
    for _ in range(60):
        opt.zero_grad()
        loss, _, _ = RF.refit_loss(x, th, tctx)
        loss.backward()
        opt.step()
        losses.append(loss.item())
    assert losses[-1] < 0.8 * losses[0]
    # the final angles evaluated by the oracle agree with the GPU loss
    lt = R.loss(th.detach().cpu().numpy().astype(np.float64), x.cpu().numpy().astype(np.float64))
    loss, _, _ = RF.refit_loss(x, th, tctx)
    assert abs(loss.item() - lt) <= 1e-5 * max(1.0, abs(lt))


def test_graphed_step_matches_eager_on_every_replay(tctx):
    """The captured step, replayed with the angles updated in place between
    replays (and eager work in between), gives the eager loss and gradient
    each time, and the oracle's within the fp32 tolerances."""
    xh = _vectors(131072)
    x = torch.tensor(xh, dtype=torch.float32, device="cuda")
    th = torch.tensor(np.linspace(-0.2, 0.25, 31), dtype=torch.float32, device="cuda", requires_grad=True)
    step = RF.GraphedRefitStep(x, th, tctx)
    for rep in range(4):
        with torch.no_grad():
            th.add_(0.01 * (rep + 1))                   # new angles, same tensor
        loss = step.replay().item()
        g = th.grad.clone()
        t = th.detach().clone().requires_grad_(True)      # eager reference at the same angles
        le, _, _ = RF.refit_loss(x, t, tctx)
        le.backward()
        torch.cuda.synchronize()
        assert abs(loss - le.item()) <= 1e-6 * max(1.0, abs(le.item())), f"replay {rep} loss"
        assert torch.allclose(g, t.grad, rtol=1e-6, atol=1e-7 * t.grad.abs().max().item()), f"replay {rep} grad"
        thn = th.detach().cpu().numpy().astype(np.float64)
        gref = R.grad(thn, xh)
        assert np.abs(g.cpu().numpy() - gref).max() <= 1e-4 * np.abs(gref).max(), f"replay {rep} vs oracle"
