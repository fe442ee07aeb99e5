"""GPU parity of the batched adjustment design search (ta_design_search,
section 2 / Fig. 1) against the oracle: objective, gradient and adjustment
at given angles to FP64 rounding, and whole Adam runs."""

import numpy as np
import pytest

import synth
from oracle import design as Dz
from oracle import transforms as T

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402
from paper_2505_23618_amd import design as PD  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ta.Context(0)


def _run(ctx, n, restarts, steps, lr, lam, seed, scale=0.8):
    mats, cands, labels = PD.study(n, restarts)
    starts = synth.design_starts(len(cands), PD.n_angles(n), seed, scale)
    th = torch.from_numpy(starts.copy()).cuda()
    out = ctx.design_search(torch.from_numpy(mats).cuda(), torch.from_numpy(cands).cuda(), th, steps, lr, lam,
                            want_grad=True, want_adj=True)
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["theta"] = th.cpu().numpy()
    return mats, cands, labels, starts, res


def _oracle_case(labels, i, n):
    bk, tk, mode = labels[i]
    b, d = T.matrix(bk, n), T.matrix(tk, n)
    return b, d, mode, Dz.sigma_for(b, d, mode)


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_evaluation_parity(ctx, n):
    """steps = 0: objective terms, gradient and M at random angles."""
    print(f"case design eval n={n}", flush=True)
    mats, cands, labels, starts, res = _run(ctx, n, 1, 0, 0.01, 1.0, seed=n)
    rng = np.random.default_rng(n)
    for i in rng.choice(len(cands), 12, replace=False):
        b, d, mode, sg = _oracle_case(labels, i, n)
        f, sp, err = Dz.objective(starts[i], b, d, mode, sg)
        assert res["obj"][i] == pytest.approx([f, sp, err], rel=1e-12, abs=1e-12)
        g = Dz.gradient(starts[i], b, d, mode, sg)
        assert np.abs(res["grad"][i] - g).max() < 1e-11 * max(1.0, np.abs(g).max())
        assert np.abs(res["adj"][i] - Dz.adjustment(starts[i], n, sg)).max() < 1e-13
        assert (res["theta"][i] == starts[i]).all()


@pytest.mark.parametrize("n", [4, 8, 16])
def test_adam_run_parity(ctx, n):
    print(f"case design adam n={n}", flush=True)
    steps, lr = 25, 0.01
    mats, cands, labels, starts, res = _run(ctx, n, 1, steps, lr, 1.0, seed=100 + n)
    rng = np.random.default_rng(200 + n)
    for i in rng.choice(len(cands), 4, replace=False):
        b, d, mode, sg = _oracle_case(labels, i, n)
        th = Dz.adam(starts[i], b, d, mode, sg, 1.0, lr, steps)
        assert np.abs(res["theta"][i] - th).max() < 1e-9
        assert res["obj"][i][0] == pytest.approx(Dz.objective(th, b, d, mode, sg)[0], rel=1e-9)


def test_eq2_optimum_reached_on_gpu(ctx):
    """lam = 0: the search reaches the exact adjustment B^T D (pre) / D B^T
    (post), as the oracle's Adam does with the same settings."""
    n = 4
    mats, cands, labels, starts, res = _run(ctx, n, 1, 3000, 0.02, 0.0, seed=5, scale=0.0)
    for i, lab in enumerate(labels):
        if lab[:2] != ("S3", "S7"):
            continue
        b, d, mode, sg = _oracle_case(labels, i, n)
        assert res["obj"][i][2] < 1e-6, lab
        assert np.abs(res["adj"][i] - Dz.target(b, d, mode)).max() < 2e-3


def test_bad_candidates_and_repeatability(ctx):
    n = 8
    mats, cands, labels = PD.study(n, 1)
    cands = cands[:6].copy()
    cands[1, 0] = 99          # base index out of range
    cands[3, 2] = 2           # bad mode
    cands[4, 3] = 0           # bad sign
    starts = synth.design_starts(len(cands), PD.n_angles(n), 9)
    outs = []
    for _ in range(2):
        th = torch.from_numpy(starts.copy()).cuda()
        o = ctx.design_search(torch.from_numpy(mats).cuda(), torch.from_numpy(cands).cuda(), th, 10, 0.01)
        outs.append((o["obj"].cpu().numpy(), th.cpu().numpy()))
    obj = outs[0][0]
    assert np.isnan(obj[[1, 3, 4]]).all() and np.isfinite(obj[[0, 2, 5]]).all()
    assert np.array_equal(outs[0][0][[0, 2, 5]], outs[1][0][[0, 2, 5]])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_errors(ctx):
    m = torch.zeros((2, 6, 6), dtype=torch.float64, device="cuda")
    c = torch.zeros((1, 4), dtype=torch.int32, device="cuda")
    th = torch.zeros((1, 15), dtype=torch.float64, device="cuda")
    with pytest.raises(ta.TadjError) as e:
        ctx.design_search(m, c, th, 1, 0.01)
    assert e.value.code == ta.TA_EUNSUPPORTED
    m = torch.zeros((2, 8, 8), dtype=torch.float64, device="cuda")
    th = torch.zeros((1, 28), dtype=torch.float64, device="cuda")
    with pytest.raises(ta.TadjError) as e:
        ctx.design_search(m, c, th, 1, -0.01)
    assert e.value.code == ta.TA_EINVAL
