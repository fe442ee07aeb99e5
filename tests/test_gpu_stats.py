"""GPU parity of the quantised-coefficient statistics (ta_coef_stats), the
coding-gain proxy for the coding results (Tables 2 and 3): symbol
histograms, escape bits, energy and distortion sums bit-exact against the
oracle; per-position rates and the summary within 1e-12 (FP64 reductions
in another order)."""

import math

import numpy as np
import pytest

import synth
from oracle import stats as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ta.Context(0)


def _laplace_blocks(nb, h, w, seed, top=3000.0):
    """Coefficient-like data: Laplacian per position, scale falling from `top`
    at position 0 to about 1, so both the near and the far levels occur."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.arange(h * w)
    scale = top * np.exp(-p / max(1.0, h * w / 8.0)) + 1.0
    y = rng.laplace(0.0, scale, size=(nb, h * w))
    return np.clip(np.rint(y), -32768, 32767).astype(np.int16).reshape(nb, h, w)


def _compare(ctx, x, step, offset):
    got = ctx.coef_stats(torch.from_numpy(np.ascontiguousarray(x)).cuda(), step, offset)
    g = {k: v.cpu().numpy() for k, v in got.items()}
    ref = S.coef_stats(x, step, offset)
    bad = np.argwhere(g["hist"].astype(np.int64) != ref["hist"])
    assert bad.size == 0, f"hist mismatches {len(bad)}, first (pos, bin) {bad[:3].tolist()}"
    assert (g["esc_bits"] == ref["esc_bits"]).all()
    assert (g["energy"] == ref["energy"]).all()
    assert (g["dist"] == ref["dist"]).all()
    assert np.allclose(g["rate"], ref["rate"], rtol=0, atol=1e-12)
    for i, name in enumerate(ta.SUMMARY_FIELDS):
        want, have = ref["summary"][name], g["summary"][i]
        if math.isinf(want):
            assert have == want, name
        else:
            assert have == pytest.approx(want, rel=1e-12, abs=1e-12), name
    return g


SHAPES = [(4, 4), (8, 8), (4, 16), (16, 16), (8, 32), (32, 32), (16, 64), (64, 64)]


@pytest.mark.parametrize("h,w", SHAPES)
def test_parity_laplace_ragged(ctx, h, w):
    nb = 2 * max(1, 256 // (h * w)) * 37 + 3           # several steps and a ragged tail
    print(f"case stats laplace {h}x{w} nb={nb}", flush=True)
    x = _laplace_blocks(nb, h, w, seed=h * 100 + w)
    _compare(ctx, x, 24, 12)


@pytest.mark.parametrize("step,offset", [(1, 0), (2, 1), (7, 3), (64, 32), (64, 21), (1000, 999), (32768, 0),
                                         (32768, 32767)])
def test_parity_quantisers(ctx, step, offset):
    print(f"case stats step={step} offset={offset}", flush=True)
    x = _laplace_blocks(301, 4, 8, seed=step)
    _compare(ctx, x, step, offset)


@pytest.mark.parametrize("kind", ["extreme16", "full16", "checker", "zeros"])
def test_parity_adversarial(ctx, kind):
    print(f"case stats adversarial {kind}", flush=True)
    x = synth.adversarial_blocks(8, 8, kind, seed=2, n=45)
    _compare(ctx, x, 3, 1)
    _compare(ctx, x[:, :4, :4].copy(), 1, 0)


def test_all_minimum_values(ctx):
    x = np.full((70, 4, 4), -32768, np.int16)
    g = _compare(ctx, x, 1, 0)
    assert (g["hist"][:, 0] == 70).all() and (g["esc_bits"] == 70 * 29).all()


def test_empty_batch_gives_zeros(ctx):
    x = np.zeros((0, 16, 16), np.int16)
    g = _compare(ctx, x, 16, 8)
    assert (g["summary"] == 0).all() and (g["hist"] == 0).all()


def test_many_blocks_per_workgroup_and_repeatable(ctx):
    """More steps than any one workgroup may count in 16 bits force the
    host to widen the grid; two calls are bitwise identical."""
    x = _laplace_blocks(70000, 4, 4, seed=11, top=40.0)
    g1 = _compare(ctx, x, 4, 2)
    g2 = {k: v.cpu().numpy() for k, v in ctx.coef_stats(torch.from_numpy(x).cuda(), 4, 2).items()}
    for k in g1:
        assert (g1[k] == g2[k]).all(), k


def test_errors(ctx):
    x = torch.zeros((4, 8, 8), dtype=torch.int16, device="cuda")
    with pytest.raises(ta.TadjError) as e:
        ctx.coef_stats(x, 0, 0)
    assert e.value.code == ta.TA_EINVAL
    with pytest.raises(ta.TadjError) as e:
        ctx.coef_stats(x, 8, 8)
    assert e.value.code == ta.TA_EINVAL
    with pytest.raises(ta.TadjError) as e:
        ctx.coef_stats(torch.zeros((4, 2, 8), dtype=torch.int16, device="cuda"), 8, 4)
    assert e.value.code == ta.TA_EUNSUPPORTED


def test_full_workload_sampled_positions(ctx):
    """The benchmark's 262,144-block 32x32 workload through the adjusted
    DST-7 forward, then the statistics in one call; every position's
    histogram sums to the block count, and sampled positions are checked
    against the oracle over all blocks."""
    ids = ta.load_params(ctx)
    ctx.axis(120, ta.DST3, ta.ADJ_BAND, False, ids["band_S3_S7_N32_K4"])
    x = torch.from_numpy(synth.workload_blocks("cfg2_32x32")).cuda()
    y = ctx.fwd(x, 120, 120)
    step, off = 64, 32
    g = {k: v.cpu().numpy() for k, v in ctx.coef_stats(y, step, off).items()}
    nb = y.shape[0]
    assert (g["hist"].sum(axis=1) == nb).all()
    yc = y.reshape(nb, -1).cpu().numpy()
    pos = np.array([0, 1, 32, 33, 100, 511, 777, 1023])
    ref = S.coef_stats(yc[:, pos].reshape(nb, 1, len(pos)), step, off)
    assert (g["hist"][pos].astype(np.int64) == ref["hist"]).all()
    assert (g["esc_bits"][pos] == ref["esc_bits"]).all()
    assert (g["energy"][pos] == ref["energy"]).all() and (g["dist"][pos] == ref["dist"]).all()
    assert np.allclose(g["rate"][pos], ref["rate"], rtol=0, atol=1e-12)
    # summary from the per-position arrays
    ncoef = nb * 1024.0
    assert g["summary"][0] == pytest.approx(g["rate"].mean(), rel=1e-12)
    assert g["summary"][1] == pytest.approx(g["dist"].sum() / ncoef, rel=1e-12)
    assert g["summary"][2] == pytest.approx(g["energy"].sum() / ncoef, rel=1e-12)
    assert g["summary"][3] == pytest.approx(S.coding_gain_db(g["energy"] / nb), abs=1e-9)
    assert g["summary"][5] == pytest.approx(1 - g["hist"][:, 32].sum() / ncoef, rel=1e-12)
    assert g["summary"][6] == pytest.approx((g["hist"][:, 0].sum() + g["hist"][:, 64].sum()) / ncoef, rel=1e-12)


def test_graph_replay_and_buffer_reuse(ctx):
    """The statistics launch sequence captured in a HIP graph replays to the
    eager result (the empty-batch path clears with a kernel, not a memset);
    a result dict is reused across calls of different batch sizes."""
    x = _laplace_blocks(3000, 16, 16, seed=21)
    xd = torch.from_numpy(x).cuda()
    buf = ctx.coef_stats(xd, 24, 12)
    ref = {k: v.clone() for k, v in buf.items() if k != "workspace"}
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ctx.coef_stats(xd, 24, 12, out=buf)
    for rep in range(3):
        for k in ref:
            buf[k].fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(buf[k], ref[k]), f"replay {rep}: {k}"
    # reuse with a smaller and then a larger batch of the same block shape
    for nb in (17, 4000):
        xs = _laplace_blocks(nb, 16, 16, seed=nb)
        got = ctx.coef_stats(torch.from_numpy(xs).cuda(), 24, 12, out=buf)
        want = S.coef_stats(xs, 24, 12)
        assert (got["hist"].cpu().numpy().astype(np.int64) == want["hist"]).all()
        assert (got["energy"].cpu().numpy() == want["energy"]).all()
