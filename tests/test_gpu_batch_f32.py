"""GPU parity of the fp32 batched uneven-block path (planned and unplanned)
against the FP64 oracle: per block, max |Y_gpu - Y_ref| <= 1e-5 max |Y_ref|
(an all-zero reference requires exact zeros)."""

import numpy as np
import pytest

import synth
from tests.batchcase import block_rel_errors, descriptors, oracle_frames_fp, register_axes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402

TOL = 1e-5


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ta.Context(0)
    ids = ta.load_params(ctx)
    register_axes(ctx, ids)
    return ctx, ta.load_param_file()


def small_workload():
    # 2 frames of 448 x 200 with a ragged CTU row; all 25 block sizes occur
    return synth.frames_workload(nframes=2, width=448, height=200, seed=30)


def inputs(frames):
    rng = np.random.Generator(np.random.PCG64(17))
    return [frames.astype(np.float32), rng.standard_normal(frames.shape).astype(np.float32) * 1000.0]


def run_planned(ctx, d, x, inverse):
    plan = ta.Plan(ctx, d, dtype=ta.F32)
    xd = torch.from_numpy(x).cuda()
    y = torch.zeros_like(xd)
    (plan.inv if inverse else plan.fwd)(xd, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def run_unplanned(ctx, d, x, inverse):
    xd = torch.from_numpy(x).cuda()
    y = torch.zeros_like(xd)
    dev = ctx.blocks_to_device(d)
    (ctx.transform_inv if inverse else ctx.transform_fwd)(dev, xd, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("path", ["planned", "unplanned"])
def test_f32_batched_forward_inverse(env, path):
    ctx, params = env
    frames, rows = small_workload()
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    run = run_planned if path == "planned" else run_unplanned
    for k, x in enumerate(inputs(frames)):
        print(f"fp32 batched {path} input {k}: {len(rows)} blocks", flush=True)
        y = run(ctx, d, x, False)
        err = block_rel_errors(y, oracle_frames_fp(x, rows, params), rows)
        assert err.max() <= TOL, f"forward: worst block {err.argmax()} rel err {err.max():.3e}"
        z = run(ctx, d, y, True)
        err = block_rel_errors(z, oracle_frames_fp(y, rows, params, inverse=True), rows)
        assert err.max() <= TOL, f"inverse: worst block {err.argmax()} rel err {err.max():.3e}"


def test_f32_batched_zero_blocks_exact(env):
    ctx, _ = env
    frames, rows = small_workload()
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    x = np.zeros(frames.shape, np.float32)
    for run in (run_planned, run_unplanned):
        for inverse in (False, True):
            assert (run(ctx, d, x, inverse) == 0).all()


def test_f32_plan_autotune_and_graph_replay(env):
    ctx, params = env
    frames, rows = small_workload()
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    plan = ta.Plan(ctx, d, dtype=ta.F32)
    x = torch.from_numpy(frames.astype(np.float32)).cuda()
    y, z = torch.zeros_like(x), torch.zeros_like(x)
    info = plan.autotune(x, y, reps=2)
    assert info["grid"] in (256, 512, 1024, 2048, 4096, 8192)
    assert 18 <= info["region_log2"] <= 22
    dev = ctx.blocks_to_device(d)
    y2 = torch.zeros_like(x)
    ctx.transform_fwd(dev, x, y2)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.fwd(x, y, stream_handle=s.cuda_stream)
            plan.inv(y, z, stream_handle=s.cuda_stream)
            ctx.transform_fwd(dev, x, y2, stream_handle=s.cuda_stream)
    ref = oracle_frames_fp(frames, rows, params)
    for rep in range(3):
        y.fill_(7)
        z.fill_(-7)
        y2.fill_(3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        yc = y.cpu().numpy()
        assert block_rel_errors(yc, ref, rows).max() <= TOL, f"replay {rep} forward"
        assert (y2.cpu().numpy() == yc).all(), f"replay {rep} unplanned"
        refi = oracle_frames_fp(yc, rows, params, inverse=True)
        assert block_rel_errors(z.cpu().numpy(), refi, rows).max() <= TOL, f"replay {rep} inverse"


def test_f32_full_workload_sampled(env):
    """8 frames of 3840 x 2160 in fp32 (530 MB per buffer), planned and
    unplanned; sampled blocks against the oracle, the two paths bitwise equal."""
    ctx, params = env
    frames, rows = synth.frames_workload()
    print(f"fp32 full workload: {len(rows)} blocks", flush=True)
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    plan = ta.Plan(ctx, d, dtype=ta.F32)
    x = torch.from_numpy(frames.astype(np.float32)).cuda()
    y, z = torch.zeros_like(x), torch.zeros_like(x)
    plan.fwd(x, y)
    plan.inv(y, z)
    dev = ctx.blocks_to_device(d)
    y2 = torch.zeros_like(x)
    ctx.transform_fwd(dev, x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)
    del y2
    sel = np.random.Generator(np.random.PCG64(13)).choice(len(rows), 300, replace=False)
    yc = y.cpu().numpy()
    err = block_rel_errors(yc, oracle_frames_fp(frames, rows, params, select=sel), rows, sel)
    assert err.max() <= TOL, f"forward worst {err.max():.3e}"
    err = block_rel_errors(z.cpu().numpy(), oracle_frames_fp(yc, rows, params, inverse=True, select=sel), rows, sel)
    assert err.max() <= TOL, f"inverse worst {err.max():.3e}"
