"""GPU parity of the batched uneven-block path (one persistent launch per
direction) against the oracle, bit-exact, plus autotuning and graph replay."""

import numpy as np
import pytest

import synth
from tests.batchcase import descriptors, oracle_frames, register_axes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ta.Context(0)
    ids = ta.load_params(ctx)
    register_axes(ctx, ids)
    return ctx, ta.load_param_file()


def small_workload():
    # 2 frames of 448 x 200 (200 = 3*64 + 8: a ragged CTU row); this seed's
    # partition contains all 25 block sizes 4..64 x 4..64
    return synth.frames_workload(nframes=2, width=448, height=200, seed=30)


def test_batched_forward_inverse_bit_exact(env):
    ctx, params = env
    frames, rows = small_workload()
    sizes = {(int(w), int(h)) for w, h in rows[:, 3:5]}
    print(f"{len(rows)} blocks, {len(sizes)} size classes", flush=True)
    assert len(sizes) == 25
    plan = ta.Plan(ctx, descriptors(rows, frames.shape[1], frames.shape[2]))
    x = torch.from_numpy(frames).cuda()
    y = torch.zeros_like(x)
    plan.fwd(x, y)
    ref = oracle_frames(frames, rows, params)
    got = y.cpu().numpy()
    mism = np.argwhere(got != ref)
    assert mism.size == 0, f"{len(mism)} mismatches, first {mism[:3].tolist()}"
    z = torch.zeros_like(x)
    plan.inv(y, z)
    refi = oracle_frames(got, rows, params, inverse=True)
    assert (z.cpu().numpy() == refi).all()


def test_batched_adversarial_values(env):
    ctx, params = env
    frames, rows = small_workload()
    rng = np.random.Generator(np.random.PCG64(3))
    full = rng.integers(-32768, 32768, size=frames.shape).astype(np.int16)
    plan = ta.Plan(ctx, descriptors(rows, frames.shape[1], frames.shape[2]))
    x = torch.from_numpy(full).cuda()
    y = torch.zeros_like(x)
    plan.fwd(x, y)
    assert (y.cpu().numpy() == oracle_frames(full, rows, params)).all()
    z = torch.zeros_like(x)
    plan.inv(x, z)
    assert (z.cpu().numpy() == oracle_frames(full, rows, params, inverse=True)).all()


def test_autotune_and_graph_replay(env):
    ctx, params = env
    frames, rows = small_workload()
    plan = ta.Plan(ctx, descriptors(rows, frames.shape[1], frames.shape[2]))
    x = torch.from_numpy(frames).cuda()
    y = torch.zeros_like(x)
    info = plan.autotune(x, y, reps=2)
    assert info["grid"] in (256, 512, 1024, 2048, 4096, 8192)
    assert 18 <= info["region_log2"] <= 22
    ref = oracle_frames(frames, rows, params)
    # capture forward + inverse in a graph; replay with eager work in between
    z = torch.zeros_like(x)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.fwd(x, y, stream_handle=s.cuda_stream)
            plan.inv(y, z, stream_handle=s.cuda_stream)
    refi = oracle_frames(ref.astype(np.int16), rows, params, inverse=True)
    for rep in range(3):
        y.fill_(7)
        z.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert (y.cpu().numpy() == ref).all(), f"replay {rep} forward"
        assert (z.cpu().numpy() == refi).all(), f"replay {rep} inverse"


def test_plan_errors(env):
    ctx, _ = env
    frames, rows = small_workload()
    d = descriptors(rows[:10], frames.shape[1], frames.shape[2])
    bad = d.copy()
    bad["in_off"][3] += 2          # misaligned
    with pytest.raises(ta.TadjError) as e:
        ta.Plan(ctx, bad)
    assert e.value.code == ta.TA_EUNSUPPORTED
    bad = d.copy()
    bad["axis_h"][0] = 250         # unregistered axis
    with pytest.raises(ta.TadjError) as e:
        ta.Plan(ctx, bad)
    assert e.value.code == ta.TA_ENOPARAMS
    empty = ta.Plan(ctx, d[:0])
    assert empty.info()["tiles"] == 0


def test_full_workload_sampled(env):
    """8 frames of 3840 x 2160: the full batched workload, sampled blocks."""
    ctx, params = env
    frames, rows = synth.frames_workload()
    print(f"full batched workload: {len(rows)} blocks", flush=True)
    plan = ta.Plan(ctx, descriptors(rows, frames.shape[1], frames.shape[2]))
    x = torch.from_numpy(frames).cuda()
    y = torch.zeros_like(x)
    z = torch.zeros_like(x)
    plan.fwd(x, y)
    plan.inv(y, z)
    torch.cuda.synchronize()
    sel = np.random.Generator(np.random.PCG64(11)).choice(len(rows), 300, replace=False)
    ref = oracle_frames(frames, rows, params, select=sel)
    yc = y.cpu().numpy()
    refi = oracle_frames(yc, rows, params, inverse=True, select=sel)
    zc = z.cpu().numpy()
    for i in sel:
        f, bx, by, w, h = (int(v) for v in rows[i, :5])
        assert (yc[f, by:by + h, bx:bx + w] == ref[f, by:by + h, bx:bx + w]).all(), f"block {i}"
        assert (zc[f, by:by + h, bx:bx + w] == refi[f, by:by + h, bx:bx + w]).all(), f"block {i} inverse"


def test_set_tuning_keeps_outputs_bitwise(env):
    ctx, params = env
    frames, rows = small_workload()
    plan = ta.Plan(ctx, descriptors(rows, frames.shape[1], frames.shape[2]))
    x = torch.from_numpy(frames).cuda()
    y0, z0 = torch.zeros_like(x), torch.zeros_like(x)
    plan.fwd(x, y0)
    plan.inv(y0, z0)
    for grid, region in ((8, 12), (256, 18), (1024, 20), (8192, 22), (4096, 30)):
        info = plan.set_tuning(grid, region)
        assert info["grid"] == grid and info["region_log2"] == region
        y, z = torch.full_like(x, 5), torch.full_like(x, -5)
        plan.fwd(x, y)
        plan.inv(y0, z)
        torch.cuda.synchronize()
        assert torch.equal(y, y0) and torch.equal(z, z0), f"grid {grid} region {region}"
    assert (y0.cpu().numpy() == oracle_frames(frames, rows, params)).all()
    for grid, region in ((4, 20), (1024, 11), (1024, 41)):
        with pytest.raises(ta.TadjError) as e:
            plan.set_tuning(grid, region)
        assert e.value.code == ta.TA_EINVAL
