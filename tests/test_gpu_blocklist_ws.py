"""GPU parity of the device-planned block lists (ta_transform_fwd_ws /
_inv_ws: windows of descriptors planned by a kernel, then the planned
kernels) against the oracle, bit-exact, and against a host plan; descriptors
that are skipped; the per-window fallback for blocks far apart; graph replay;
workspace errors."""

import ctypes

import numpy as np
import pytest

import synth
from tests.batchcase import block_rel_errors, descriptors, oracle_frames, oracle_frames_fp, register_axes

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
    return ctx, ids, ta.load_param_file()


def small_workload():
    # 2 frames of 448 x 200 with a ragged CTU row; all 25 block sizes occur
    return synth.frames_workload(nframes=2, width=448, height=200, seed=30)


def run(ctx, d, frames, inverse=False, sentinel=None):
    x = torch.from_numpy(frames).cuda()
    y = torch.zeros_like(x) if sentinel is None else torch.full_like(x, sentinel)
    dev = ctx.blocks_to_device(d)
    ws = ctx.transform_workspace(len(d))
    (ctx.transform_inv_ws if inverse else ctx.transform_fwd_ws)(dev, x, y, ws)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("order", ["frame", "shuffled", "by_size"])
def test_device_planned_forward_inverse_bit_exact(env, order):
    ctx, _, params = env
    frames, rows = small_workload()
    print(f"{len(rows)} blocks, order {order}", flush=True)
    if order == "shuffled":
        rows = rows[np.random.Generator(np.random.PCG64(5)).permutation(len(rows))]
    elif order == "by_size":
        rows = rows[np.lexsort((rows[:, 6], rows[:, 5], rows[:, 4], rows[:, 3]))]
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    ref = oracle_frames(frames, rows, params)
    got = run(ctx, d, frames)
    mism = np.argwhere(got != ref)
    assert mism.size == 0, f"{len(mism)} mismatches, first {mism[:3].tolist()}"
    refi = oracle_frames(got, rows, params, inverse=True)
    assert (run(ctx, d, got, inverse=True) == refi).all()


def test_device_planned_equals_plan_on_full_range_values(env):
    ctx, _, params = env
    frames, rows = small_workload()
    full = np.random.Generator(np.random.PCG64(3)).integers(-32768, 32768, size=frames.shape).astype(np.int16)
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    plan = ta.Plan(ctx, d)
    x = torch.from_numpy(full).cuda()
    yp, zp = torch.zeros_like(x), torch.zeros_like(x)
    plan.fwd(x, yp)
    plan.inv(x, zp)
    torch.cuda.synchronize()
    assert (run(ctx, d, full) == yp.cpu().numpy()).all()
    assert (run(ctx, d, full, inverse=True) == zp.cpu().numpy()).all()
    assert (yp.cpu().numpy() == oracle_frames(full, rows, params)).all()


def test_skipped_descriptors_leave_output_untouched(env):
    ctx, _, params = env
    frames, rows = small_workload()
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    # every defect below is one the planner checks before any buffer is touched
    planted = {}
    rng = np.random.Generator(np.random.PCG64(9))
    picks = rng.choice(len(d), 6, replace=False)
    defects = ["size", "misaligned", "stride", "axis_range", "unregistered", "negative"]
    for i, kind in zip(picks, defects):
        planted[int(i)] = kind
        if kind == "size":
            d["log2w"][i] = 7
        elif kind == "misaligned":
            d["in_off"][i] += 2
        elif kind == "stride":
            d["in_stride"][i] = (1 << int(d["log2w"][i])) - 4
        elif kind == "axis_range":
            d["axis_v"][i] = 300
        elif kind == "unregistered":
            d["axis_h"][i] = 250
        elif kind == "negative":
            d["out_off"][i] = -8
    got = run(ctx, d, frames, sentinel=12345)
    ref = oracle_frames(frames, rows, params)
    for i in range(len(rows)):
        f, bx, by, w, h = (int(v) for v in rows[i, :5])
        blk = got[f, by:by + h, bx:bx + w]
        if i in planted:
            assert (blk == 12345).all(), f"planted {planted[i]} at {i} was written"
        else:
            assert (blk == ref[f, by:by + h, bx:bx + w]).all(), f"block {i}"


def test_window_spanning_more_than_the_delta_range(env):
    """Two windows' worth of blocks where one block sits 2^30 + 64 input
    elements past the others: its window falls back to one tile per block,
    based at each block's own offsets; the other window plans normally."""
    ctx, _, params = env
    frames, rows = small_workload()
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    n0 = len(d)
    far = (1 << 30) + 64
    frame_elems = frames.shape[1] * frames.shape[2]
    total = far + frame_elems
    print(f"input buffer of {total * 2 / 2**30:.2f} GiB", flush=True)
    x = torch.zeros(total, dtype=torch.int16, device="cuda")
    x[:2 * frame_elems] = torch.from_numpy(frames.reshape(-1)).cuda()
    # block 0 of frame 0 is read from the far copy of frame 0
    x[far:far + frame_elems] = torch.from_numpy(frames[0].reshape(-1)).cuda()
    d2 = d.copy()
    d2["in_off"][0] = far + (d["in_off"][0] - 0)
    assert d["in_off"][0] < frame_elems
    y = torch.full((2 * frame_elems,), 777, dtype=torch.int16, device="cuda")
    dev = ctx.blocks_to_device(d2)
    ws = ctx.transform_workspace(n0)
    ctx.transform_fwd_ws(dev, x, y, ws)
    torch.cuda.synchronize()
    got = y.cpu().numpy().reshape(frames.shape)
    ref = oracle_frames(frames, rows, params)
    assert (got == ref).all()
    del x
    torch.cuda.empty_cache()


def test_graph_replay(env):
    ctx, _, params = env
    frames, rows = small_workload()
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    dev = ctx.blocks_to_device(d)
    ws = ctx.transform_workspace(len(d))
    x = torch.from_numpy(frames).cuda()
    y, z = torch.zeros_like(x), torch.zeros_like(x)
    ctx.transform_fwd_ws(dev, x, y, ws)           # eager first: occupancy query outside the capture
    ref = oracle_frames(frames, rows, params)
    refi = oracle_frames(ref.astype(np.int16), rows, params, inverse=True)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ctx.transform_fwd_ws(dev, x, y, ws, stream_handle=s.cuda_stream)
            ctx.transform_inv_ws(dev, y, z, ws, stream_handle=s.cuda_stream)
    for rep in range(3):
        y.fill_(7)
        z.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert (y.cpu().numpy() == ref).all(), f"replay {rep} forward"
        assert (z.cpu().numpy() == refi).all(), f"replay {rep} inverse"
        y2 = torch.full_like(x, 3)
        ctx.transform_fwd_ws(dev, x, y2, ws)       # eager, same workspace, between replays
        torch.cuda.synchronize()
        assert (y2.cpu().numpy() == ref).all(), f"eager {rep}"


def test_call_errors(env):
    ctx, _, _ = env
    frames, rows = small_workload()
    d = descriptors(rows[:8], frames.shape[1], frames.shape[2])
    dev = ctx.blocks_to_device(d)
    x = torch.from_numpy(frames).cuda()
    y = torch.zeros_like(x)
    L, vp = ta.lib(), ctypes.c_void_p
    need = ctypes.c_int64(0)
    assert L.ta_transform_workspace(8, ctypes.byref(need)) == ta.TA_OK and need.value > 0
    ws = torch.empty(need.value + 512, dtype=torch.uint8, device="cuda")
    args = (ctx._h, vp(dev.data_ptr()), 8, vp(x.data_ptr()), vp(y.data_ptr()), ta.I16)
    s = vp(torch.cuda.current_stream().cuda_stream)
    assert L.ta_transform_fwd_ws(*args, None, need.value, s) == ta.TA_EINVAL
    assert L.ta_transform_fwd_ws(*args, vp(ws.data_ptr() + 64), need.value, s) == ta.TA_EINVAL   # misaligned
    assert L.ta_transform_fwd_ws(*args, vp(ws.data_ptr()), need.value - 1, s) == ta.TA_EINVAL    # short
    assert L.ta_transform_fwd_ws(ctx._h, vp(dev.data_ptr()), 8, vp(x.data_ptr()), vp(x.data_ptr()), ta.I16,
                                 vp(ws.data_ptr()), need.value, s) == ta.TA_EINVAL                # aliasing
    assert L.ta_transform_fwd_ws(*args, vp(ws.data_ptr()), need.value, s) == ta.TA_OK
    torch.cuda.synchronize()


def test_full_workload_equals_plan_and_oracle(env):
    """8 frames of 3840 x 2160 in frame order (143 windows, the last ragged):
    bitwise equal to the host plan, sampled blocks against the oracle."""
    ctx, _, params = env
    frames, rows = synth.frames_workload()
    print(f"full workload device-planned: {len(rows)} blocks", flush=True)
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    dev = ctx.blocks_to_device(d)
    ws = ctx.transform_workspace(len(d))
    x = torch.from_numpy(frames).cuda()
    y, z = torch.zeros_like(x), torch.zeros_like(x)
    ctx.transform_fwd_ws(dev, x, y, ws)
    ctx.transform_inv_ws(dev, y, z, ws)
    plan = ta.Plan(ctx, d)
    yp, zp = torch.zeros_like(x), torch.zeros_like(x)
    plan.fwd(x, yp)
    plan.inv(yp, zp)
    torch.cuda.synchronize()
    assert torch.equal(y, yp) and torch.equal(z, zp)
    sel = np.random.Generator(np.random.PCG64(13)).choice(len(rows), 200, replace=False)
    ref = oracle_frames(frames, rows, params, select=sel)
    yc = y.cpu().numpy()
    for i in sel:
        f, bx, by, w, h = (int(v) for v in rows[i, :5])
        assert (yc[f, by:by + h, bx:bx + w] == ref[f, by:by + h, bx:bx + w]).all(), f"block {i}"


@pytest.mark.parametrize("workload", ["small", "full"])
def test_fp32_device_planned_equals_plan_and_oracle(env, workload):
    """fp32 lists: the device-planned tiles run batch_f32 like a host plan's,
    so the outputs are bitwise equal to the plan's; the small case is also
    checked against the FP64 oracle (per block, 1e-5 of the block's largest
    reference value)."""
    ctx, _, params = env
    frames, rows = small_workload() if workload == "small" else synth.frames_workload()
    print(f"fp32 device-planned, {len(rows)} blocks", flush=True)
    d = descriptors(rows, frames.shape[1], frames.shape[2])
    dev = ctx.blocks_to_device(d)
    ws = ctx.transform_workspace(len(d))
    x = torch.from_numpy(frames.astype(np.float32)).cuda()
    y, z = torch.zeros_like(x), torch.zeros_like(x)
    ctx.transform_fwd_ws(dev, x, y, ws)
    ctx.transform_inv_ws(dev, y, z, ws)
    plan = ta.Plan(ctx, d, dtype=ta.F32)
    yp, zp = torch.zeros_like(x), torch.zeros_like(x)
    plan.fwd(x, yp)
    plan.inv(yp, zp)
    torch.cuda.synchronize()
    assert torch.equal(y, yp) and torch.equal(z, zp)
    if workload == "small":
        yc = y.cpu().numpy()
        err = block_rel_errors(yc, oracle_frames_fp(frames.astype(np.float32), rows, params), rows)
        assert err.max() <= 1e-5, f"forward: worst block {err.argmax()} rel err {err.max():.3e}"
        err = block_rel_errors(z.cpu().numpy(), oracle_frames_fp(yc, rows, params, inverse=True), rows)
        assert err.max() <= 1e-5, f"inverse: worst block {err.argmax()} rel err {err.max():.3e}"
