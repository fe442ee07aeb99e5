"""GPU parity of the general transforms against the oracle: every axis kind
(tests/kinds.py: all six bases, bands with K = 2, 4, 6, 8, sub-blocks with
B = 2, 4, 6, 8, 16 and N / 2, with and without the DCT-8 flip) at every size
4..64 on both axes, in packed batches without a specialised kernel, in
planned block lists and in unplanned block lists.  Fixed point must be
bit-exact; fp32 within 1e-5 of the FP64 oracle per block (max |Y - Y_ref| <=
1e-5 max |Y_ref|)."""

import numpy as np
import pytest

import synth
from oracle import fixed as F
from oracle import fp as P
from tests.kinds import KINDS, SIZES, Catalogue, kinds_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402

TOL = 1e-5


@pytest.fixture(scope="module")
def cat():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ta.Context(0)
    ids = ta.load_params(ctx)
    c = Catalogue(ctx, ids, ta.load_param_file())
    ctx.set_impl(2)     # VALU kernels: packed pairs without a specialised kernel go to the general kernel
    return c


def _pairs(w, h):
    """Kind pairs (horizontal, vertical) for a W x H block: every kind that
    exists at W on the rows, each paired with a kind that exists at H."""
    kh, kv = kinds_for(w), kinds_for(h)
    return [(kh[i], kv[(3 * i + 1) % len(kv)]) for i in range(len(kh))]


def _rel_err(got, ref):
    e = np.abs(got - ref).reshape(len(ref), -1).max(axis=1)
    s = np.abs(ref).reshape(len(ref), -1).max(axis=1)
    return np.where(e == 0, 0.0, e / np.where(s > 0, s, 1e-300))


@pytest.mark.parametrize("h", SIZES)
@pytest.mark.parametrize("w", SIZES)
def test_packed_every_kind_bit_exact(cat, w, h):
    """Packed batches of every kind pair at W x H (ragged: 2 tiles + 3
    blocks), AR(1) residuals and full-range int16, forward and inverse."""
    ctx = cat.ctx
    nb = 2 * (256 // max(w, h)) + 3
    print(f"packed general {w}x{h} nb={nb}", flush=True)
    sets = [synth.ar1_blocks(nb, h, w, 0.95, 16.0, seed=300 + w + h),
            synth.adversarial_blocks(h, w, "full16", seed=9, n=nb)]
    for ih, iv in _pairs(w, h):
        ah, av = cat.axis[(ih, w)], cat.axis[(iv, h)]
        oh, ov = cat.oracle[(ih, w)], cat.oracle[(iv, h)]
        for x in sets:
            y = ctx.fwd(torch.from_numpy(x).cuda(), ah, av).cpu().numpy()
            yr = F.fwd2d(x, oh, ov)
            assert (y == yr).all(), f"forward {KINDS[ih][0]} x {KINDS[iv][0]}"
            z = ctx.inv(torch.from_numpy(x).cuda(), ah, av).cpu().numpy()
            assert (z == F.inv2d(x, oh, ov)).all(), f"inverse {KINDS[ih][0]} x {KINDS[iv][0]}"


@pytest.mark.parametrize("h", SIZES)
@pytest.mark.parametrize("w", SIZES)
def test_packed_every_kind_f32(cat, w, h):
    ctx = cat.ctx
    nb = 2 * (256 // max(w, h)) + 3
    x = synth.ar1_blocks(nb, h, w, 0.95, 16.0, seed=400 + w + h).astype(np.float32)
    for ih, iv in _pairs(w, h):
        ah, av = cat.axis[(ih, w)], cat.axis[(iv, h)]
        oh, ov = cat.oracle[(ih, w)], cat.oracle[(iv, h)]
        y = ctx.fwd(torch.from_numpy(x).cuda(), ah, av).cpu().numpy()
        assert _rel_err(y, P.fwd2d(x, oh, ov)).max() <= TOL, f"forward {KINDS[ih][0]} x {KINDS[iv][0]}"
        z = ctx.inv(torch.from_numpy(x).cuda(), ah, av).cpu().numpy()
        assert _rel_err(z, P.inv2d(x, oh, ov)).max() <= TOL, f"inverse {KINDS[ih][0]} x {KINDS[iv][0]}"


# ---------------------------------------------------------------- block lists
def _frames_with_kinds(seed=31):
    """Two 448 x 200 frames (all 25 block sizes), each block's axis kinds
    drawn uniformly from the kinds that exist at its width and height."""
    frames, rows = synth.frames_workload(nframes=2, width=448, height=200, seed=30)
    rng = np.random.Generator(np.random.PCG64(seed))
    kh = np.array([rng.choice(kinds_for(int(w))) for w in rows[:, 3]])
    kv = np.array([rng.choice(kinds_for(int(h))) for h in rows[:, 4]])
    return frames, rows, kh, kv


def _descriptors(cat, rows, kh, kv, fh, fw):
    d = np.zeros(len(rows), ta.BLOCK_DTYPE)
    off = rows[:, 0].astype(np.int64) * fh * fw + rows[:, 2].astype(np.int64) * fw + rows[:, 1]
    d["in_off"] = off
    d["out_off"] = off
    d["in_stride"] = fw
    d["out_stride"] = fw
    d["log2w"] = np.log2(rows[:, 3]).astype(np.uint8)
    d["log2h"] = np.log2(rows[:, 4]).astype(np.uint8)
    d["axis_h"] = [cat.axis[(int(k), int(w))] for k, w in zip(kh, rows[:, 3])]
    d["axis_v"] = [cat.axis[(int(k), int(h))] for k, h in zip(kv, rows[:, 4])]
    return d


def _oracle(cat, frames, rows, kh, kv, inverse, fp):
    out = np.zeros(frames.shape, np.float64 if fp else np.int64)
    groups = {}
    for i, r in enumerate(rows):
        groups.setdefault((int(r[3]), int(r[4]), int(kh[i]), int(kv[i])), []).append(i)
    for (w, h, ih, iv), idx in groups.items():
        stack = np.stack([frames[rows[i, 0], rows[i, 2]:rows[i, 2] + h, rows[i, 1]:rows[i, 1] + w] for i in idx])
        oh, ov = cat.oracle[(ih, w)], cat.oracle[(iv, h)]
        mod = P if fp else F
        res = (mod.inv2d if inverse else mod.fwd2d)(stack, oh, ov)
        for j, i in enumerate(idx):
            out[rows[i, 0], rows[i, 2]:rows[i, 2] + h, rows[i, 1]:rows[i, 1] + w] = res[j]
    return out


def _run(cat, d, x, path, inverse, dtype):
    xd = torch.from_numpy(x).cuda()
    y = torch.zeros_like(xd)
    if path == "planned":
        plan = ta.Plan(cat.ctx, d, dtype=dtype)
        (plan.inv if inverse else plan.fwd)(xd, y)
    else:
        dev = cat.ctx.blocks_to_device(d)
        (cat.ctx.transform_inv if inverse else cat.ctx.transform_fwd)(dev, xd, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("path", ["planned", "unplanned"])
def test_block_list_every_kind_bit_exact(cat, path):
    frames, rows, kh, kv = _frames_with_kinds()
    d = _descriptors(cat, rows, kh, kv, frames.shape[1], frames.shape[2])
    print(f"{path}: {len(rows)} blocks, {len(set(zip(kh, kv)))} kind pairs", flush=True)
    full = np.random.Generator(np.random.PCG64(4)).integers(-32768, 32768, size=frames.shape).astype(np.int16)
    for x in (frames, full):
        for inverse in (False, True):
            got = _run(cat, d, x, path, inverse, ta.I16)
            ref = _oracle(cat, x, rows, kh, kv, inverse, fp=False)
            mism = np.argwhere(got != ref)
            assert mism.size == 0, f"inverse={inverse}: {len(mism)} mismatches, first {mism[:3].tolist()}"


@pytest.mark.parametrize("path", ["planned", "unplanned"])
def test_block_list_every_kind_f32(cat, path):
    frames, rows, kh, kv = _frames_with_kinds(seed=32)
    d = _descriptors(cat, rows, kh, kv, frames.shape[1], frames.shape[2])
    x = frames.astype(np.float32)
    for inverse in (False, True):
        got = _run(cat, d, x, path, inverse, ta.F32)
        ref = _oracle(cat, x, rows, kh, kv, inverse, fp=True)
        worst = 0.0
        for r in rows:
            f, bx, by, w, h = (int(v) for v in r[:5])
            g, e = got[f, by:by + h, bx:bx + w], ref[f, by:by + h, bx:bx + w]
            err, sc = np.abs(g - e).max(), np.abs(e).max()
            worst = max(worst, 0.0 if err == 0 else err / sc if sc > 0 else np.inf)
        assert worst <= TOL, f"inverse={inverse}: worst block {worst:.3g}"


def test_planned_equals_unplanned_general(cat):
    frames, rows, kh, kv = _frames_with_kinds(seed=33)
    d = _descriptors(cat, rows, kh, kv, frames.shape[1], frames.shape[2])
    for inverse in (False, True):
        assert (_run(cat, d, frames, "planned", inverse, ta.I16) ==
                _run(cat, d, frames, "unplanned", inverse, ta.I16)).all()
