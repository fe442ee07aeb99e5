"""GPU parity at integer-matrix precisions m other than 8 (the context's m
sets the integer base tables and the core shifts; the specialised kernels
hold the m = 8 tables, so these contexts run every fixed-point transform on
the general kernel): packed batches, planned and unplanned block lists,
bit-exact against the oracle at the same m, AR(1) and full-range inputs."""

import numpy as np
import pytest

import synth
from oracle import fixed as F
from tests.kinds import KINDS, SIZES, Catalogue, kinds_for
from tests.test_gpu_general import _descriptors, _frames_with_kinds

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402

BD = 8


@pytest.fixture(scope="module", params=[6, 7, 9])
def cat(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ta.Context(0, bit_depth=BD, m=request.param)
    ids = ta.load_params(ctx)
    return Catalogue(ctx, ids, ta.load_param_file())


@pytest.mark.parametrize("h", SIZES)
@pytest.mark.parametrize("w", SIZES)
def test_packed_bit_exact_at_m(cat, w, h):
    m = cat.ctx.m
    nb = 256 // max(w, h) + 3
    print(f"precision m={m} packed {w}x{h}", flush=True)
    sets = [synth.ar1_blocks(nb, h, w, 0.95, 16.0, seed=500 + w + h),
            synth.adversarial_blocks(h, w, "full16", seed=10, n=nb)]
    kh, kv = kinds_for(w), kinds_for(h)
    for i in range(0, len(kh), 3):          # every third kind on the rows, paired along
        ih, iv = kh[i], kv[(5 * i + 2) % len(kv)]
        ah, av = cat.axis[(ih, w)], cat.axis[(iv, h)]
        oh, ov = cat.oracle[(ih, w)], cat.oracle[(iv, h)]
        for x in sets:
            y = cat.ctx.fwd(torch.from_numpy(x).cuda(), ah, av).cpu().numpy()
            assert (y == F.fwd2d(x, oh, ov, bd=BD, m=m)).all(), f"forward {KINDS[ih][0]} x {KINDS[iv][0]}"
            z = cat.ctx.inv(torch.from_numpy(x).cuda(), ah, av).cpu().numpy()
            assert (z == F.inv2d(x, oh, ov, bd=BD, m=m)).all(), f"inverse {KINDS[ih][0]} x {KINDS[iv][0]}"


@pytest.mark.parametrize("path", ["planned", "unplanned"])
def test_block_list_bit_exact_at_m(cat, path):
    m = cat.ctx.m
    frames, rows, kh, kv = _frames_with_kinds(seed=40 + m)
    d = _descriptors(cat, rows, kh, kv, frames.shape[1], frames.shape[2])
    for inverse in (False, True):
        xd = torch.from_numpy(frames).cuda()
        y = torch.zeros_like(xd)
        if path == "planned":
            plan = ta.Plan(cat.ctx, d)
            (plan.inv if inverse else plan.fwd)(xd, y)
        else:
            dev = cat.ctx.blocks_to_device(d)
            (cat.ctx.transform_inv if inverse else cat.ctx.transform_fwd)(dev, xd, y)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        groups = {}
        for i, r in enumerate(rows):
            groups.setdefault((int(r[3]), int(r[4]), int(kh[i]), int(kv[i])), []).append(i)
        for (w, h, ih, iv), idx in groups.items():
            stack = np.stack([frames[rows[i, 0], rows[i, 2]:rows[i, 2] + h, rows[i, 1]:rows[i, 1] + w] for i in idx])
            oh, ov = cat.oracle[(ih, w)], cat.oracle[(iv, h)]
            ref = (F.inv2d if inverse else F.fwd2d)(stack, oh, ov, bd=BD, m=m)
            for j, i in enumerate(idx):
                f, bx, by = int(rows[i, 0]), int(rows[i, 1]), int(rows[i, 2])
                assert (got[f, by:by + h, bx:bx + w] == ref[j]).all(), f"block {i} inverse={inverse}"


def test_matrix_cores_and_multi_need_m8(cat):
    ctx = cat.ctx
    x = torch.zeros((4, 32, 32), dtype=torch.int16, device="cuda")
    a = cat.axis[(0, 32)]
    ctx.set_impl(1)
    try:
        with pytest.raises(ta.TadjError) as e:
            ctx.fwd(x, a, a)
        assert e.value.code == ta.TA_EUNSUPPORTED
    finally:
        ctx.set_impl(0)
    ids = ta.load_params(ctx)
    with pytest.raises(ta.TadjError) as e:
        ctx.fwd_multi(x, ids["post_C2_S7_N32_B8"])
    assert e.value.code == ta.TA_EUNSUPPORTED
