"""GPU parity of the block-list backward (ta_transform_bwd) and of parameter
sets registered by their angles, against the FP64 oracle
(oracle/blockgrad.py): dL/dX per block within 1e-5 of max |dL/dX_ref| of
the block, the angle gradient within 1e-4 of max |g_ref|, bitwise
repeatable; the angle set used on rows, columns, both, flipped and not,
beside axes of other kinds that must not contribute."""

import numpy as np
import pytest

from oracle import adjust as OA
from oracle import blockgrad as BG
from oracle import fixed as F
from oracle.fixed import Axis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402

FW, FH = 256, 192          # frame of the test's blocks (elements)
SET_ID = 150


def _set_cases():
    rng = np.random.Generator(np.random.PCG64(70))
    out = []
    for n, taps in ((8, 2), (16, 4), (32, 6), (64, 4)):
        out.append(BG.AngleSet("band", n, rng.uniform(-0.6, 0.6, OA.n_angles(n, taps // 2)), taps=taps))
    for n, b, with_q0 in ((16, 4, False), (32, 8, True), (64, 16, True)):
        q0 = OA.rotation_product(b, rng.uniform(-1.0, 1.0, b * (b - 1) // 2)) if with_q0 else None
        out.append(BG.AngleSet("post", n, rng.uniform(-0.6, 0.6, b * (b - 1) // 2), b=b, q0=q0))
    return out


CASES = _set_cases()


def _ids(c):
    return f"{c.kind}{c.n}_{c.taps or c.b}"


def _register(ctx, aset, params, ids):
    """The angle set on axes 200 (plain) and 201 (flipped), and other axes:
    202 frozen 4-tap band at 16 (not the set), 203 direct DST-7, 204 DCT-2."""
    if aset.kind == "band":
        ctx.set_band_angles(SET_ID, aset.n, aset.taps, aset.angles)
        base = ta.DST3
        ctx.axis(200, base, ta.ADJ_BAND, False, SET_ID)
        ctx.axis(201, base, ta.ADJ_BAND, True, SET_ID)
        use = lambda f: BG.AxisUse("S3", "band", f, True)           # noqa: E731
    else:
        ctx.set_post_angles(SET_ID, aset.n, aset.b, aset.angles, aset.q0)
        base = ta.DCT2
        ctx.axis(200, base, ta.ADJ_POST, False, SET_ID)
        ctx.axis(201, base, ta.ADJ_POST, True, SET_ID)
        use = lambda f: BG.AxisUse("C2", "post", f, True)           # noqa: E731
    e = params["band_S3_S7_N16_K4"]
    ctx.axis(202, ta.DST3, ta.ADJ_BAND, False, ids["band_S3_S7_N16_K4"])
    ctx.axis(203, ta.DST7)
    ctx.axis(204, ta.DCT2)
    lib = {200: use(False), 201: use(True), 202: BG.AxisUse("S3", "band", False, False, a=np.asarray(e["a_f64"])),
           203: BG.AxisUse("S7"), 204: BG.AxisUse("C2")}
    return lib


def _blocks(aset):
    """(x, y, w, h, axis_h, axis_v): the set on rows, columns, both (plain
    and flipped), and blocks that do not use it."""
    n = aset.n
    cand = [(n, n, 200, 200), (n, n, 201, 200), (n, 16, 200, 202), (16, n, 202, 201),
            (n, 8, 201, 204), (8, n, 204, 200), (n, n, 203, 201), (16, 16, 202, 204), (8, 4, 204, 204)]
    out, x, y, rowh = [], 0, 0, 0
    for w, h, ah, av in cand:
        if x + w > FW:
            x, y = 0, y + rowh
            rowh = 0
        assert y + h <= FH
        out.append((x, y, w, h, ah, av))
        x += w
        rowh = max(rowh, h)
    return out


def _descriptors(blocks):
    d = np.zeros(len(blocks), ta.BLOCK_DTYPE)
    for i, (x, y, w, h, ah, av) in enumerate(blocks):
        d[i] = (y * FW + x, y * FW + x, FW, FW, int(np.log2(w)), int(np.log2(h)), ah, av, 0)
    return d


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ta.Context(0)
    ids = ta.load_params(ctx)
    return ctx, ids, ta.load_param_file()


@pytest.mark.parametrize("aset", CASES, ids=[_ids(c) for c in CASES])
def test_backward_matches_oracle(env, aset):
    ctx, ids, params = env
    lib = _register(ctx, aset, params, ids)
    blocks = _blocks(aset)
    print(f"backward {_ids(aset)}: {len(blocks)} blocks", flush=True)
    rng = np.random.Generator(np.random.PCG64(71))
    xf = rng.standard_normal((FH, FW)).astype(np.float32) * 50.0
    gyf = rng.standard_normal((FH, FW)).astype(np.float32)
    dev = ctx.blocks_to_device(_descriptors(blocks))
    x, gy = torch.from_numpy(xf).cuda(), torch.from_numpy(gyf).cuda()
    gx = torch.zeros_like(x)
    gth = torch.empty(len(aset.angles), dtype=torch.float32, device="cuda")
    ctx.transform_bwd(dev, x, gy, gx, gth, SET_ID)
    gx2, gth2 = torch.zeros_like(x), torch.empty_like(gth)
    ctx.transform_bwd(dev, x, gy, gx2, gth2, SET_ID)
    torch.cuda.synchronize()
    assert torch.equal(gx, gx2) and torch.equal(gth, gth2), "not bitwise repeatable"
    xb = [xf[y:y + h, bx:bx + w].astype(np.float64) for bx, y, w, h, _, _ in blocks]
    gb = [gyf[y:y + h, bx:bx + w].astype(np.float64) for bx, y, w, h, _, _ in blocks]
    axes = [(lib[ah], lib[av]) for *_, ah, av in blocks]
    gx_ref, gth_ref = BG.backward(xb, axes, gb, aset)
    got = gx.cpu().numpy()
    for k, (bx, y, w, h, _, _) in enumerate(blocks):
        err = np.abs(got[y:y + h, bx:bx + w] - gx_ref[k]).max()
        assert err <= 1e-5 * np.abs(gx_ref[k]).max(), f"dL/dX of block {k}"
    g = gth.cpu().numpy()
    assert np.abs(g - gth_ref).max() <= 1e-4 * np.abs(gth_ref).max(), f"angle gradient, max err {np.abs(g - gth_ref).max()}"


@pytest.mark.parametrize("aset", CASES[:2] + CASES[4:6], ids=[_ids(c) for c in CASES[:2] + CASES[4:6]])
def test_angle_sets_transform_like_their_matrices(env, aset):
    """A set registered by its angles transforms (fp32 and fixed point) as
    the oracle's matrix of those angles (integer version rounded half away
    from zero at scale 2^10)."""
    ctx, ids, params = env
    _register(ctx, aset, params, ids)
    n = aset.n
    m = aset.matrix()
    mi = OA.round_half_away(m * 1024.0)
    if aset.kind == "band":
        oax = Axis(base="S3", adj="band", a_int=mi, a_f=m)
    else:
        oax = Axis(base="C2", adj="post", q_int=mi, q_f=m)
    x = (np.random.Generator(np.random.PCG64(72)).standard_normal((9, n, n)) * 60).round().astype(np.int16)
    y = ctx.fwd(torch.from_numpy(x).cuda(), 200, 200).cpu().numpy()
    assert (y == F.fwd2d(x, oax, oax)).all()
    yf = ctx.fwd(torch.from_numpy(x.astype(np.float32)).cuda(), 200, 200).cpu().numpy()
    from oracle import fp as P
    ref = P.fwd2d(x.astype(np.float64), oax, oax)
    assert np.abs(yf - ref).max() <= 1e-5 * np.abs(ref).max()


def test_backward_errors(env):
    ctx, ids, _ = env
    x = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    dev = ctx.blocks_to_device(np.zeros(0, ta.BLOCK_DTYPE))
    with pytest.raises(ta.TadjError) as e:
        ctx.transform_bwd(dev, x, x, torch.zeros_like(x), torch.zeros(4, device="cuda"), ids["band_S3_S7_N16_K4"])
    assert e.value.code == ta.TA_ENOPARAMS          # a set registered as matrices has no angles
