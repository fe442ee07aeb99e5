"""GPU parity of the fixed-point path: bit-exact against the CPU oracle.

Every case runs through the C ABI (via the ctypes binding) on seeded inputs
at sizes the oracle finishes quickly, with a ragged last tile, plus the
adversarial value sets (extreme residuals, full-range int16 coefficients);
the full 262,144-block 32x32 workload is checked on sampled blocks.
"""

import numpy as np
import pytest

import synth
from oracle import adjust as OA
from oracle import fixed as F
from oracle.fixed import Axis
from tests.libcases import CASES, Registered

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402


@pytest.fixture(scope="module")
def reg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Registered(0)


# forward cases that also have a matrix-core (int8 MFMA) kernel
MFMA_FWD = ["cfg2_dst7_k4", "cfg2_dct8_k4", "cfg2_dst7_k6", "direct_dst7_32", "dct2_32", "direct_dct8_32"]
# inverse cases with a matrix-core kernel
MFMA_INV = ["direct_dst7_32", "dct2_32", "direct_dct8_32"]


@pytest.fixture
def impl(reg, request):
    reg.ctx.set_impl(request.param)
    yield request.param
    reg.ctx.set_impl(0)


def _ragged(w, h):
    nb_per_wg = 256 // max(w, h)
    return 3 * nb_per_wg + 5


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run_case(reg, name, x, inverse):
    ah, av = reg.axes[name]
    oh, ov = reg.oracle_axes(name)
    xd = _gpu(x)
    if not inverse:
        got = reg.ctx.fwd(xd, ah, av).cpu().numpy()
        ref = F.fwd2d(x, oh, ov)
    else:
        got = reg.ctx.inv(xd, ah, av).cpu().numpy()
        ref = F.inv2d(x, oh, ov)
    torch.cuda.synchronize()
    return got, ref


@pytest.mark.parametrize("name", list(CASES))
def test_forward_inverse_bit_exact_ar1(reg, name):
    w, h = CASES[name][:2]
    nb = _ragged(w, h)
    print(f"case {name} {w}x{h} nb={nb}", flush=True)
    x = synth.ar1_blocks(nb, h, w, 0.95, 16.0, seed=101)
    got, ref = _run_case(reg, name, x, inverse=False)
    assert got.dtype == np.int16
    mism = np.argwhere(got != ref)
    assert mism.size == 0, f"{len(mism)} mismatches, first at {mism[:3].tolist()}"
    got2, ref2 = _run_case(reg, name, got, inverse=True)
    assert (got2 == ref2).all()


@pytest.mark.parametrize("kind", ["zeros", "pos", "neg", "checker", "uniform_res", "full16", "extreme16"])
@pytest.mark.parametrize("name", ["cfg2_dst7_k4", "cfg2_dct8_k4", "cfg3_post16_64", "dct2_32",
                                  "dst7_band_4", "dst2_dct8_16x8", "direct_dst7_32"])
def test_adversarial_values(reg, name, kind):
    w, h = CASES[name][:2]
    print(f"case {name} {kind}", flush=True)
    x = synth.adversarial_blocks(h, w, kind, seed=5, n=_ragged(w, h))
    for inverse in (False, True):
        got, ref = _run_case(reg, name, x, inverse)
        assert (got == ref).all(), f"inverse={inverse}"


@pytest.mark.parametrize("outside", [False, True, "deep"], ids=["edge_inside", "one_outside", "deep_edge"])
@pytest.mark.parametrize("name", ["cfg2_dst7_k4", "cfg2_dct8_k4", "dct2_32", "post8_32", "cfg1_dct2_band_16",
                                  "cfg3_post16_64"])
def test_dct2_butterfly_range_edge(reg, name, outside):
    """The DCT-2 butterfly (forward DCT-2 cores, inverse DST-3/DCT-3 cores)
    takes its packed first level only when every input of the wave lies in
    [-2^14, 2^14).  Inputs drawn from the edges of that range exercise the
    packed level at its limits; one value just outside it in a single block
    sends that block's waves down the int32 path while neighbouring waves
    stay packed.  Both must give the oracle's result.  "deep": values near
    +-2^13, so the first level stays packed while the sums feeding the next
    packed level straddle +-2^14 (the deeper levels' own check)."""
    w, h = CASES[name][:2]
    nb = _ragged(w, h)
    rng = np.random.Generator(np.random.PCG64(77))
    if outside == "deep":
        x = rng.choice(np.array([-8193, -8192, -1, 0, 8191, 8192], np.int16), size=(nb, h, w))
    else:
        x = rng.choice(np.array([-16384, -16383, -1, 0, 16382, 16383], np.int16), size=(nb, h, w))
    if outside is True:
        x[nb // 2, h // 3, w // 2] = 16384
        x[nb - 1, h - 1, 0] = -16385
    print(f"case {name} outside={outside}", flush=True)
    for inverse in (False, True):
        got, ref = _run_case(reg, name, x, inverse)
        assert (got == ref).all(), f"inverse={inverse}"


def test_empty_batch_is_noop(reg):
    ah, av = reg.axes["cfg2_dst7_k4"]
    x = torch.zeros((0, 32, 32), dtype=torch.int16, device="cuda")
    y = reg.ctx.fwd(x, ah, av)
    assert y.shape == (0, 32, 32)


def test_single_block(reg):
    x = synth.ar1_blocks(1, 32, 32, 0.95, 16.0, seed=9)
    got, ref = _run_case(reg, "cfg2_dst7_k4", x, inverse=False)
    assert (got == ref).all()


def test_deterministic_reruns(reg):
    ah, av = reg.axes["cfg2_dst7_k4"]
    x = _gpu(synth.ar1_blocks(1000, 32, 32, 0.95, 16.0, seed=3))
    a = reg.ctx.fwd(x, ah, av)
    b = reg.ctx.fwd(x, ah, av)
    c = reg.ctx.inv(a, ah, av)
    d = reg.ctx.inv(b, ah, av)
    assert torch.equal(a, b) and torch.equal(c, d)


def test_errors(reg):
    ah, av = reg.axes["cfg2_dst7_k4"]
    x = torch.zeros((4, 32, 32), dtype=torch.int16, device="cuda")
    # parameter set of the wrong size for a 16x16 block
    with pytest.raises(ta.TadjError) as e:
        reg.ctx.fwd(torch.zeros((4, 16, 16), dtype=torch.int16, device="cuda"), ah, av)
    assert e.value.code == ta.TA_EUNSUPPORTED
    # unregistered axis
    with pytest.raises(ta.TadjError) as e:
        reg.ctx.fwd(x, 250, 250)
    assert e.value.code == ta.TA_ENOPARAMS
    # aliasing in/out
    with pytest.raises(ta.TadjError) as e:
        reg.ctx.fwd(x, ah, av, out=x)
    assert e.value.code == ta.TA_EINVAL
    # a combination without a specialised kernel runs on the general kernel
    s7 = reg.axes["direct_dst7_32"][0]
    xs = synth.ar1_blocks(4, 32, 32, 0.95, 16.0, seed=12)
    oh, ov = reg.oracle_axes("cfg2_dst7_k4")[0], reg.oracle_axes("direct_dst7_32")[1]
    assert (reg.ctx.fwd(_gpu(xs), ah, s7).cpu().numpy() == F.fwd2d(xs, oh, ov)).all()
    # ... but not when the matrix-core kernels are required
    reg.ctx.set_impl(1)
    try:
        with pytest.raises(ta.TadjError) as e:
            reg.ctx.fwd(x, ah, s7)
        assert e.value.code == ta.TA_EUNSUPPORTED
    finally:
        reg.ctx.set_impl(0)


@pytest.mark.parametrize("name,wl", [("cfg2_dst7_k4", "cfg2_32x32"), ("cfg3_post16_64", "cfg3_64x64")])
def test_full_size_sampled(reg, name, wl):
    """Full workload in the benchmark's launch configuration; the oracle
    checks a random sample of blocks of the forward and inverse outputs."""
    x = synth.workload_blocks(wl)
    print(f"full {name}: {x.shape}", flush=True)
    ah, av = reg.axes[name]
    xd = _gpu(x)
    y = reg.ctx.fwd(xd, ah, av)
    z = reg.ctx.inv(y, ah, av)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(77))
    idx = np.sort(rng.choice(x.shape[0], size=48, replace=False))
    idx = np.concatenate([idx, [0, x.shape[0] - 1]])
    oh, ov = reg.oracle_axes(name)
    ys = y[torch.from_numpy(idx).cuda()].cpu().numpy()
    zs = z[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert (ys == F.fwd2d(x[idx], oh, ov)).all()
    assert (zs == F.inv2d(ys, oh, ov)).all()
    del xd, y, z


@pytest.mark.parametrize("impl", [1, 2], indirect=True, ids=["matrix", "valu"])
@pytest.mark.parametrize("name", MFMA_FWD)
def test_matrix_core_forward_bit_exact(reg, name, impl):
    """The int8-MFMA forward kernels and the VALU butterfly kernels both match
    the oracle bit for bit (AR(1) data, ragged count, adversarial sets)."""
    w, h = CASES[name][:2]
    ah, av = reg.axes[name]
    oh, ov = reg.oracle_axes(name)
    print(f"impl {impl} case {name}", flush=True)
    sets = [synth.ar1_blocks(61, h, w, 0.95, 16.0, seed=202)]
    sets += [synth.adversarial_blocks(h, w, k, seed=6, n=7) for k in
             ("pos", "neg", "checker", "uniform_res", "full16", "extreme16")]
    for x in sets:
        got = reg.ctx.fwd(_gpu(x), ah, av).cpu().numpy()
        ref = F.fwd2d(x, oh, ov)
        mism = np.argwhere(got != ref)
        assert mism.size == 0, f"{len(mism)} mismatches, first {mism[:3].tolist()}"


@pytest.mark.parametrize("impl", [1], indirect=True, ids=["matrix"])
def test_matrix_core_full_size_sampled(reg, impl):
    x = synth.workload_blocks("cfg2_32x32")
    ah, av = reg.axes["cfg2_dst7_k4"]
    y = reg.ctx.fwd(_gpu(x), ah, av)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(78))
    idx = np.concatenate([np.sort(rng.choice(x.shape[0], size=48, replace=False)), [0, x.shape[0] - 1]])
    oh, ov = reg.oracle_axes("cfg2_dst7_k4")
    assert (y[torch.from_numpy(idx).cuda()].cpu().numpy() == F.fwd2d(x[idx], oh, ov)).all()


@pytest.mark.parametrize("impl", [1, 2], indirect=True, ids=["matrix", "valu"])
@pytest.mark.parametrize("name", MFMA_INV)
def test_matrix_core_inverse_bit_exact(reg, name, impl):
    w, h = CASES[name][:2]
    ah, av = reg.axes[name]
    oh, ov = reg.oracle_axes(name)
    print(f"impl {impl} inverse case {name}", flush=True)
    sets = [F.fwd2d(synth.ar1_blocks(61, h, w, 0.95, 16.0, seed=203), oh, ov).astype(np.int16)]
    sets += [synth.adversarial_blocks(h, w, k, seed=7, n=7) for k in
             ("pos", "neg", "checker", "uniform_res", "full16", "extreme16")]
    for x in sets:
        got = reg.ctx.inv(_gpu(x), ah, av).cpu().numpy()
        ref = F.inv2d(x, oh, ov)
        mism = np.argwhere(got != ref)
        assert mism.size == 0, f"{len(mism)} mismatches, first {mism[:3].tolist()}"


@pytest.mark.parametrize("impl", [1], indirect=True, ids=["matrix"])
@pytest.mark.parametrize("name", MFMA_INV)
def test_matrix_core_inverse_full_size_sampled(reg, name, impl):
    """The persistent matrix-core inverse at the benchmark's size (262,144
    blocks, every wave walks many blocks with its next block prefetched),
    on the coefficients of the AR(1) workload and on full-range int16
    coefficients; the oracle checks sampled blocks, including the first and
    the last."""
    x = synth.workload_blocks("cfg2_32x32")
    ah, av = reg.axes[name]
    oh, ov = reg.oracle_axes(name)
    print(f"full-size matrix-core inverse {name}", flush=True)
    rng = np.random.Generator(np.random.PCG64(79))
    idx = np.concatenate([np.sort(rng.choice(x.shape[0], size=48, replace=False)), [0, 1, x.shape[0] - 1]])
    ti = torch.from_numpy(idx).cuda()
    y = reg.ctx.fwd(_gpu(x), ah, av)
    z = reg.ctx.inv(y, ah, av)
    torch.cuda.synchronize()
    ys = y[ti].cpu().numpy()
    assert (ys == F.fwd2d(x[idx], oh, ov)).all()
    assert (z[ti].cpu().numpy() == F.inv2d(ys, oh, ov)).all()
    del y, z
    c = torch.randint(-32768, 32768, x.shape, dtype=torch.int16, generator=torch.Generator().manual_seed(80))
    z = reg.ctx.inv(c.cuda(), ah, av)
    torch.cuda.synchronize()
    assert (z[ti].cpu().numpy() == F.inv2d(c.numpy()[idx], oh, ov)).all()


def _random_band(n, taps, seed):
    """A K-tap band from random Givens angles (a valid parameter set that
    differs from the frozen one), integer version at scale 2^10."""
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.uniform(-0.6, 0.6, OA.n_angles(n, taps // 2))
    a_f = OA.band_matrix(n, taps // 2, theta)
    return OA.round_half_away(a_f * 1024.0), a_f


@pytest.mark.parametrize("impl", [1, 2], indirect=True, ids=["matrix", "valu"])
@pytest.mark.parametrize("taps", [4, 6])
@pytest.mark.parametrize("flip", [False, True], ids=["dst7", "dct8"])
def test_two_band_sets(reg, taps, flip, impl):
    """Rows and columns with different band parameter sets of the same size
    and kind: the matrix-core forward then keeps one set of tap registers per
    axis.  Checked in both directions on AR(1) and full-range inputs, with
    the frozen set on one axis and a random one on the other, both ways.
    (The DCT-3 + 6-tap pair has no specialised kernel and runs on the
    general kernel.)"""
    ctx = reg.ctx
    a_int, a_f = _random_band(32, taps, seed=90 + taps)
    pid = 200 + taps
    ctx.set_band(pid, a_int, a_f, taps)
    frozen = reg.params[f"band_S3_S7_N32_K{taps}"]
    ax_r = ctx.axis(240 + taps + int(flip), ta.DST3, ta.ADJ_BAND, flip, pid)
    ax_f = ctx.axis(230 + taps + int(flip), ta.DST3, ta.ADJ_BAND, flip, reg.ids[f"band_S3_S7_N32_K{taps}"])
    o_r = Axis(base="S3", adj="band", flip=flip, a_int=a_int, a_f=a_f)
    o_f = Axis(base="S3", adj="band", flip=flip, a_int=np.asarray(frozen["a_int"], np.int64),
               a_f=np.asarray(frozen["a_f64"]))
    sets = [synth.ar1_blocks(61, 32, 32, 0.95, 16.0, seed=204),
            synth.adversarial_blocks(32, 32, "full16", seed=8, n=7),
            synth.adversarial_blocks(32, 32, "extreme16", seed=8, n=7)]
    print(f"impl {impl} two band sets K={taps} flip={flip}", flush=True)
    if impl == 1 and flip and taps == 6:
        # no matrix-core kernel for the DCT-3 + 6-tap pair: forcing the matrix
        # cores is refused, and the default selection runs the general kernel
        with pytest.raises(ta.TadjError) as e:
            ctx.fwd(_gpu(sets[0]), ax_f, ax_r)
        assert e.value.code == ta.TA_EUNSUPPORTED
        impl = 0
    for (ah, av, oh, ov) in ((ax_f, ax_r, o_f, o_r), (ax_r, ax_f, o_r, o_f)):
        for x in sets:
            ctx.set_impl(impl)
            y = ctx.fwd(_gpu(x), ah, av).cpu().numpy()
            yr = F.fwd2d(x, oh, ov).astype(np.int16)
            assert (y == yr).all(), "forward"
            ctx.set_impl(2)          # the band inverse runs on VALU only
            z = ctx.inv(_gpu(yr), ah, av).cpu().numpy()
            assert (z == F.inv2d(yr, oh, ov)).all(), "inverse"


@pytest.mark.parametrize("impl", [1], indirect=True, ids=["matrix"])
def test_two_band_sets_full_size_sampled(reg, impl):
    """The persistent matrix-core forward with two band sets at the
    benchmark's size, on sampled blocks."""
    ctx = reg.ctx
    a_int, a_f = _random_band(32, 4, seed=94)
    ctx.set_band(210, a_int, a_f, 4)
    ah = ctx.axis(250, ta.DST3, ta.ADJ_BAND, False, reg.ids["band_S3_S7_N32_K4"])
    av = ctx.axis(251, ta.DST3, ta.ADJ_BAND, False, 210)
    frozen = reg.params["band_S3_S7_N32_K4"]
    oh = Axis(base="S3", adj="band", a_int=np.asarray(frozen["a_int"], np.int64), a_f=np.asarray(frozen["a_f64"]))
    ov = Axis(base="S3", adj="band", a_int=a_int, a_f=a_f)
    x = synth.workload_blocks("cfg2_32x32")
    y = ctx.fwd(_gpu(x), ah, av)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(81))
    idx = np.concatenate([np.sort(rng.choice(x.shape[0], size=48, replace=False)), [0, x.shape[0] - 1]])
    assert (y[torch.from_numpy(idx).cuda()].cpu().numpy() == F.fwd2d(x[idx], oh, ov)).all()


def test_binding_rejects_bad_outputs(reg):
    """The C ABI receives only pointers, so the binding checks a caller's
    output tensor before the call: shape, dtype, contiguity, and block sides
    that are powers of two in 4..64."""
    ah, av = reg.axes["cfg2_dst7_k4"]
    x = torch.zeros((4, 32, 32), dtype=torch.int16, device="cuda")
    for bad in (torch.empty((3, 32, 32), dtype=torch.int16, device="cuda"),
                torch.empty((4, 32, 32), dtype=torch.float32, device="cuda"),
                torch.empty((4, 32, 64), dtype=torch.int16, device="cuda")[:, :, ::2]):
        with pytest.raises(ValueError):
            reg.ctx.fwd(x, ah, av, out=bad)
    with pytest.raises(ValueError):
        reg.ctx.fwd(torch.zeros((4, 48, 48), dtype=torch.int16, device="cuda"), ah, av)
    pid = reg.ids["post_C2_S7_N32_B8"]
    with pytest.raises(ValueError):
        reg.ctx.fwd_multi(x, pid, out=torch.empty((4, 4, 32, 32), dtype=torch.int16, device="cuda"))
