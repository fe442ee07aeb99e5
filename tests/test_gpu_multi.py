"""GPU parity of the encoder evaluation of the five separable transforms
(ta_fwd_multi): each of the five outputs must equal, bit for bit, the
oracle's fixed-point forward with the corresponding axes, and the library's
own packed forward with those axes."""

import numpy as np
import pytest

import synth
from oracle import fixed as F
from tests.libcases import oracle_axis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2505_23618_amd as ta  # noqa: E402

# (N, B, parameter set of the DST-7 sub-block design)
SIZES = [(32, 8, "post_C2_S7_N32_B8"), (64, 16, "post_C2_S7_N64_B16")]
# (vertical, horizontal) per output; "C2" plain DCT-2, "S7" DCT-2 + Q, "C8" DCT-2 + S Q S
ORDER = [("C2", "C2"), ("S7", "S7"), ("S7", "C8"), ("C8", "S7"), ("C8", "C8")]


class Setup:
    def __init__(self, bd=8):
        self.bd = bd
        self.ctx = ta.Context(0, bit_depth=bd)
        self.ids = ta.load_params(self.ctx)
        self.params = ta.load_param_file()
        self.axes = {}
        nxt = 200
        for n, b, pname in SIZES:
            for name, adj, flip in (("C2", ta.ADJ_NONE, False), ("S7", ta.ADJ_POST, False), ("C8", ta.ADJ_POST, True)):
                self.ctx.axis(nxt, ta.DCT2, adj, flip, self.ids[pname] if adj else 0)
                self.axes[(n, name)] = (nxt, oracle_axis(self.params, ta.DCT2, adj, flip, pname if adj else None))
                nxt += 1


@pytest.fixture(scope="module")
def st():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return Setup()


def _check_all(st, n, pname, x):
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    got = st.ctx.fwd_multi(xd, st.ids[pname]).cpu().numpy()
    assert got.shape == (5,) + x.shape
    for k, (v, h) in enumerate(ORDER):
        ah, oh = st.axes[(n, h)]
        av, ov = st.axes[(n, v)]
        ref = F.fwd2d(x, oh, ov, bd=st.bd)
        mism = np.argwhere(got[k] != ref)
        assert mism.size == 0, f"output {k} ({v}, {h}): {len(mism)} mismatches, first {mism[:3].tolist()}"
        lib = st.ctx.fwd(xd, ah, av).cpu().numpy()
        assert (lib == got[k]).all(), f"output {k} differs from the packed forward"


@pytest.mark.parametrize("n,b,pname", SIZES)
def test_five_transforms_bit_exact_ar1(st, n, b, pname):
    nb = 3 * (256 // n) + 5                       # ragged last tile
    print(f"case multi {n} B={b} nb={nb}", flush=True)
    x = synth.ar1_blocks(nb, n, n, 0.95, 16.0, seed=61)
    _check_all(st, n, pname, x)


@pytest.mark.parametrize("kind", ["extreme16", "full16", "checker", "zeros"])
@pytest.mark.parametrize("n,b,pname", SIZES)
def test_five_transforms_adversarial(st, n, b, pname, kind):
    print(f"case multi {n} {kind}", flush=True)
    x = synth.adversarial_blocks(n, n, kind, seed=8, n=2 * (256 // n) + 1)
    _check_all(st, n, pname, x)


@pytest.mark.parametrize("bd", [6, 10, 12])
def test_five_transforms_at_bit_depth(bd):
    """The row and column shifts follow bd; residuals of that bit depth and
    full-range int16 values."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = Setup(bd)
    try:
        rng = np.random.Generator(np.random.PCG64(3000 + bd))
        lim = (1 << bd) - 1
        for n, b, pname in SIZES:
            nb = 2 * (256 // n) + 3
            print(f"case multi {n} B={b} bd {bd}", flush=True)
            for x in (rng.integers(-lim, lim + 1, size=(nb, n, n)), rng.integers(-32768, 32768, size=(nb, n, n))):
                _check_all(s, n, pname, x.astype(np.int16))
    finally:
        s.ctx.close()


def test_single_block_and_empty(st):
    x = synth.ar1_blocks(1, 32, 32, 0.95, 16.0, seed=4)
    _check_all(st, 32, "post_C2_S7_N32_B8", x)
    e = torch.zeros((0, 32, 32), dtype=torch.int16, device="cuda")
    assert st.ctx.fwd_multi(e, st.ids["post_C2_S7_N32_B8"]).shape == (5, 0, 32, 32)


def test_full_workload_sampled(st):
    """The benchmark's 262,144-block 32x32 workload in one launch; sampled
    blocks checked against the oracle."""
    x = synth.workload_blocks("cfg2_32x32")
    xd = torch.from_numpy(x).cuda()
    got = st.ctx.fwd_multi(xd, st.ids["post_C2_S7_N32_B8"])
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(12))
    idx = np.unique(np.concatenate([rng.integers(0, x.shape[0], 64), [0, x.shape[0] - 1]]))
    sub = got[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    for k, (v, h) in enumerate(ORDER):
        ref = F.fwd2d(x[idx], st.axes[(32, h)][1], st.axes[(32, v)][1])
        assert (sub[k] == ref).all(), f"output {k}"


def test_errors(st):
    x = torch.zeros((4, 32, 32), dtype=torch.int16, device="cuda")
    with pytest.raises(ta.TadjError) as e:
        st.ctx.fwd_multi(x, st.ids["band_S3_S7_N32_K4"])           # not a sub-block set
    assert e.value.code == ta.TA_ENOPARAMS
    with pytest.raises(ta.TadjError) as e:
        st.ctx.fwd_multi(x, st.ids["post_C2_S7_N64_B16"])          # set for another size
    assert e.value.code == ta.TA_EINVAL
    with pytest.raises(ta.TadjError) as e:
        st.ctx.fwd_multi(x, st.ids["post_C2_S7_N32_B16"])          # B = 16 at N = 32 not built
    assert e.value.code == ta.TA_EUNSUPPORTED
