"""GPU parity at other bit depths than 8: the fixed-point shifts depend on
bd (forward rows log2 W + bd + m - 15, inverse rows m + 14 - bd), and the
packed kernels take a different code path for the inverse rows when that
shift is not 14.  Bit-exact against the oracle run with the same bd."""

import numpy as np
import pytest

from oracle import fixed as F
from tests.libcases import CASES, Registered

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BITDEPTHS = [6, 7, 10, 12]
NAMES = ["cfg2_dst7_k4", "cfg2_dct8_k4", "dct2_32", "cfg1_dct2_band_16", "cfg3_post16_64", "dst3_dct3_8",
         "dst7_band_4", "dct2_dst7band_8x32"]


@pytest.fixture(scope="module", params=BITDEPTHS)
def reg(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return request.param, Registered(0, bit_depth=request.param)


@pytest.mark.parametrize("name", NAMES)
def test_fwd_inv_bit_exact_at_bit_depth(reg, name):
    bd, r = reg
    w, h = CASES[name][:2]
    ah, av = r.axes[name]
    oh, ov = r.oracle_axes(name)
    nb = 2 * (256 // max(w, h)) + 3
    print(f"bd {bd} case {name} {w}x{h} nb={nb}", flush=True)
    rng = np.random.Generator(np.random.PCG64(1000 + bd))
    lim = (1 << bd) - 1
    sets = [rng.integers(-lim, lim + 1, size=(nb, h, w)).astype(np.int16),
            rng.integers(-32768, 32768, size=(nb, h, w)).astype(np.int16)]
    for x in sets:
        xd = torch.from_numpy(x).cuda()
        y = r.ctx.fwd(xd, ah, av)
        assert (y.cpu().numpy() == F.fwd2d(x, oh, ov, bd=bd)).all(), "forward"
        z = r.ctx.inv(xd, ah, av)
        assert (z.cpu().numpy() == F.inv2d(x, oh, ov, bd=bd)).all(), "inverse of the input"
        z2 = r.ctx.inv(y, ah, av)
        assert (z2.cpu().numpy() == F.inv2d(y.cpu().numpy(), oh, ov, bd=bd)).all(), "inverse of the forward"


# cases with a matrix-core (int8 MFMA) kernel: forward for all, inverse for
# the first two
MFMA_CASES = ["direct_dst7_32", "dct2_32", "cfg2_dst7_k4"]


@pytest.mark.parametrize("name", MFMA_CASES)
def test_matrix_cores_at_bit_depth(reg, name):
    """The matrix-core kernels take the same bd-dependent shifts."""
    bd, r = reg
    w, h = CASES[name][:2]
    ah, av = r.axes[name]
    oh, ov = r.oracle_axes(name)
    nb = 2 * (256 // max(w, h)) + 3
    print(f"bd {bd} matrix-core case {name}", flush=True)
    rng = np.random.Generator(np.random.PCG64(1100 + bd))
    lim = (1 << bd) - 1
    sets = [rng.integers(-lim, lim + 1, size=(nb, h, w)).astype(np.int16),
            rng.integers(-32768, 32768, size=(nb, h, w)).astype(np.int16)]
    r.ctx.set_impl(1)
    try:
        for x in sets:
            xd = torch.from_numpy(x).cuda()
            assert (r.ctx.fwd(xd, ah, av).cpu().numpy() == F.fwd2d(x, oh, ov, bd=bd)).all(), "forward"
            if name != "cfg2_dst7_k4":
                assert (r.ctx.inv(xd, ah, av).cpu().numpy() == F.inv2d(x, oh, ov, bd=bd)).all(), "inverse"
    finally:
        r.ctx.set_impl(0)
